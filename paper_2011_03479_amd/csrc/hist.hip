// Slope optimisation (Sec. III-F): histograms of the pair distances, separately for edges and
// non-edges, and the bisection of d DL / d sigma = 0 on them.
//
// Histogram layout: nbins bins uniform in the squared distance on [0, r2_max).  A pair's bin
// is the integer part of min(r2 * inv_w, nbins - 1) with inv_w = nbins / r2_max rounded to
// single precision, from the single-precision squared distance summed over the coordinates
// in order with fused multiply-adds (the sweeps' sqdist) - a decision any implementation
// that rounds the same way reproduces exactly.  A bin stands for the distance
// sqrt((b + 1/2) r2_max / nbins).
//
// Kernels:
//   k_hist_small<D>  d <= 16: four waves per workgroup, each wave takes whole 64 x 64 tiles
//                    (rows in registers, columns rotating through the DPP schedule), counts
//                    in a 32-bit LDS histogram (one LDS atomic per pair); the workgroup adds
//                    its histogram into its own 64-bit slot of a partial buffer (no global
//                    atomics) after at most 2^31 pairs and at the end, so no LDS bin can wrap
//                    whatever n is.
//   k_hist_wide<D>   d > 16: the workgroup stages a tile's rows and columns in LDS, its four
//                    waves take 16 steps each, coordinates summed in order.
//   k_hist_edges     one lane per CSR entry with i < j (the same squared distance), one
//                    64-bit atomic per edge.
//   k_hist_reduce    all-pair counts = sum of the workgroups' partial histograms (fixed order).
// Non-edge counts are the difference of the two (exact integers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "tiles.h"

namespace gempe {
namespace {

constexpr int kHistThreads = 256;
constexpr int kHistMaxGrid = 512;
// Rounds of four 64 x 64 tiles a workgroup counts in its 32-bit LDS bins before it adds them
// into its 64-bit partial histogram: at most 4 * 4096 pairs per round, so no bin can reach
// 2^32 between flushes.
constexpr long long kHistFlushRounds = 1ll << 17;
static_assert(kHistFlushRounds * 4 * 64 * 64 < (1ll << 32), "an LDS bin could wrap between flushes");

// Adds the workgroup's LDS bins into its 64-bit slot (written on the first flush) and clears
// them.  Called by every thread of the workgroup.
__device__ __forceinline__ void flush_bins(unsigned *hb, unsigned long long *mine, int nbins, bool &first) {
    __syncthreads();
    for (int q = threadIdx.x; q < nbins; q += kHistThreads) {
        const unsigned long long v = hb[q];
        mine[q] = first ? v : mine[q] + v;
        hb[q] = 0u;
    }
    first = false;
    __syncthreads();
}

__device__ __forceinline__ int bin_of(float r2, float inv_w, float top) {
    return (int)fminf(r2 * inv_w, top);
}

template <int D>
__global__ __launch_bounds__(kHistThreads) void k_hist_small(const float *__restrict__ X, int n, int d, int nt,
                                                             long long tiles, int nbins, float inv_w,
                                                             unsigned long long *__restrict__ partial) {
    extern __shared__ unsigned hb[];
    for (int q = threadIdx.x; q < nbins; q += kHistThreads) hb[q] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int dir = rot_dir(lane);
    const float top = (float)(nbins - 1);
    unsigned long long *mine = partial + (size_t)blockIdx.x * nbins;
    bool first = true;
    long long rounds = 0;
    // every wave runs the same number of rounds (a wave past the last tile idles), so the
    // flushes below are reached by the whole workgroup
    for (long long t0 = (long long)blockIdx.x * 4; t0 < tiles; t0 += (long long)gridDim.x * 4) {
        if (++rounds > kHistFlushRounds) {
            flush_bins(hb, mine, nbins, first);
            rounds = 1;
        }
        const long long t = t0 + wave;
        if (t >= tiles) continue;
        int I, J;
        tile_of(t, nt, I, J);
        const int i = I * 64 + lane;
        const int jc = J * 64 + lane;
        float xi[D], xc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xi[k] = (i < n && k < d) ? X[(size_t)i * d + k] : 0.0f;
            xc[k] = (jc < n && k < d) ? X[(size_t)jc * d + k] : 0.0f;
        }
        for (int s = 0; s < 64; ++s) {
            const int j = J * 64 + ((lane + dir * s) & 63);
            float diff[D];
            const float r2 = sqdist<D>(xi, xc, diff);
            if (i < j && j < n) atomicAdd(&hb[bin_of(r2, inv_w, top)], 1u);
#pragma unroll
            for (int k = 0; k < D; ++k) xc[k] = rot1(xc[k]);
        }
    }
    flush_bins(hb, mine, nbins, first);
}

template <int D>
__global__ __launch_bounds__(kHistThreads) void k_hist_wide(const float *__restrict__ X, int n, int d, int nt,
                                                            long long tiles, int nbins, float inv_w,
                                                            unsigned long long *__restrict__ partial) {
    extern __shared__ unsigned hb[];
    constexpr int S = D + 1;  // padded stride: lane-private rows hit distinct banks
    float *xr = reinterpret_cast<float *>(hb + nbins);  // rows [64][S]
    float *xc = xr + 64 * S;                            // columns [64][S]
    for (int q = threadIdx.x; q < nbins; q += kHistThreads) hb[q] = 0u;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const float top = (float)(nbins - 1);
    unsigned long long *mine = partial + (size_t)blockIdx.x * nbins;
    bool first = true;
    long long count = 0;
    // the workgroup stages one 64 x 64 tile; its four waves take 16 of the 64 steps each
    for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
        if (++count > 4 * kHistFlushRounds) {
            __syncthreads();  // the previous tile's counts are all in
            flush_bins(hb, mine, nbins, first);
            count = 1;
        }
        int I, J;
        tile_of(t, nt, I, J);
        __syncthreads();  // the previous tile is consumed
        for (int q = threadIdx.x; q < 64 * S; q += kHistThreads) {
            const int c = q / S, k = q - c * S;
            const int ri = I * 64 + c, cj = J * 64 + c;
            xr[q] = (ri < n && k < d) ? X[(size_t)ri * d + k] : 0.0f;
            xc[q] = (cj < n && k < d) ? X[(size_t)cj * d + k] : 0.0f;
        }
        __syncthreads();
        const int i = I * 64 + lane;
        for (int s = wave * 16; s < wave * 16 + 16; ++s) {
            const int c = (lane + s) & 63;
            const int j = J * 64 + c;
            const float *a = xr + lane * S;
            const float *b = xc + c * S;
            float r2 = 0.0f;
            for (int k = 0; k < D; ++k) {
                const float df = a[k] - b[k];
                r2 = __builtin_fmaf(df, df, r2);
            }
            if (i < j && j < n) atomicAdd(&hb[bin_of(r2, inv_w, top)], 1u);
        }
    }
    flush_bins(hb, mine, nbins, first);
}

__global__ void k_hist_edges(const float *__restrict__ X, int d, const int32_t *__restrict__ coo_row,
                             const int32_t *__restrict__ col, long long nnz, int nbins, float inv_w,
                             unsigned long long *__restrict__ hist_edge) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int i = coo_row[e], j = col[e];
    if (i >= j) return;
    const float *xi = X + (size_t)i * d;
    const float *xj = X + (size_t)j * d;
    float r2 = 0.0f;
    for (int k = 0; k < d; ++k) {
        const float df = xi[k] - xj[k];
        r2 = __builtin_fmaf(df, df, r2);
    }
    atomicAdd(&hist_edge[bin_of(r2, inv_w, (float)(nbins - 1))], 1ull);
}

__global__ void k_hist_reduce(const unsigned long long *__restrict__ partial, int parts, int nbins,
                              unsigned long long *__restrict__ hist_all) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    unsigned long long acc = 0;
    for (int w = 0; w < parts; ++w) acc += partial[(size_t)w * nbins + b];
    hist_all[b] = acc;
}

__global__ void k_fill_zero_u64(unsigned long long *p, int count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = 0ull;
}

// Bounding box of the coordinates: per coordinate the minimum and maximum, as order-
// preserving integer codes of the floats (so integer atomics give float min / max).
__device__ __forceinline__ int float_order(float f) {
    const int b = __float_as_int(f);
    return b >= 0 ? b : (b ^ 0x7fffffff);
}

__global__ void k_box_init(int *box, int d) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < d) {
        box[k] = 0x7fffffff;          // min code
        box[d + k] = (int)0x80000000; // max code
    }
}

__global__ void k_box(const float *__restrict__ X, int n, int d, int *box) {
    // thread = (vertex block, coordinate): each thread scans 64 vertices of one coordinate
    const int k = blockIdx.y;
    const int i0 = (blockIdx.x * blockDim.x + threadIdx.x) * 64;
    int lo = 0x7fffffff, hi = (int)0x80000000;
    for (int i = i0; i < i0 + 64 && i < n; ++i) {
        const int c = float_order(X[(size_t)i * d + k]);
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int ol = __shfl_xor(lo, off, 64), oh = __shfl_xor(hi, off, 64);
        lo = ol < lo ? ol : lo;
        hi = oh > hi ? oh : hi;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&box[k], lo);
        atomicMax(&box[d + k], hi);
    }
}

int hist_padded_dim(int d) { return d <= 4 ? d : d <= 8 ? 8 : d <= 16 ? 16 : d <= 32 ? 32 : d <= 64 ? 64 : 128; }

struct HistPlan {
    int D, nt, grid;
    long long tiles;
    size_t lds;
};

HistPlan hist_plan(int n, int d, int nbins) {
    HistPlan h;
    h.D = hist_padded_dim(d);
    h.nt = (n + 63) / 64;
    h.tiles = (long long)h.nt * (h.nt + 1) / 2;
    const long long per_wg = h.D > 16 ? 1 : 4;  // tiles a workgroup takes at once
    h.grid = (int)std::max<long long>(1, std::min<long long>(kHistMaxGrid, (h.tiles + per_wg - 1) / per_wg));
    h.lds = sizeof(unsigned) * (size_t)nbins + (h.D > 16 ? sizeof(float) * 2 * 64 * (h.D + 1) : 0);
    return h;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <int D>
void launch_hist_small(const HistPlan &h, const float *X, int n, int d, int nbins, float inv_w,
                       unsigned long long *partial,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_hist_small<D>, dim3(h.grid), dim3(kHistThreads), h.lds, s, X, n, d, h.nt, h.tiles, nbins,
                       inv_w, partial);
}
template <int D>
void launch_hist_wide(const HistPlan &h, const float *X, int n, int d, int nbins, float inv_w,
                      unsigned long long *partial,
                      hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hist_wide<D>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL(k_hist_wide<D>, dim3(h.grid), dim3(kHistThreads), h.lds, s, X, n, d, h.nt, h.tiles, nbins,
                       inv_w, partial);
}

// ------------------------------------------------------------------------------------
// Host: phi(tau) / Phi(tau) in double precision, and the bisection on the histograms.
// ------------------------------------------------------------------------------------
double mills_inverse(double t) {
    if (t < -30.0) {
        // asymptotic normal tail (Abramowitz and Stegun 26.2.12): Phi(t) ~ phi(t) S / |t|
        const double q = 1.0 / (t * t);
        const double S = 1.0 + q * (-1.0 + q * (3.0 + q * (-15.0 + q * (105.0 + q * (-945.0)))));
        return -t / S;
    }
    const double phi = std::exp(-0.5 * t * t) * 0.39894228040143267794;
    const double Phi = 0.5 * std::erfc(-t * 0.70710678118654752440);
    return phi / Phi;
}

// d DL / d sigma up to the factor 1 / (sigma ln 2): sum over bins of count tau R(tau).
double slope_condition(double sigma, int nbins, double r2_max, const uint64_t *all, const uint64_t *edge,
                       double mu) {
    double F = 0.0;
    for (int b = 0; b < nbins; ++b) {
        if (!all[b]) continue;
        const double delta = std::sqrt((b + 0.5) * r2_max / nbins);
        const double tn = (delta - mu) / sigma;  // a non-edge; an edge has -tn
        const double ne = (double)(all[b] - edge[b]), e = (double)edge[b];
        if (ne > 0.0) F += ne * tn * mills_inverse(tn);
        if (e > 0.0) F += e * (-tn) * mills_inverse(-tn);
    }
    return F;
}

}  // namespace
}  // namespace gempe

using namespace gempe;

size_t gempe_hist_partial_bytes(int n, int d, int nbins) {
    const HistPlan h = hist_plan(n, d, nbins);
    return align256(sizeof(unsigned long long) * (size_t)h.grid * (size_t)nbins) + 256;
}

hipError_t gempe_launch_histogram(const gempe_graph_s *g, int d, const float *X, int nbins, float r2_max,
                                  unsigned long long *hist_all, unsigned long long *hist_edge, void *scratch,
                                  hipStream_t s) {
    const HistPlan h = hist_plan(g->n, d, nbins);
    const float inv_w = (float)((double)nbins / (double)r2_max);
    unsigned long long *partial = static_cast<unsigned long long *>(scratch);
    switch (h.D) {
        case 1: launch_hist_small<1>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 2: launch_hist_small<2>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 3: launch_hist_small<3>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 4: launch_hist_small<4>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 8: launch_hist_small<8>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 16: launch_hist_small<16>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 32: launch_hist_wide<32>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        case 64: launch_hist_wide<64>(h, X, g->n, d, nbins, inv_w, partial, s); break;
        default: launch_hist_wide<128>(h, X, g->n, d, nbins, inv_w, partial, s); break;
    }
    hipLaunchKernelGGL(k_hist_reduce, dim3((nbins + 255) / 256), dim3(256), 0, s, partial, h.grid, nbins, hist_all);
    hipLaunchKernelGGL(k_fill_zero_u64, dim3((nbins + 255) / 256), dim3(256), 0, s, hist_edge, nbins);
    if (g->nnz > 0)
        hipLaunchKernelGGL(k_hist_edges, dim3((unsigned)((g->nnz + 255) / 256)), dim3(256), 0, s, X, d, g->coo_row,
                           g->col_idx, (long long)g->nnz, nbins, inv_w, hist_edge);
    return hipGetLastError();
}

hipError_t gempe_launch_box(const gempe_graph_s *g, int d, const float *X, int *box, hipStream_t s) {
    hipLaunchKernelGGL(k_box_init, dim3((d + 127) / 128), dim3(128), 0, s, box, d);
    const int groups = (g->n + 63) / 64;  // 64 vertices per thread
    hipLaunchKernelGGL(k_box, dim3((groups + 255) / 256, d), dim3(256), 0, s, X, g->n, d, box);
    return hipGetLastError();
}

float gempe_box_code_to_float(int c) {
    const int b = c >= 0 ? c : (c ^ 0x7fffffff);
    float f;
    std::memcpy(&f, &b, sizeof(f));
    return f;
}

double gempe_bisect_sigma(int nbins, double r2_max, const uint64_t *all, const uint64_t *edge, double mu,
                          double lo, double hi, int iters) {
    if (slope_condition(lo, nbins, r2_max, all, edge, mu) >= 0.0) return lo;
    if (slope_condition(hi, nbins, r2_max, all, edge, mu) <= 0.0) return hi;
    for (int it = 0; it < iters; ++it) {
        const double s = std::sqrt(lo * hi);
        if (slope_condition(s, nbins, r2_max, all, edge, mu) < 0.0) lo = s; else hi = s;
    }
    return std::sqrt(lo * hi);
}
