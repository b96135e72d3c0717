// Negative-sampled weighted majorization (Sec. III-C, Fig. nonedges, Fig. algo): O(m) work
// per iteration instead of O(n^2).
//
// The pairs of one step: every edge (i, j), i < j, once, and for each of its ends a sampled
// non-edge - g for i and h for j - each drawn with its own 32-bit LCG (s <- 1103515245 s + 1,
// the generator of the paper), its state seeded from SplitMix64(seed + 2 e + side), e the
// CSR index of (i, j) with i < j and side 0 for i, 1 for j, so the draws do not depend on
// how lanes are scheduled.  A draw maps the low 23 bits of s to a float f in [1, 2) and
// takes floor(f n - n) in single precision (multiply, then subtract); it is rejected when it
// is the vertex itself, outside [0, n) or adjacent to it - adjacency is a probe of the exact
// edge hash, the per-sample use the hash was built for - and the LCG steps again, at most
// max_tries draws.  Each pair adds its gradient term c (x_a - x_b) and its parabola weight
// w = dl''/2 to both ends, and its dl to the loss; x <- x - g / (2 z) then applies Eq. 5
// over that multiset of pairs.
//
// Layout: one lane per DIRECTED CSR entry (r, c), lanes in CSR order.  The lane adds the
// edge's term for row r (the mirror entry (c, r) adds it for c; the edge's dl is counted by
// the entry with r < c) and draws the sample of r that belongs to this edge end: side 0 and
// e = its own index when r < c, else side 1 and e = the index of (c, r) in row c (binary
// search of the sorted row).  Both of r's terms are summed over the lanes of each row run
// before one atomic per run (a wave covers a few rows); only the sample's far end g takes a
// scattered atomic: about d + 1 per directed entry instead of 6 (d + 1) per edge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.h"
#include "pairfn.h"
#include "tiles.h"

namespace gempe {
namespace {

constexpr int kSampledBlock = 256;

__device__ __forceinline__ int draw_non_neighbour(int v, int n, unsigned state, int max_tries,
                                                  const unsigned long long *__restrict__ table,
                                                  unsigned long long cap) {
    const float nf = (float)n;
    for (int t = 0; t < max_tries; ++t) {
        state = 1103515245u * state + 1u;
        const float f = __uint_as_float(0x3f800000u | (state & 0x7fffffu));
        const float prod = f * nf;
        const int c = (int)floorf(prod - nf);
        if (c < 0 || c >= n || c == v) continue;
        if (gempe_hash_contains(table, cap, gempe_edge_key(v, c))) continue;
        return c;
    }
    return -1;
}

// Index of (c, r) in the sorted CSR row c (the edge is known to exist).
__device__ __forceinline__ long long mirror_index(const int64_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col, int c, int r) {
    long long lo = row_ptr[c], hi = row_ptr[c + 1];
    while (lo < hi) {
        const long long mid = lo + ((hi - lo) >> 1);
        if (col[mid] < r) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kSampledBlock) void k_sampled(const float *__restrict__ X, int n, int d,
                                                            const int64_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ coo_row,
                                                            const int32_t *__restrict__ col, long long nnz,
                                                            const unsigned long long *__restrict__ table,
                                                            unsigned long long cap, unsigned long long seed,
                                                            int max_tries, PairParams P, float *__restrict__ G,
                                                            float *__restrict__ Z, int32_t *__restrict__ samples,
                                                            float *__restrict__ partials) {
    __shared__ float wsum[kSampledBlock / 64];
    const long long e = (long long)blockIdx.x * kSampledBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    float loss = 0.0f;
    int r = -1, c = 0, g = -1;
    float cce = 0.0f, we = 0.0f, ccs = 0.0f, ws = 0.0f;
    if (e < nnz) {
        r = coo_row[e];
        c = col[e];
        const int side = r > c ? 1 : 0;
        const long long ec = side ? mirror_index(row_ptr, col, c, r) : e;
        const unsigned s0 = (unsigned)(gempe_mix64(seed + 2ull * (unsigned long long)ec + (unsigned long long)side +
                                                   0x9e3779b97f4a7c15ull) >> 32);
        g = draw_non_neighbour(r, n, s0, max_tries, table, cap);
        if (samples) {
            if (side) {
                samples[2 * e] = -1;
                samples[2 * e + 1] = -1;
                samples[2 * ec + 1] = g;
            } else {
                samples[2 * e] = g;
            }
        }
        const float *xr = X + (size_t)r * d;
        const float *xc = X + (size_t)c * d;
        float r2 = 0.0f;
        for (int k = 0; k < d; ++k) {
            const float df = xr[k] - xc[k];
            r2 = __builtin_fmaf(df, df, r2);
        }
        float dl;
        pair_eval_t<true>(r2, -1.0f, P, dl, cce, we);
        if (r < c) loss += dl;
        if (g >= 0) {
            const float *xg = X + (size_t)g * d;
            float r2s = 0.0f;
            for (int k = 0; k < d; ++k) {
                const float df = xr[k] - xg[k];
                r2s = __builtin_fmaf(df, df, r2s);
            }
            pair_eval_t<true>(r2s, 1.0f, P, dl, ccs, ws);
            loss += dl;
        }
    }
    // row r: both terms summed over the run of r in this wave, one atomic per run; the
    // sample's far end g: a scattered atomic
    for (int k = 0; k < d; ++k) {
        float vr = 0.0f, vg = 0.0f;
        if (r >= 0) {
            const float xk = X[(size_t)r * d + k];
            vr = cce * (xk - X[(size_t)c * d + k]);
            if (g >= 0) {
                vg = ccs * (xk - X[(size_t)g * d + k]);
                vr += vg;
            }
        }
        if (seg_sum_to_head(r, lane, vr)) atomicAdd(&G[(size_t)r * d + k], vr);
        if (g >= 0) atomicAdd(&G[(size_t)g * d + k], -vg);
    }
    float zr = (r >= 0) ? we + (g >= 0 ? ws : 0.0f) : 0.0f;
    if (seg_sum_to_head(r, lane, zr)) atomicAdd(&Z[r], zr);
    if (g >= 0) atomicAdd(&Z[g], ws);
    float v = loss;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

__global__ void k_sampled_zero(float *G, long long nd, float *Z, int n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nd) G[k] = 0.0f;
    if (k < n) Z[k] = 0.0f;
}

// FP64 sum of the block partials in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_sampled_loss(const float *__restrict__ partials, long long nb,
                                                     double *loss, unsigned *status) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (long long q = threadIdx.x; q < nb; q += 256) acc += (double)partials[q];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (loss) *loss = sh[0];
        if (!isfinite(sh[0])) atomicOr(status, 1u);
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace gempe

using namespace gempe;

// Workspace: G float[n d] | Z float[n] | partials float[nnz / 256] | status word.
size_t gempe_sampled_ws_bytes(const gempe_graph_s *g, int d) {
    const long long nb = std::max<long long>(1, (g->nnz + kSampledBlock - 1) / kSampledBlock);
    return align256(sizeof(float) * (size_t)g->n * d) + align256(sizeof(float) * (size_t)g->n) +
           align256(sizeof(float) * (size_t)nb) + 256;
}

hipError_t gempe_launch_sampled_step(const gempe_graph_s *g, int d, float *X, unsigned long long seed, int max_tries,
                                     int32_t *samples, double *loss, const PairParamsHost &pph, unsigned char *ws,
                                     bool clear_status, hipStream_t s) {
    const int n = g->n;
    const long long nd = (long long)n * d;
    const long long nb = std::max<long long>(1, (g->nnz + kSampledBlock - 1) / kSampledBlock);
    float *G = reinterpret_cast<float *>(ws);
    float *Z = reinterpret_cast<float *>(ws + align256(sizeof(float) * (size_t)nd));
    float *part = reinterpret_cast<float *>(reinterpret_cast<unsigned char *>(Z) + align256(sizeof(float) * (size_t)n));
    unsigned *status = reinterpret_cast<unsigned *>(reinterpret_cast<unsigned char *>(part) +
                                                    align256(sizeof(float) * (size_t)nb));
    const PairParams P{pph.mu_s,   pph.inv_sigma, pph.c_neg,   pph.c_pos,   pph.tk_scale,
                       pph.tk_off, pph.slope_k,   pph.r_scale, pph.w_scale, pph.wk2, pph.table_full, 0};
    const long long zn = std::max<long long>(nd, n);
    hipLaunchKernelGGL(k_sampled_zero, dim3((unsigned)((zn + 255) / 256)), dim3(256), 0, s, G, nd, Z, n);
    if (clear_status)
        hipLaunchKernelGGL(k_sampled_zero, dim3(1), dim3(64), 0, s, reinterpret_cast<float *>(status), 1LL,
                           reinterpret_cast<float *>(status), 0);
    if (g->nnz > 0)
        hipLaunchKernelGGL(k_sampled, dim3((unsigned)nb), dim3(kSampledBlock), 0, s, X, n, d, g->row_ptr, g->coo_row,
                           g->col_idx,
                           (long long)g->nnz, g->hash, (unsigned long long)g->hash_cap, seed, max_tries, P, G, Z,
                           samples, part);
    else
        hipLaunchKernelGGL(k_sampled_zero, dim3(1), dim3(64), 0, s, part, 1LL, part, 0);
    hipLaunchKernelGGL(k_sampled_loss, dim3(1), dim3(256), 0, s, part, nb, loss, status);
    return gempe_launch_wm_update(X, G, Z, d, nd, s);
}

unsigned *gempe_sampled_status(const gempe_graph_s *g, int d, unsigned char *ws) {
    const long long nd = (long long)g->n * d;
    const long long nb = std::max<long long>(1, (g->nnz + kSampledBlock - 1) / kSampledBlock);
    return reinterpret_cast<unsigned *>(ws + align256(sizeof(float) * (size_t)nd) +
                                        align256(sizeof(float) * (size_t)g->n) + align256(sizeof(float) * (size_t)nb));
}
