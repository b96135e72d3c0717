// FP32 all-pairs sweep of the GEMPE coding cost and its gradient (gfx950).
//
// Decomposition.  The n(n-1)/2 unordered pairs are covered by square super tiles of
// T x T vertices on and above the block diagonal (tile (I, J), I <= J).  One workgroup
// owns one tile; its W waves each hold 64 R rows in registers (R rows per lane) and
// sweep the tile's columns in blocks of 64 that are staged once in LDS and shared by the
// waves.  Inside a 64-column block lane l pairs its rows with column (l + s) mod 64 at
// step s = 0..63 (a Latin-square schedule: at every step the 64 lanes touch 64 distinct
// columns), so
//   - the row side of the gradient, g_i += cc (x_i - x_j), accumulates in registers;
//   - the column side, g_j -= cc (x_i - x_j), accumulates in a register that moves one
//     lane per step with a DPP wave rotation, so it follows its column through the
//     lanes and is back in lane l (holding column l) after 64 steps;
//   - the W waves' column partials are combined in LDS and leave with one global FP32
//     atomic per (column, coordinate) per tile; rows leave once per tile.
// Sums are two-level: per 64-column block in registers, then across blocks, then across
// tiles (atomics).  The loss partial of a tile is one FP32 number written to a fixed
// slot; the final sum over slots is FP64 in a fixed order (deterministic loss).
//
// Every pair is scored as a non-edge in the sweep.  Edges are corrected exactly by a
// second pass over the CSR entries (k_edges): it adds dl+ - dl- and (cc+ - cc-)(x_i - x_j)
// computed with the same FP32 code at the same distance, and counts every pair i<j it
// scores as an edge after confirming it in the exact edge hash.  Membership per pair is
// therefore exact, and the O(n^2) sweep carries no per-pair membership test.
//
// Wide embeddings (d > 16) use k_sweep_wide: the same schedule with rows, row
// gradients, columns and column gradients all in LDS (the Latin-square schedule makes
// the read-modify-writes race-free without atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "pairfn.h"

namespace gempe {

constexpr int kXcd = 8;  // MI355X: workgroups are dealt round-robin over 8 XCDs

// Upper-triangle tile t (row-major over I <= J < nt) -> (I, J).
__device__ inline void tile_of(long long t, int nt, int &I, int &J) {
    double b = 2.0 * nt + 1.0;
    long long i = (long long)floor((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
    if (i < 0) i = 0;
    if (i > nt - 1) i = nt - 1;
    auto start = [nt](long long ii) { return ii * nt - ii * (ii - 1) / 2; };
    while (i > 0 && start(i) > t) --i;
    while (i + 1 < nt && start(i + 1) <= t) ++i;
    I = (int)i;
    J = (int)(i + (t - start(i)));
}

// Workgroup b -> tile index such that the workgroups one XCD receives (b = x, x+8, ...)
// take consecutive tiles (same row strip: x_I stays in that XCD's L2).
__device__ inline long long xcd_item(long long b, long long per_xcd) {
    return (b % kXcd) * per_xcd + b / kXcd;
}

__device__ __forceinline__ float rot1(float v) {
    // DPP wave rotation by one lane (row_mask/bank_mask all, no bound control)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int D>
__device__ __forceinline__ float sqdist(const float (&a)[D], const float (&b)[D], float (&diff)[D]) {
    float r2 = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        diff[k] = a[k] - b[k];
        r2 = __builtin_fmaf(diff[k], diff[k], r2);
    }
    return r2;
}

// ------------------------------------------------------------------------------------
// Register-resident sweep, d <= 16.
// ------------------------------------------------------------------------------------
template <int D, int R, int W, bool ROWLOSS>
__global__ __launch_bounds__(64 * W) void k_sweep_small(const float *__restrict__ X, int n, int d,
                                                        int nt, long long items, long long per_xcd,
                                                        float *__restrict__ G,
                                                        float *__restrict__ rowloss,
                                                        float *__restrict__ partials, PairParams P) {
    constexpr int T = 64 * R * W;
    constexpr int NC = D + (ROWLOSS ? 1 : 0);
    __shared__ float xs[64 * D];
    __shared__ float cs[W > 1 ? 64 * NC : 1];
    __shared__ float lsum[W];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const long long t = xcd_item(blockIdx.x, per_xcd);
    if (t >= items) return;  // uniform over the workgroup
    int I, J;
    tile_of(t, nt, I, J);
    // rotation direction of the DPP wave rotate (data from lane l+1 or l-1)
    const int dir = (__float_as_int(rot1(__int_as_float(lane))) == ((lane + 1) & 63)) ? 1 : -1;

    const int row0 = I * T + wave * 64 * R;
    int irow[R];
    float xi[R][D], gi[R][D], li[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        irow[r] = row0 + r * 64 + lane;
        li[r] = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            gi[r][k] = 0.0f;
            xi[r][k] = (irow[r] < n && k < d) ? X[(size_t)irow[r] * d + k] : 0.0f;
        }
    }
    const bool masked = (I == J) || ((long long)(J + 1) * T > n);
    float loss_acc = 0.0f;

    for (int cb = 0; cb < T / 64; ++cb) {
        const int c0 = J * T + cb * 64;
        __syncthreads();
        for (int k = threadIdx.x; k < 64 * D; k += 64 * W) {
            int c = k / D, dd = k - c * D, j = c0 + c;
            xs[k] = (j < n && dd < d) ? X[(size_t)j * d + dd] : 0.0f;
        }
        if (W > 1)
            for (int k = threadIdx.x; k < 64 * NC; k += 64 * W) cs[k] = 0.0f;
        __syncthreads();

        // every pair of this wave and block has j <= i: nothing to do
        const bool skip = masked && (c0 + 63 <= row0);
        float colacc[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) colacc[k] = 0.0f;
        float blk_loss = 0.0f;
        float bg[R][D];
        float bl[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bl[r] = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) bg[r][k] = 0.0f;
        }
        if (!skip) {
            for (int s = 0; s < 64; ++s) {
                const int c = (lane + dir * s) & 63;
                const int j = c0 + c;
                float xc[D];
#pragma unroll
                for (int k = 0; k < D; ++k) xc[k] = xs[c * D + k];
                float tc[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) tc[k] = 0.0f;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float diff[D];
                    float r2 = sqdist<D>(xi[r], xc, diff);
                    float dl, cc;
                    pair_nonedge(r2, P, dl, cc);
                    if (masked) {
                        bool valid = (irow[r] < j) && (j < n);
                        dl = valid ? dl : 0.0f;
                        cc = valid ? cc : 0.0f;
                    }
                    blk_loss += dl;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        float f = cc * diff[k];
                        bg[r][k] += f;
                        tc[k] += f;
                    }
                    if (ROWLOSS) {
                        bl[r] += dl;
                        tc[NC - 1] += dl;
                    }
                }
#pragma unroll
                for (int k = 0; k < NC; ++k) colacc[k] = rot1(colacc[k] + tc[k]);
            }
        }
        // lane l now holds the column partial of column c0 + l
        const int jc = c0 + lane;
        if (W == 1) {
            if (!skip && jc < n) {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k < d) atomicAdd(&G[(size_t)jc * d + k], -colacc[k]);
                if (ROWLOSS) atomicAdd(&rowloss[jc], colacc[NC - 1]);
            }
        } else {
            if (!skip) {
#pragma unroll
                for (int k = 0; k < NC; ++k) atomicAdd(&cs[lane * NC + k], colacc[k]);
            }
            __syncthreads();
            for (int k = threadIdx.x; k < 64 * NC; k += 64 * W) {
                int c = k / NC, dd = k - c * NC, j = c0 + c;
                if (j < n) {
                    if (dd < D) {
                        if (dd < d) atomicAdd(&G[(size_t)j * d + dd], -cs[k]);
                    } else if (ROWLOSS) {
                        atomicAdd(&rowloss[j], cs[k]);
                    }
                }
            }
        }
        loss_acc += blk_loss;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            li[r] += bl[r];
#pragma unroll
            for (int k = 0; k < D; ++k) gi[r][k] += bg[r][k];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (irow[r] < n) {
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (k < d) atomicAdd(&G[(size_t)irow[r] * d + k], gi[r][k]);
            if (ROWLOSS) atomicAdd(&rowloss[irow[r]], li[r]);
        }
    }
    float ws = wave_sum(loss_acc);
    if (lane == 0) lsum[wave] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.0f;
#pragma unroll
        for (int w = 0; w < W; ++w) tot += lsum[w];
        partials[t] = tot;
    }
}

// ------------------------------------------------------------------------------------
// LDS-resident sweep for wide embeddings (d in 17..128), one wave per workgroup, T = 64.
// ------------------------------------------------------------------------------------
template <int D, bool ROWLOSS>
__global__ __launch_bounds__(64) void k_sweep_wide(const float *__restrict__ X, int n, int d, int nt,
                                                   long long items, long long per_xcd,
                                                   float *__restrict__ G, float *__restrict__ rowloss,
                                                   float *__restrict__ partials, PairParams P) {
    constexpr int S = D + 1;  // padded stride: lane-private rows hit distinct banks
    extern __shared__ float lds[];
    float *xr = lds;           // rows    [64][S]
    float *gr = xr + 64 * S;   // row gradients
    float *xc = gr + 64 * S;   // columns
    float *gc = xc + 64 * S;   // column gradients
    const int lane = threadIdx.x;
    const long long t = xcd_item(blockIdx.x, per_xcd);
    if (t >= items) return;
    int I, J;
    tile_of(t, nt, I, J);
    const int i = I * 64 + lane;
    for (int k = lane; k < 64 * S; k += 64) {
        int c = k / S, dd = k - c * S;
        int ri = I * 64 + c, cj = J * 64 + c;
        xr[k] = (ri < n && dd < d) ? X[(size_t)ri * d + dd] : 0.0f;
        xc[k] = (cj < n && dd < d) ? X[(size_t)cj * d + dd] : 0.0f;
        gr[k] = 0.0f;
        gc[k] = 0.0f;
    }
    __syncthreads();
    const bool masked = (I == J) || ((long long)(J + 1) * 64 > n);
    float loss = 0.0f, lrow = 0.0f;
    for (int s = 0; s < 64; ++s) {
        const int c = (lane + s) & 63;
        const int j = J * 64 + c;
        const float *a = xr + lane * S;
        const float *b = xc + c * S;
        float r2 = 0.0f;
        for (int k = 0; k < D; ++k) {
            float df = a[k] - b[k];
            r2 = __builtin_fmaf(df, df, r2);
        }
        float dl, cc;
        pair_nonedge(r2, P, dl, cc);
        if (masked) {
            bool valid = (i < j) && (j < n);
            dl = valid ? dl : 0.0f;
            cc = valid ? cc : 0.0f;
        }
        loss += dl;
        if (ROWLOSS) lrow += dl;
        float *ga = gr + lane * S;
        float *gb = gc + c * S;
        for (int k = 0; k < D; ++k) {
            float f = cc * (a[k] - b[k]);
            ga[k] += f;
            gb[k] -= f;
        }
        if (ROWLOSS) gb[D] += dl;  // the pad column carries the column row-loss
        // next step reads columns another lane just wrote: keep LDS program order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    for (int k = lane; k < 64 * S; k += 64) {
        int c = k / S, dd = k - c * S;
        int ri = I * 64 + c, cj = J * 64 + c;
        if (dd < d) {
            if (ri < n) atomicAdd(&G[(size_t)ri * d + dd], gr[k]);
            if (cj < n) atomicAdd(&G[(size_t)cj * d + dd], gc[k]);
        } else if (ROWLOSS && dd == D && cj < n) {
            atomicAdd(&rowloss[cj], gc[k]);
        }
    }
    if (ROWLOSS && i < n) atomicAdd(&rowloss[i], lrow);
    float wsum = wave_sum(loss);
    if (lane == 0) partials[t] = wsum;
}

// ------------------------------------------------------------------------------------
// Exact edge correction over CSR entries.
// ------------------------------------------------------------------------------------
constexpr int kEdgeBlock = 256;

template <bool ROWLOSS>
__global__ __launch_bounds__(kEdgeBlock) void k_edges(const float *__restrict__ X, int d,
                                                      const int32_t *__restrict__ coo_row,
                                                      const int32_t *__restrict__ col, long long nnz,
                                                      const unsigned long long *__restrict__ table,
                                                      unsigned long long cap, float *__restrict__ G,
                                                      float *__restrict__ rowloss,
                                                      float *__restrict__ partials,
                                                      unsigned long long *hits, PairParams P) {
    __shared__ float wsum[kEdgeBlock / 64];
    __shared__ unsigned whit[kEdgeBlock / 64];
    long long e = (long long)blockIdx.x * kEdgeBlock + threadIdx.x;
    float dloss = 0.0f;
    unsigned hit = 0;
    if (e < nnz) {
        const int i = coo_row[e];
        const int j = col[e];
        const float *xi = X + (size_t)i * d;
        const float *xj = X + (size_t)j * d;
        float r2 = 0.0f;
        for (int k = 0; k < d; ++k) {
            float df = xi[k] - xj[k];
            r2 = __builtin_fmaf(df, df, r2);
        }
        float dlp, ccp, dln, ccn;
        pair_eval(r2, -1.0f, P, dlp, ccp);
        pair_eval(r2, 1.0f, P, dln, ccn);
        const float dcc = ccp - ccn;
        for (int k = 0; k < d; ++k) atomicAdd(&G[(size_t)i * d + k], dcc * (xi[k] - xj[k]));
        const float ddl = dlp - dln;
        if (ROWLOSS) atomicAdd(&rowloss[i], ddl);
        if (i < j) {
            dloss = ddl;
            hit = gempe_hash_contains(table, cap, gempe_edge_key(i, j)) ? 1u : 0u;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float s = wave_sum(dloss);
    unsigned long long b = __ballot(hit != 0);
    if (lane == 0) {
        wsum[wave] = s;
        whit[wave] = (unsigned)__popcll(b);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.0f;
        unsigned h = 0;
        for (int w = 0; w < kEdgeBlock / 64; ++w) tot += wsum[w], h += whit[w];
        partials[blockIdx.x] = tot;
        if (h) atomicAdd(hits, (unsigned long long)h);
    }
}

// ------------------------------------------------------------------------------------
// Small kernels: zero fill, FP64 fixed-order loss reduction, X -= eta G.
// ------------------------------------------------------------------------------------
__global__ void k_zero(float *__restrict__ a, long long na, float *__restrict__ b, long long nb,
                       unsigned long long *counters, int ncounters) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = k; q < na; q += stride) a[q] = 0.0f;
    for (long long q = k; q < nb; q += stride) b[q] = 0.0f;
    if (k < ncounters) counters[k] = 0ull;
}

constexpr int kFinBlock = 256;

__device__ inline double block_sum_fixed(const float *__restrict__ partials, long long count,
                                         double *sh) {
    double acc = 0.0;
    for (long long q = threadIdx.x; q < count; q += kFinBlock) acc += (double)partials[q];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kFinBlock / 2; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(kFinBlock) void k_finalize(const float *__restrict__ partials,
                                                        long long count, double *loss,
                                                        const unsigned long long *hits,
                                                        int64_t *hits_out, unsigned *status) {
    __shared__ double sh[kFinBlock];
    double tot = block_sum_fixed(partials, count, sh);
    if (threadIdx.x == 0) {
        *loss = tot;
        if (hits_out) *hits_out = (int64_t)*hits;
        if (!isfinite(tot)) atomicOr(status, kStatusNonFinite);
    }
}

__global__ void k_axpy(float *__restrict__ X, const float *__restrict__ G, float eta, long long count) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) X[k] = __builtin_fmaf(-eta, G[k], X[k]);
}

}  // namespace gempe

// ======================================================================================
// Host side: plan, workspace layout, launches.
// ======================================================================================
using namespace gempe;

namespace {

int padded_dim(int d) {
    if (d <= 4) return d;
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    return 128;
}

long long tiles_for(int n, int T) {
    long long nt = (n + T - 1) / T;
    return nt * (nt + 1) / 2;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

SweepPlan gempe_make_plan(const gempe_graph_s *g, int d) {
    SweepPlan p;
    p.D = padded_dim(d);
    if (p.D <= 16) {
        // largest tiles that still give >= 8 waves per SIMD (256 CUs x 4 SIMDs)
        static const int cand_small[][2] = {{4, 4}, {2, 4}, {1, 4}, {1, 2}, {1, 1}};
        static const int cand_16[][2] = {{2, 4}, {1, 4}, {1, 2}, {1, 1}};
        const int(*cand)[2] = p.D <= 4 ? cand_small : cand_16;
        int nc = p.D <= 4 ? 5 : 4;
        p.R = 1;
        p.W = 1;
        for (int c = 0; c < nc; ++c) {
            int T = 64 * cand[c][0] * cand[c][1];
            if (tiles_for(g->n, T) * cand[c][1] >= 8 * 1024) {
                p.R = cand[c][0];
                p.W = cand[c][1];
                break;
            }
        }
        p.T = 64 * p.R * p.W;
    } else {
        p.R = 1;
        p.W = 1;
        p.T = 64;
    }
    p.nt = (g->n + p.T - 1) / p.T;
    p.items = (long long)p.nt * (p.nt + 1) / 2;
    long long per = (p.items + kXcd - 1) / kXcd;
    p.grid = per * kXcd;
    p.edge_blocks = (int)std::max<long long>(1, (g->nnz + kEdgeBlock - 1) / kEdgeBlock);
    p.partials = p.items + p.edge_blocks;
    return p;
}

WsLayout gempe_ws_layout(const gempe_graph_s *g, int d, const SweepPlan &plan) {
    WsLayout L;
    size_t nd = (size_t)g->n * (size_t)d;
    size_t off = 0;
    L.counters = off;
    off += 256;
    L.partials = off;
    off = align256(off + sizeof(float) * (size_t)plan.partials);
    L.gbuf = off;
    off = align256(off + sizeof(float) * nd);
    L.xbuf = off;
    off = align256(off + sizeof(float) * 2 * nd);
    L.gring = off;
    off = align256(off + sizeof(float) * 3 * nd);
    L.ppart = off;
    off = align256(off + sizeof(float) * 2 * (size_t)plan.partials);
    L.barrier = off;
    off += 256;
    L.total = off;
    return L;
}

PairParamsHost gempe_pair_params(const gempe_params *p) {
    PairParamsHost h;
    h.mu = (float)p->mu;
    h.inv_sigma = (float)(1.0 / p->sigma);
    h.d1_scale = (float)(-1.0 / (p->sigma * 0.69314718055994530942));
    return h;
}

namespace {

template <int D, int R, int W, bool RL>
void launch_small(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                  float *part, PairParams P) {
    long long per = pl.grid / kXcd;
    hipLaunchKernelGGL((k_sweep_small<D, R, W, RL>), dim3((unsigned)pl.grid), dim3(64 * W), 0, s, X, n, d,
                       pl.nt, pl.items, per, G, rl, part, P);
}

template <int D, bool RL>
void launch_small_rw(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                     float *part, PairParams P) {
    if (pl.R == 1 && pl.W == 1) return launch_small<D, 1, 1, RL>(pl, s, X, n, d, G, rl, part, P);
    if (pl.R == 1 && pl.W == 2) return launch_small<D, 1, 2, RL>(pl, s, X, n, d, G, rl, part, P);
    if (pl.R == 1 && pl.W == 4) return launch_small<D, 1, 4, RL>(pl, s, X, n, d, G, rl, part, P);
    if (pl.R == 2 && pl.W == 4) return launch_small<D, 2, 4, RL>(pl, s, X, n, d, G, rl, part, P);
    if constexpr (D <= 4) {
        if (pl.R == 4 && pl.W == 4) return launch_small<D, 4, 4, RL>(pl, s, X, n, d, G, rl, part, P);
    }
}

template <int D, bool RL>
void launch_wide(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                 float *part, PairParams P) {
    long long per = pl.grid / kXcd;
    size_t lds = sizeof(float) * 4 * 64 * (D + 1);
    hipLaunchKernelGGL((k_sweep_wide<D, RL>), dim3((unsigned)pl.grid), dim3(64), lds, s, X, n, d, pl.nt,
                       pl.items, per, G, rl, part, P);
}

template <bool RL>
void launch_sweep(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                  float *part, PairParams P) {
    switch (pl.D) {
        case 1: return launch_small_rw<1, RL>(pl, s, X, n, d, G, rl, part, P);
        case 2: return launch_small_rw<2, RL>(pl, s, X, n, d, G, rl, part, P);
        case 3: return launch_small_rw<3, RL>(pl, s, X, n, d, G, rl, part, P);
        case 4: return launch_small_rw<4, RL>(pl, s, X, n, d, G, rl, part, P);
        case 8: return launch_small_rw<8, RL>(pl, s, X, n, d, G, rl, part, P);
        case 16: return launch_small_rw<16, RL>(pl, s, X, n, d, G, rl, part, P);
        case 32: return launch_wide<32, RL>(pl, s, X, n, d, G, rl, part, P);
        case 64: return launch_wide<64, RL>(pl, s, X, n, d, G, rl, part, P);
        default: return launch_wide<128, RL>(pl, s, X, n, d, G, rl, part, P);
    }
}

}  // namespace

hipError_t gempe_launch_loss_grad(const gempe_graph_s *g, int d, const SweepPlan &plan, const float *X,
                                  float *grad, float *row_loss, float *partials, unsigned char *counters,
                                  double *loss, int64_t *hits_out, const PairParamsHost &pph,
                                  hipStream_t s, bool clear_status) {
    PairParams P{pph.mu, pph.inv_sigma, pph.d1_scale};
    const int n = g->n;
    const long long nd = (long long)n * d;
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(counters);
    unsigned *status = reinterpret_cast<unsigned *>(counters + 8);
    {
        long long big = std::max<long long>(nd, row_loss ? n : 0);
        unsigned blocks = (unsigned)std::min<long long>(4096, std::max<long long>(1, (big + 255) / 256));
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, grad, nd, row_loss, row_loss ? (long long)n : 0,
                           cnt, clear_status ? 2 : 1);
    }
    if (row_loss)
        launch_sweep<true>(plan, s, X, n, d, grad, row_loss, partials, P);
    else
        launch_sweep<false>(plan, s, X, n, d, grad, row_loss, partials, P);
    float *epart = partials + plan.items;
    if (g->nnz > 0) {
        if (row_loss)
            hipLaunchKernelGGL((k_edges<true>), dim3(plan.edge_blocks), dim3(kEdgeBlock), 0, s, X, d, g->coo_row,
                               g->col_idx, (long long)g->nnz, g->hash, (unsigned long long)g->hash_cap, grad,
                               row_loss, epart, cnt, P);
        else
            hipLaunchKernelGGL((k_edges<false>), dim3(plan.edge_blocks), dim3(kEdgeBlock), 0, s, X, d, g->coo_row,
                               g->col_idx, (long long)g->nnz, g->hash, (unsigned long long)g->hash_cap, grad,
                               row_loss, epart, cnt, P);
    } else {
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, epart, (long long)plan.edge_blocks, nullptr, 0LL,
                           nullptr, 0);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, s, partials, plan.partials, loss, cnt,
                       hits_out, status);
    return hipGetLastError();
}

hipError_t gempe_launch_axpy(float *X, const float *G, float eta, long long count, hipStream_t s) {
    unsigned blocks = (unsigned)std::max<long long>(1, (count + 255) / 256);
    hipLaunchKernelGGL(k_axpy, dim3(blocks), dim3(256), 0, s, X, G, eta, count);
    return hipGetLastError();
}
