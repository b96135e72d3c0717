// FP32 all-pairs sweep of the GEMPE coding cost and its gradient (gfx950).
//
// Decomposition.  The n(n-1)/2 unordered pairs are covered by square tiles on and above
// the block diagonal.  A wave holds 64 R rows in registers (R rows per lane) and meets
// columns in blocks of 64.  Within a block, lane l pairs its rows with column
// (l + s) mod 64 at step s = 0..63 (a Latin-square schedule: at every step the 64 lanes
// touch 64 distinct columns).  The column's coordinates and its gradient accumulator
// travel with it: both move one lane per step by a DPP wave rotation, so the inner loop
// touches neither LDS nor memory, and after 64 steps lane l again holds column l.
//   - row side of the gradient, g_i += cc (x_i - x_j): registers;
//   - column side, g_j -= cc (x_i - x_j): the rotating accumulator, flushed once per
//     block (several waves first combine theirs through private LDS slots);
//   - loss: per-lane FP32 sums, one FP32 partial per work unit in a fixed slot, summed
//     in FP64 in slot order (deterministic).
//
// Every pair is scored as a non-edge in the sweep.  Edges are corrected exactly by a
// pass over the CSR entries: it adds dl+ - dl- and (cc+ - cc-)(x_i - x_j), computed by
// the same FP32 code at the same distance, so membership per pair is exact without a
// membership test in the O(n^2) loop.  The standalone edge kernel also counts the pairs
// i<j it scores as edges after confirming each one in the exact edge hash.
//
// Three entry kernels:
//   k_sweep_small   d <= 16, one launch per evaluation, tiles of 64 R W rows shared by W
//                   waves (large n);
//   k_sweep_wide    17 <= d <= 128, rows/columns and both gradients in LDS;
//   k_iter          d <= 16, small n: one fused launch per gradient-descent iteration
//                   (sweep, edge pass, previous step, FP64 loss of the previous
//                   iteration), one workgroup per 64 x 64 tile with its four waves
//                   splitting the 64 steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "pairfn.h"
#include "ltab_stage.h"
#include "tiles.h"

namespace gempe {

// The two-float4 form (pair_nonedge_tab2) of the same table: 2 kLtabF4 float4, staged by a
// workgroup of 256 threads in two halves, so that other loads can be issued between them:
// ltab2_load reads this thread's entries, ltab2_store writes them to LDS.
constexpr int kLtab2Per = (kLtabF4 + 255) / 256;
__device__ __forceinline__ void ltab2_load(float4 (&c)[kLtab2Per]) {
    const float4 *src = reinterpret_cast<const float4 *>(kLtab);
#pragma unroll
    for (int r = 0; r < kLtab2Per; ++r) {
        const int q = (int)threadIdx.x + 256 * r;
        c[r] = src[q < kLtabF4 ? q : kLtabF4 - 1];
    }
}
__device__ __forceinline__ void ltab2_store(float4 *dst, const float4 (&c)[kLtab2Per], float slope_k) {
#pragma unroll
    for (int r = 0; r < kLtab2Per; ++r) {
        const int q = (int)threadIdx.x + 256 * r;
        if (q < kLtabF4) {
            const float n0 = rintf(c[r].x);
            dst[2 * q] = make_float4(__int_as_float((int)n0), c[r].x - n0, c[r].y, c[r].z);
            dst[2 * q + 1] =
                make_float4(c[r].w, slope_k * c[r].y, slope_k * (2.0f * c[r].z), slope_k * (3.0f * c[r].w));
        }
    }
}

// The long sweeps drop the below-table test (P.table_full) only from this dimension up:
// at d = 2 the version with the test measured faster (the test's branch is never taken,
// and the compiler schedules that loop better), at d = 16 the version without it.
constexpr int kNoChkMinD = 8;

template <bool W = false, bool TWO = false, bool CHK = true>
__device__ __forceinline__ void nonedge(float r2, const PairParams &P, const float4 *tab, float tko, float &dl,
                                        float &cc, float &w) {
    nonedge_eval<W, TWO, CHK>(r2, P, tab, tko, kLtabSegs, dl, cc, w);
}

// What the per-vertex "extra" output of a sweep accumulates (the array called rowloss /
// extra in the kernels): nothing, the row loss L_i = sum_j dl_ij, or the weighted-
// majorization denominator z_i = sum_j w_ij (Eq. 5).
constexpr int kExNone = 0, kExRowLoss = 1, kExZ = 2;

// Coordinates of the current iterate: X[v], or X[v] - eta G[v] when a step of gradient
// descent is applied on the fly (fused iteration).  Both the sweep and the edge pass read
// through this view, so they see bit-identical coordinates.
struct XView {
    const float *X;
    const float *Gp;  // previous gradient, or nullptr
    float neg_eta;
    int d;
    __device__ __forceinline__ float at(long long v, int k) const {
        size_t o = (size_t)v * d + k;
        return Gp ? __builtin_fmaf(neg_eta, Gp[o], X[o]) : X[o];
    }
};


// Steps [s0, s1) of the Latin-square schedule against one block of 64 columns starting at
// col0.  At step s lane l meets column c_l(s) = col0 + ((l + dir s) mod 64); xc holds that
// column's coordinates and rotates after each step.  colacc lags one step: before step s
// it holds the partial of column c_l(s-1) = c_{l-dir}(s), so rotating it by one lane
// realigns it with c_l(s), and the rotation and this step's addition are one DPP add.
// After the last step lane l holds the partial of column c_l(s1 - 1).
// CHK: test each pair for tau below the table (may be false when P.table_full).
template <int D, int R, bool MASK, int EX, bool TWO = false, bool CHK = true>
__device__ __forceinline__ void sweep_steps(const float (&xi)[R][D], const int (&irow)[R], float (&xc)[D],
                                            float (&colacc)[D + (EX != 0 ? 1 : 0)], float (&gi)[R][D],
                                            float (&li)[R], float &loss, int lane, int dir, int col0, int n,
                                            int s0, int s1, const PairParams &P, const float4 *tab) {
    constexpr int NC = D + (EX != 0 ? 1 : 0);
    const float tko = table_offset(P, kLtabZero);
    for (int s = s0; s < s1; ++s) {
        int j = 0;
        if (MASK) j = col0 + ((lane + dir * s) & 63);
        float tc[NC];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float diff[D];
            float r2 = sqdist_eps<D>(xi[r], xc, diff);
            float dl, cc, w = 0.0f;
            nonedge<EX == kExZ, TWO, CHK>(r2, P, tab, tko, dl, cc, w);
            if (MASK) {
                bool valid = (irow[r] < j) && (j < n);
                dl = valid ? dl : 0.0f;
                cc = valid ? cc : 0.0f;
                w = valid ? w : 0.0f;
            }
            loss += dl;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                gi[r][k] = __builtin_fmaf(cc, diff[k], gi[r][k]);
                tc[k] = (r == 0) ? cc * diff[k] : __builtin_fmaf(cc, diff[k], tc[k]);
            }
            if (EX) {
                const float ex = (EX == kExZ) ? w : dl;
                li[r] += ex;
                tc[NC - 1] = (r == 0) ? ex : tc[NC - 1] + ex;
            }
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) colacc[k] = rot1_fold(colacc[k]) + tc[k];
#pragma unroll
        for (int k = 0; k < D; ++k) xc[k] = rot1(xc[k]);
    }
}

// ------------------------------------------------------------------------------------
// Register-resident sweep, d <= 16, one launch per evaluation.
// ------------------------------------------------------------------------------------
template <int D, int R, int W, int EX>
__global__ __launch_bounds__(64 * W) void k_sweep_small(const float *__restrict__ X, int n, int d,
                                                        int nt, long long items, long long per_xcd,
                                                        float *__restrict__ G,
                                                        float *__restrict__ rowloss,
                                                        float *__restrict__ partials, PairParams P, int shard,
                                                        int nshards) {
    constexpr int T = 64 * R * W;
    constexpr int NC = D + (EX != 0 ? 1 : 0);
    __shared__ float cs[W > 1 ? W * 64 * NC : 1];  // per-wave column partials
    __shared__ float lsum[W];
    __shared__ float4 ltab[kLtabF4];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    long long t = xcd_item(blockIdx.x, per_xcd);
    if (t >= items) return;  // uniform over the workgroup
    if (P.reverse) t = items - 1 - t;
    stage_ltab(ltab);
    __syncthreads();
    int I, J;
    item_tile(t, nt, shard, nshards, I, J);
    const int dir = rot_dir(lane);

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
        if (W > 1) __syncthreads();  // the previous block's column partials are consumed
        // every pair of this wave and block has j <= i: nothing to do
        const bool skip = masked && (c0 + 63 <= row0);
        float colacc[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) colacc[k] = 0.0f;
        // two-level sums: per 64-column block, then across blocks
        float blk = 0.0f;
        float bg[R][D], bl[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bl[r] = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) bg[r][k] = 0.0f;
        }
        if (!skip) {
            float xc[D];
            const int jc = c0 + lane;
#pragma unroll
            for (int k = 0; k < D; ++k) xc[k] = (jc < n && k < d) ? X[(size_t)jc * d + k] : 0.0f;
            if (D >= kNoChkMinD && P.table_full) {
                if (masked)
                    sweep_steps<D, R, true, EX, false, false>(xi, irow, xc, colacc, bg, bl, blk, lane, dir, c0, n,
                                                              0, 64, P, ltab);
                else
                    sweep_steps<D, R, false, EX, false, false>(xi, irow, xc, colacc, bg, bl, blk, lane, dir, c0,
                                                               n, 0, 64, P, ltab);
            } else {
                if (masked)
                    sweep_steps<D, R, true, EX>(xi, irow, xc, colacc, bg, bl, blk, lane, dir, c0, n, 0, 64, P,
                                                ltab);
                else
                    sweep_steps<D, R, false, EX>(xi, irow, xc, colacc, bg, bl, blk, lane, dir, c0, n, 0, 64, P,
                                                 ltab);
            }
        }
        // lane l now holds the partial of column c_l(63)
        const int jc = c0 + ((lane + 63 * dir) & 63);
        if (W == 1) {
            if (!skip && jc < n) {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k < d) atomicAdd(&G[(size_t)jc * d + k], -colacc[k]);
                if (EX) atomicAdd(&rowloss[jc], colacc[NC - 1]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NC; ++k) cs[(wave * 64 + (jc - c0)) * NC + k] = skip ? 0.0f : colacc[k];
            __syncthreads();
            for (int k = threadIdx.x; k < 64 * NC; k += 64 * W) {
                int c = k / NC, dd = k - c * NC, j = c0 + c;
                float v = 0.0f;
#pragma unroll
                for (int w = 0; w < W; ++w) v += cs[w * 64 * NC + k];
                if (j < n) {
                    if (dd < D) {
                        if (dd < d) atomicAdd(&G[(size_t)j * d + dd], -v);
                    } else if (EX) {
                        atomicAdd(&rowloss[j], v);
                    }
                }
            }
        }
        loss_acc += blk;
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
            if (EX) atomicAdd(&rowloss[irow[r]], li[r]);
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
// LDS-resident sweep for wide embeddings (d in 17..128, and the exact pass of the BF16
// screen), one wave per workgroup, tiles of 64 x 64.
// ------------------------------------------------------------------------------------
// FLUSH (BF16 screen's exact pass only): a step whose 64 exact distances all satisfy
// delta^2 >= far2 = (mu + near_k sigma)^2 skips the pair function and the gradient: those
// pairs are far non-edges, flushed exactly as the screen flushes them.  D = 16 (the BF16
// path's dense tiles with per-vertex extras) takes the non-edge value from the staged table
// ltab, as that path's other passes do; wider tiles the closed form.
template <int D, int EX, bool FLUSH>
__device__ float wide_tile(const float *__restrict__ X, int n, int d, int I, int J, float *__restrict__ G,
                           float *__restrict__ rowloss, const PairParams &P, float *lds, float far2,
                           const float4 *ltab) {
    constexpr int S = D + 1;  // padded stride: lane-private rows hit distinct banks
    float *xr = lds;           // rows    [64][S]
    float *gr = xr + 64 * S;   // row gradients
    float *xc = gr + 64 * S;   // columns
    float *gc = xc + 64 * S;   // column gradients
    const int lane = threadIdx.x;
    const int i = I * 64 + lane;
    __syncthreads();  // the previous tile's LDS contents are consumed
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
        if (FLUSH && __ballot(!(r2 >= far2)) == 0ull) continue;  // wave-uniform: every pair far
        float dl, cc, w = 0.0f;
        if (D == 16)
            nonedge<EX == kExZ>(r2 + kFltMin, P, ltab, table_offset(P, kLtabZero), dl, cc, w);
        else
            pair_eval_t<EX == kExZ, !FLUSH>(r2, 1.0f, P, dl, cc, w);  // flushed far pairs need no tail
        if (masked) {
            bool valid = (i < j) && (j < n);
            dl = valid ? dl : 0.0f;
            cc = valid ? cc : 0.0f;
            w = valid ? w : 0.0f;
        }
        if (FLUSH && r2 >= far2) dl = 0.0f, cc = 0.0f, w = 0.0f;
        loss += dl;
        const float ex = (EX == kExZ) ? w : dl;
        if (EX) lrow += ex;
        float *ga = gr + lane * S;
        float *gb = gc + c * S;
        for (int k = 0; k < D; ++k) {
            float f = cc * (a[k] - b[k]);
            ga[k] += f;
            gb[k] -= f;
        }
        if (EX) gb[D] += ex;  // the pad column carries the column's extra sum
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
        } else if (EX && dd == D && cj < n) {
            atomicAdd(&rowloss[cj], gc[k]);
        }
    }
    if (EX && i < n) atomicAdd(&rowloss[i], lrow);
    return wave_sum(loss);
}

template <int D, int EX>
__global__ __launch_bounds__(64) void k_sweep_wide(const float *__restrict__ X, int n, int d, int nt,
                                                   long long items, long long per_xcd,
                                                   float *__restrict__ G, float *__restrict__ rowloss,
                                                   float *__restrict__ partials, PairParams P, int shard,
                                                   int nshards) {
    extern __shared__ float lds[];
    long long t = xcd_item(blockIdx.x, per_xcd);
    if (t >= items) return;
    if (P.reverse) t = items - 1 - t;
    int I, J;
    item_tile(t, nt, shard, nshards, I, J);
    float l = wide_tile<D, EX, false>(X, n, d, I, J, G, rowloss, P, lds, 0.0f, nullptr);
    if (threadIdx.x == 0) partials[t] = l;
}

// Exact FP32 pass over the tiles the BF16 screen flagged: list[0..*count) holds upper-
// triangle 64 x 64 tile indices in increasing order; partial slot q belongs to list[q].
template <int D, int EX>
__global__ __launch_bounds__(64) void k_sweep_wide_list(const float *__restrict__ X, int n, int d, int nt,
                                                        const int *__restrict__ list, const int *__restrict__ count,
                                                        float *__restrict__ G, float *__restrict__ rowloss,
                                                        float *__restrict__ partials, PairParams P, float far2,
                                                        const unsigned char *__restrict__ dense,
                                                        const int *__restrict__ all_dense) {
    extern __shared__ float lds[];
    if (*all_dense) return;  // the full matrix-core sweep took every tile (uniform over the grid)
    __shared__ float4 ltab[D == 16 ? kLtabF4 : 1];
    if (D == 16) stage_ltab(ltab);  // ordered before use by the tile's first barrier
    const int cnt = *count;
    for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
        if (!dense[q]) continue;  // finished by the sparse pass (k_near_tiles)
        int I, J;
        tile_of(list[q], nt, I, J);
        float l = wide_tile<D, EX, true>(X, n, d, I, J, G, rowloss, P, lds, far2, ltab);
        if (threadIdx.x == 0) partials[q] = l;
    }
}

// ------------------------------------------------------------------------------------
// Exact edge correction of one CSR entry (i, j) in the fused iteration (two-float4 table):
// the gradient change (cc+ - cc-)(x_i - x_j) of row i, and dl+ - dl- (the caller counts the
// loss for i < j only: each undirected edge has two entries, each updating its own row).
// ------------------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ float edge_entry(const XView &xv, int i, int j, float (&dg)[D], const PairParams &P,
                                            const float4 *tab) {
    float xi[D], xj[D], diff[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xi[k] = k < xv.d ? xv.at(i, k) : 0.0f;
        xj[k] = k < xv.d ? xv.at(j, k) : 0.0f;
    }
    float r2 = sqdist_eps<D>(xi, xj, diff);
    float dlp, ccp, dln, ccn, wn;
    pair_eval(r2, -1.0f, P, dlp, ccp);
    nonedge<false, true>(r2, P, tab, table_offset(P, kLtabZero), dln, ccn, wn);
    const float dcc = ccp - ccn;
#pragma unroll
    for (int k = 0; k < D; ++k) dg[k] = dcc * diff[k];
    return dlp - dln;
}

constexpr int kEdgeBlock = 256;

template <int EX>
__global__ __launch_bounds__(kEdgeBlock) void k_edges(const float *__restrict__ X, int d,
                                                      const int32_t *__restrict__ coo_row,
                                                      const int32_t *__restrict__ col, long long nnz,
                                                      const unsigned long long *__restrict__ table,
                                                      unsigned long long cap, float *__restrict__ G,
                                                      float *__restrict__ rowloss,
                                                      float *__restrict__ partials,
                                                      unsigned long long *hits, PairParams P,
                                                      int strip_rows, int nt, int shard, int nshards) {
    __shared__ float wsum[kEdgeBlock / 64];
    __shared__ unsigned whit[kEdgeBlock / 64];
    __shared__ float4 ltab[kLtabF4];
    stage_ltab(ltab);
    __syncthreads();
    long long e = (long long)blockIdx.x * kEdgeBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float dloss = 0.0f, ddl = 0.0f, dcc = 0.0f, dw = 0.0f;
    unsigned hit = 0;
    int i = -1, j = 0;
    if (e < nnz) {
        i = coo_row[e];
        j = col[e];
        const float *xi = X + (size_t)i * d;
        const float *xj = X + (size_t)j * d;
        float r2 = 1.17549435e-38f;  // from FLT_MIN, as the sweeps' sqdist_eps
        for (int k = 0; k < d; ++k) {
            float df = xi[k] - xj[k];
            r2 = __builtin_fmaf(df, df, r2);
        }
        float dlp, ccp, dln, ccn, wp = 0.0f, wn = 0.0f;
        pair_eval_t<EX == kExZ>(r2, -1.0f, P, dlp, ccp, wp);
        nonedge<EX == kExZ>(r2, P, ltab, table_offset(P, kLtabZero), dln, ccn, wn);
        // a shard corrects only the edges of its own tiles (the entry keeps its row key, so
        // the row runs stay contiguous, and adds nothing)
        const bool own = nshards <= 1 || strip_owned(min(i, j) / strip_rows, nt, shard, nshards);
        dcc = own ? ccp - ccn : 0.0f;
        ddl = own ? dlp - dln : 0.0f;
        dw = own ? wp - wn : 0.0f;
        if (i < j && own) {
            dloss = ddl;
            hit = hits && gempe_hash_contains(table, cap, gempe_edge_key(i, j)) ? 1u : 0u;
        }
    }
    // row sums of the gradient change (and of the row loss), one atomic per row run
    for (int k = 0; k < d; ++k) {
        float v = (i >= 0) ? dcc * (X[(size_t)i * d + k] - X[(size_t)j * d + k]) : 0.0f;
        if (seg_sum_to_head(i, lane, v)) atomicAdd(&G[(size_t)i * d + k], v);
    }
    if (EX) {
        float v = (EX == kExZ) ? dw : ddl;
        if (seg_sum_to_head(i, lane, v)) atomicAdd(&rowloss[i], v);
    }
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

// Exact edge correction for wide embeddings (d > 16): one wave per CSR row i, split into
// four groups of 16 lanes that take four of the row's entries at a time (lane s of a group
// holds coordinates s, s+16, ... of x_i and of its gradient change), so four x_j rows are in
// flight per wave and the pair function runs once per entry per group.  The row's column
// indices are loaded once per 64 entries, one per lane.  The squared distance is
// group16_sqdist, the one the BF16 path's exact near-pair pass uses.  At the end the four
// groups' gradient changes are summed (fixed order) and added with one atomic per
// coordinate.  `hits` (membership of each pair i<j in the edge hash, a consistency check) is
// counted only when the caller asks for it.
template <int D, int EX>
__global__ __launch_bounds__(256) void k_edges_rows(const float *__restrict__ X, int n, int d,
                                                    const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const unsigned long long *__restrict__ table,
                                                    unsigned long long cap, float *__restrict__ G,
                                                    float *__restrict__ rowloss, float *__restrict__ partials,
                                                    unsigned long long *hits, PairParams P, int strip_rows,
                                                    int nt, int shard, int nshards) {
    constexpr int C = D / 16;
    __shared__ float wsum[4];
    __shared__ unsigned whit[4];
    // d = 16 (the BF16 path) takes the non-edge value from the table, as its near-pair and
    // dense passes do
    __shared__ float4 ltab[D == 16 ? kLtabF4 : 1];
    if (D == 16) {
        stage_ltab(ltab);
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, sub = lane & 15;
    const int i = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wave);
    float dloss = 0.0f, lrow = 0.0f;
    unsigned hitc = 0;
    if (i < n) {
        const float *xi = X + (size_t)i * d;
        float xr[C], g[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int c = sub + 16 * k;
            xr[k] = c < d ? xi[c] : 0.0f;
            g[k] = 0.0f;
        }
        const long long e0 = row_ptr[i], e1 = row_ptr[i + 1];
        for (long long base = e0; base < e1; base += 64) {
            const int cnt = (int)min(64LL, e1 - base);
            const int jl = lane < cnt ? col[base + lane] : i;
            for (int c0 = 0; c0 < cnt; c0 += 4) {
                const int k = c0 + grp;
                const int j = __shfl(jl, k & 63, 64);
                // a shard corrects only the edges of its own tiles
                const bool valid =
                    k < cnt && (nshards <= 1 || strip_owned(min(i, j) / strip_rows, nt, shard, nshards));
                float df[C];
                const float r2 = group16_sqdist<C>(xr, X + (size_t)(valid ? j : i) * d, sub, d, df);
                float dlp, ccp, dln, ccn, wp = 0.0f, wn = 0.0f;
                pair_eval_t<EX == kExZ>(r2, -1.0f, P, dlp, ccp, wp);
                if (D == 16)
                    nonedge<EX == kExZ>(r2 + kFltMin, P, ltab, table_offset(P, kLtabZero), dln, ccn, wn);
                else
                    pair_eval_t<EX == kExZ>(r2, 1.0f, P, dln, ccn, wn);
                const float dcc = valid ? ccp - ccn : 0.0f;
#pragma unroll
                for (int q = 0; q < C; ++q) g[q] = __builtin_fmaf(dcc, df[q], g[q]);
                if (valid && sub == 0) {
                    const float ddl = dlp - dln;
                    if (EX) lrow += (EX == kExZ) ? wp - wn : ddl;
                    if (i < j) {
                        dloss += ddl;
                        if (hits && gempe_hash_contains(table, cap, gempe_edge_key(i, j))) ++hitc;
                    }
                }
            }
        }
        // groups 0 + 1 + 2 + 3 in that order, then one atomic per coordinate
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const float a01 = g[q] + __shfl_xor(g[q], 16, 64);
            g[q] = a01 + __shfl_xor(a01, 32, 64);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int c = sub + 16 * q;
            if ((q & 3) == grp && c < d) atomicAdd(&G[(size_t)i * d + c], g[q]);
        }
    }
    dloss = wave_sum(dloss);
    if (EX) {
        lrow = wave_sum(lrow);
        if (i < n && lane == 0) atomicAdd(&rowloss[i], lrow);
    }
    if (hits) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) hitc += __shfl_xor(hitc, off, 64);
    }
    if (lane == 0) {
        wsum[wave] = dloss;
        whit[wave] = hitc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        unsigned h = whit[0] + whit[1] + whit[2] + whit[3];
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

// Sum of partials[0..count) in FP64: thread t adds slots t, t+256, ... in order, then a
// fixed tree over the 256 threads.  Called by a whole 256-thread workgroup.
__device__ inline double block_sum_fixed(const float *__restrict__ partials, long long count,
                                         double *sh) {
    double acc = 0.0;
    for (long long q = threadIdx.x; q < count; q += kFinBlock) acc += (double)partials[q];
    __syncthreads();
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kFinBlock / 2; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

// Two-level FP64 sum of the loss partials, deterministic: the partials are the
// concatenation p1[0..m1) ++ p2[0..n2), m1 = *n1_dev when given (a device-side count) else
// n1; block b of the first level sums the fixed slot range [b chunk, (b + 1) chunk).
__global__ __launch_bounds__(kFinBlock) void k_reduce1(const float *__restrict__ p1, long long n1,
                                                       const int *__restrict__ n1_dev,
                                                       const float *__restrict__ p2, long long n2,
                                                       long long chunk, double *__restrict__ out) {
    __shared__ double sh[kFinBlock];
    const long long m1 = n1_dev ? (long long)*n1_dev : n1;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = std::min(lo + chunk, m1 + n2);
    double acc = 0.0;
    for (long long q = lo + threadIdx.x; q < hi; q += kFinBlock)
        acc += (double)(q < m1 ? p1[q] : p2[q - m1]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kFinBlock / 2; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kFinBlock) void k_finalize(const double *__restrict__ part, int nb, double *loss,
                                                        const unsigned long long *hits, int64_t *hits_out,
                                                        unsigned *status) {
    __shared__ double sh[kFinBlock];
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += kFinBlock) acc += part[q];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kFinBlock / 2; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *loss = sh[0];
        if (hits_out) *hits_out = (int64_t)*hits;
        if (!isfinite(sh[0])) atomicOr(status, kStatusNonFinite);
    }
}

// Weighted-majorization update (Eq. 5): x_i <- y_i / z_i, which equals x_i - g_i / (2 z_i)
// because y_i = z_i x_i - g_i / 2 (the parabola's slope matches dl' at the current distance).
// A vertex whose z_i is not positive (every w_ij underflowed, or non-finite input) stays.
__global__ void k_wm_update(float *__restrict__ X, const float *__restrict__ G, const float *__restrict__ Z,
                            int d, long long count) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const float z = Z[k / d];
    const float s = (z > 0.0f) ? 0.5f / z : 0.0f;
    X[k] = __builtin_fmaf(-G[k], s, X[k]);
}

__global__ void k_axpy(float *__restrict__ X, const float *__restrict__ G, float eta, long long count) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) X[k] = __builtin_fmaf(-eta, G[k], X[k]);
}

// ------------------------------------------------------------------------------------
// Gradient descent for d <= 16 and small n: one fused launch per iteration.
//
// Iteration k reads X_{k-1} (iterate slot (k-1)&1) and G_{k-1} (gradient slot (k-1)%3)
// and applies the previous step on the fly, x_k = X_{k-1} - eta G_{k-1}.  It accumulates
// G_k into slot k%3, writes x_k into slot k&1 for iteration k+1, clears slot (k+1)%3 (the
// slot of G_{k-2}, last read by iteration k-1), and writes one FP32 loss partial per work
// unit into partial slot k&1; one extra workgroup after the units sums the partials
// of iteration k-1 in FP64.
// A workgroup takes one 64 x 64 tile, its four waves a quarter of the 64-step schedule
// each (one per SIMD), and combines their row and column partials in LDS before one
// global flush; edge workgroups take 4 x 64 CSR entries.  The hardware dispatcher
// balances the workgroups over the CUs.  The kernel boundary is the only global
// synchronisation.  (LDS float atomics serialise badly when four waves hit the same
// lines; the waves therefore write private LDS partials that wave 0 sums in order.)
// ------------------------------------------------------------------------------------
struct IterArgs {
    float *Xc;          // caller coordinates: iterate slot 0, and the final result
    float *Xw;          // workspace iterate slot 1
    float *G0;          // three gradient slots of n*d floats each
    float *P0;          // two partial slots of `units` floats each
    double *loss_hist;  // one entry per sweep, or nullptr
    unsigned *status;
    const int32_t *coo_row;
    const int32_t *col;
    long long nnz;
    int n, d, nb, epu;  // nb: 64-vertex blocks per side; epu: CSR entries per edge wave
    long long units_edge, units;  // workgroups: [0, units_edge) edge work, then one per tile
    float neg_eta;
    PairParams P;
};

// The FP64 loss of iteration k's sweep: stored when a history is kept, and checked for
// being finite in every case (the status word then reports a diverged run).
__device__ inline void reduce_loss(const IterArgs &a, int k, double *sh) {
    double tot = block_sum_fixed(a.P0 + (size_t)(k & 1) * a.units, a.units, sh);
    if (threadIdx.x == 0) {
        if (a.loss_hist) a.loss_hist[k] = tot;
        if (!isfinite(tot)) atomicOr(a.status, kStatusNonFinite);
    }
}

// LDS of one fused-iteration workgroup.
template <int D>
struct IterLds {
    double sh[kFinBlock];
    float rowp[4][64 * D];  // per-wave partials: plain LDS stores, summed in wave order
    float colp[4][64 * D];
    float wl[4];
    float4 tab[2 * kLtabF4];  // two-float4 table form
};

// Iteration k of one gradient-descent run, executed by workgroup b of the run's
// `nthreads / 256` workgroups (gtid: this thread's index among them).
template <int D>
__device__ __forceinline__ void iter_body(const IterArgs &a, int k, int b, long long gtid, long long nthreads,
                                          IterLds<D> &L) {
    double *sh = L.sh;
    auto &rowp = L.rowp;
    auto &colp = L.colp;
    float *wl = L.wl;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long nd = (long long)a.n * a.d;
    // iterate slots by selection, not through an indexed array of pointers (which would
    // turn every coordinate access into a flat access)
    float *Xcur = (k & 1) ? a.Xw : a.Xc;
    const float *Xprev = (k == 0 || !((k - 1) & 1)) ? a.Xc : a.Xw;
    const float *Gprev = (k == 0) ? nullptr : a.G0 + (size_t)((k - 1) % 3) * nd;
    float *Gk = a.G0 + (size_t)(k % 3) * nd;
    float *Gnext = a.G0 + (size_t)((k + 1) % 3) * nd;
    float *Pk = a.P0 + (size_t)(k & 1) * a.units;
    const XView xv{Xprev, Gprev, a.neg_eta, a.d};

    // x_k = x_{k-1} - eta g_{k-1} stored for the caller and the next slot of gradients
    // cleared (nothing in this launch reads either; done last, behind the sweep, this
    // measured 2 us slower per launch)
    for (long long v = gtid; v < nd; v += nthreads) {
        if (k > 0) Xcur[v] = __builtin_fmaf(a.neg_eta, Gprev[v], Xprev[v]);
        Gnext[v] = 0.0f;
    }
    if (b >= a.units) {  // uniform over the workgroup
        // the last workgroup sums iteration k-1's loss partials, beside the tiles rather
        // than before one of them
        if (b == a.units && k > 0) reduce_loss(a, k - 1, sh);
        return;
    }
    // the table's loads and a tile workgroup's operand loads are all issued before the
    // first of them is waited for, so their latencies overlap
    float4 tabc[kLtab2Per];
    ltab2_load(tabc);
    const bool tile = b >= a.units_edge;  // uniform over the workgroup
    const int dir = rot_dir(lane);
    const int t = a.P.reverse ? (int)(a.units - 1 - b) : b - (int)a.units_edge;
    int I = 0, J = 0;
    if (tile) tile_of(t, a.nb, I, J);
    const int i = I * 64 + lane;
    const int col0 = J * 64;
    const int s0 = wave * 16;
    const int jc = col0 + ((lane + dir * s0) & 63);
    // every load at a clamped in-range index, all issued before the first is used
    float xi[1][D], xc[D];
    {
        const size_t oi = (size_t)min(i, a.n - 1) * a.d, oj = (size_t)min(jc, a.n - 1) * a.d;
        float gi0[D], gc0[D];
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int qq = min(q, a.d - 1);
            xi[0][q] = Xprev[oi + qq];
            xc[q] = Xprev[oj + qq];
            gi0[q] = Gprev ? Gprev[oi + qq] : 0.0f;
            gc0[q] = Gprev ? Gprev[oj + qq] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const bool qd = tile && q < a.d;
            xi[0][q] = (qd && i < a.n) ? __builtin_fmaf(a.neg_eta, gi0[q], xi[0][q]) : 0.0f;
            xc[q] = (qd && jc < a.n) ? __builtin_fmaf(a.neg_eta, gc0[q], xc[q]) : 0.0f;
        }
    }
    ltab2_store(L.tab, tabc, a.P.slope_k);
    __syncthreads();
    float loss = 0.0f;
    int slot = b;
    if (!tile) {
        // edge workgroups come first: their dependent gathers overlap the tiles
        const long long e0 = ((long long)b * 4 + wave) * a.epu;
        for (int q = 0; q < a.epu; q += 64) {
            const long long e = e0 + q + lane;
            int i = -1;
            float dg[D];
#pragma unroll
            for (int k2 = 0; k2 < D; ++k2) dg[k2] = 0.0f;
            if (e < a.nnz) {
                i = a.coo_row[e];
                const int j = a.col[e];
                const float ddl = edge_entry<D>(xv, i, j, dg, a.P, L.tab);
                if (i < j) loss += ddl;
            }
#pragma unroll
            for (int k2 = 0; k2 < D; ++k2) {
                if (k2 < a.d) {
                    float v = dg[k2];
                    if (seg_sum_to_head(i, lane, v)) atomicAdd(&Gk[(size_t)i * a.d + k2], v);
                }
            }
        }
    } else {
        // one 64 x 64 tile per workgroup; wave w runs steps [16 w, 16 w + 16) of the
        // schedule, the four waves' row and column partials meet in LDS
        slot = (int)a.units_edge + t;  // the loss partial of tile t, whichever workgroup runs it
        float gi[1][D], li[1], colacc[D];
        int irow[1] = {i};
#pragma unroll
        for (int q = 0; q < D; ++q) {
            gi[0][q] = 0.0f;
            colacc[q] = 0.0f;
        }
        li[0] = 0.0f;
        const bool msk = (I == J) || (col0 + 64 > a.n);
        if (a.P.table_full) {
            if (msk)
                sweep_steps<D, 1, true, false, true, false>(xi, irow, xc, colacc, gi, li, loss, lane, dir, col0,
                                                            a.n, s0, s0 + 16, a.P, L.tab);
            else
                sweep_steps<D, 1, false, false, true, false>(xi, irow, xc, colacc, gi, li, loss, lane, dir, col0,
                                                             a.n, s0, s0 + 16, a.P, L.tab);
        } else {
            if (msk)
                sweep_steps<D, 1, true, false, true>(xi, irow, xc, colacc, gi, li, loss, lane, dir, col0, a.n,
                                                     s0, s0 + 16, a.P, L.tab);
            else
                sweep_steps<D, 1, false, false, true>(xi, irow, xc, colacc, gi, li, loss, lane, dir, col0, a.n,
                                                      s0, s0 + 16, a.P, L.tab);
        }
        const int cl = (lane + dir * (s0 + 15)) & 63;  // column whose partial this lane holds
#pragma unroll
        for (int q = 0; q < D; ++q) {
            rowp[wave][lane * D + q] = gi[0][q];
            colp[wave][cl * D + q] = colacc[q];
        }
        __syncthreads();
        if (wave == 0) {
            const int jr = col0 + lane;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                if (q < a.d) {
                    const float rs = (rowp[0][lane * D + q] + rowp[1][lane * D + q]) +
                                     (rowp[2][lane * D + q] + rowp[3][lane * D + q]);
                    const float cs = (colp[0][lane * D + q] + colp[1][lane * D + q]) +
                                     (colp[2][lane * D + q] + colp[3][lane * D + q]);
                    if (i < a.n) atomicAdd(&Gk[(size_t)i * a.d + q], rs);
                    if (jr < a.n) atomicAdd(&Gk[(size_t)jr * a.d + q], -cs);
                }
            }
        }
    }
    loss = wave_sum(loss);
    if (lane == 0) wl[wave] = loss;
    __syncthreads();
    if (threadIdx.x == 0) Pk[slot] = (wl[0] + wl[1]) + (wl[2] + wl[3]);
}

template <int D>
__global__ __launch_bounds__(256) void k_iter(IterArgs a, int k) {
    __shared__ IterLds<D> lds;
    iter_body<D>(a, k, (int)blockIdx.x, (long long)blockIdx.x * blockDim.x + threadIdx.x,
                 (long long)gridDim.x * blockDim.x, lds);
}

// After K sweeps: the FP64 loss of the last sweep, and the final coordinates into the
// caller's buffer (the last step applied now when no loss of the final iterate was asked).
__device__ __forceinline__ void finish_body(const IterArgs &a, int K, int iters, int b, long long gtid,
                                            long long nthreads, double *sh) {
    const long long nd = (long long)a.n * a.d;
    if (b == 0 && K > 0) reduce_loss(a, K - 1, sh);
    if (iters <= 0) return;
    if (K == iters + 1) {  // x_iters was written to slot iters&1 by the last sweep
        if (iters & 1)
            for (long long v = gtid; v < nd; v += nthreads) a.Xc[v] = a.Xw[v];
    } else {
        const float *Xl = (iters - 1) & 1 ? a.Xw : a.Xc;
        const float *Gl = a.G0 + (size_t)((iters - 1) % 3) * nd;
        for (long long v = gtid; v < nd; v += nthreads) a.Xc[v] = __builtin_fmaf(a.neg_eta, Gl[v], Xl[v]);
    }
}

__global__ __launch_bounds__(256) void k_iter_finish(IterArgs a, int K, int iters) {
    __shared__ double sh[kFinBlock];
    finish_body(a, K, iters, (int)blockIdx.x, (long long)blockIdx.x * blockDim.x + threadIdx.x,
                (long long)gridDim.x * blockDim.x, sh);
}

// ------------------------------------------------------------------------------------
// Continuous batching: many independent gradient-descent runs (jobs) advance by one
// iteration per launch ("tick").  Job q owns workgroups [u0, u0 + blocks) of the tick;
// its iteration index is k = tick - k0.  For k < K the workgroups run iteration k exactly
// as k_iter does for a single run (same per-tile partials and reduction order); at k = K
// they run the finishing step (loss of the last sweep, final coordinates).  Jobs share
// nothing but the launch, so a job's result does not depend on its companions.
// ------------------------------------------------------------------------------------
struct BatchEntry {
    IterArgs a;
    long long u0;      // first workgroup of this job in the tick
    long long blocks;  // workgroups of this job (its units)
    int k0;            // tick of the job's iteration 0
    int K;             // sweeps (iters, +1 when the loss of the final iterate is kept)
    int iters;
    int pad;
};

template <int D>
__global__ __launch_bounds__(256) void k_iter_batch(const BatchEntry *__restrict__ tab, int njobs, int tick) {
    __shared__ IterLds<D> lds;
    const long long b = blockIdx.x;
    // the job whose workgroup range holds b (entries ordered by u0)
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].u0 <= b) lo = mid; else hi = mid - 1;
    }
    const BatchEntry &e = tab[lo];
    const long long lb = b - e.u0;
    if (lb >= e.blocks) return;  // uniform over the workgroup (cannot happen for a dense table)
    const int k = tick - e.k0;
    const long long gtid = lb * blockDim.x + threadIdx.x;
    const long long nthreads = e.blocks * blockDim.x;
    if (k >= 0 && k < e.K)
        iter_body<D>(e.a, k, (int)lb, gtid, nthreads, lds);
    else if (k == e.K)
        finish_body(e.a, e.K, e.iters, (int)lb, gtid, nthreads, lds.sh);
}

}  // namespace gempe

// ======================================================================================
// Host side: plan, workspace layout, launches.
// ======================================================================================
using namespace gempe;

namespace {
PairParams dev_params(const PairParamsHost &h) {
    return PairParams{h.mu_s,   h.inv_sigma, h.c_neg,   h.c_pos,   h.tk_scale,
                      h.tk_off, h.slope_k,   h.r_scale, h.w_scale, h.wk2, h.table_full, h.reverse};
}
}  // namespace

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

constexpr long long kPersistMaxTiles = 65536;  // 64x64 tiles: n up to ~23k
constexpr int kMfmaMinN = 8192;                 // d = 16 sweeps on the matrix cores from this n on
constexpr int kMfmaWideMinN = 4096;             // d = 32, 64, 128 likewise
constexpr int kEdgesPerUnit = 64;
constexpr int kRed1Blocks = 1024;  // first level of the FP64 loss reduction  // CSR entries per edge wave: one per lane

}  // namespace

long long gempe_shard_items(int nt, int s, int G) {
    if (G <= 1) return (long long)nt * (nt + 1) / 2;
    long long c = 0;
    for (int p = s; p <= nt - 1 - p; p += G) c += (p == nt - 1 - p) ? (long long)(nt - p) : (long long)nt + 1;
    return c;
}

SweepPlan gempe_make_plan(const gempe_graph_s *g, int d, bool bf16) {
    SweepPlan p;
    if (bf16) {
        // screen on 128x128 tiles, exact FP32 pass over flagged 64x64 tiles (LDS kernel)
        p.bf16 = true;
        p.D = d <= 16 ? 16 : d <= 32 ? 32 : d <= 64 ? 64 : 128;
        p.R = 1;
        p.W = 1;
        p.T = 64;
        p.nt = (g->n + 63) / 64;
        p.items = (long long)p.nt * (p.nt + 1) / 2;
        p.grid = std::min<long long>(p.items, 2048);
        p.edge_blocks = (int)std::max<long long>(1, ((long long)g->n + 3) / 4);  // one wave per row
        p.partials = p.items + p.edge_blocks;
        // d = 16, 32, 64, 128: an evaluation whose screen flags most tiles (d = 16 from a
        // spread start, any d from a contracted one: nearly every pair within the near
        // distance) runs the full matrix-core sweep instead of the list
        if ((d == 16 && g->n >= kMfmaMinN) || ((d == 32 || d == 64 || d == 128) && g->n >= kMfmaWideMinN)) {
            for (int chunk : {32, 16, 8}) {
                const long long it = gempe_mfma_items(g->n, chunk);
                const long long grid = (it + kXcd - 1) / kXcd * kXcd;
                if ((it >= 16384 || chunk == 8) && grid * 256 < (1LL << 32) && 2 * it <= p.items) {
                    p.mfma_chunk = chunk;
                    p.mfma_items = it;
                    p.mfma_grid = grid;
                    break;
                }
            }
        }
        return p;
    }
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
    p.edge_blocks = p.D > 16 ? (int)std::max<long long>(1, ((long long)g->n + 3) / 4)
                             : (int)std::max<long long>(1, (g->nnz + kEdgeBlock - 1) / kEdgeBlock);
    p.partials = p.items + p.edge_blocks;

    // d = 16 (and 32, 64, 128) on the matrix cores for large n (loss and gradient without
    // per-vertex extras):
    // the longest chunks of column blocks per item (less staging and flushing per pair; 32
    // measured as fast as 64 or 128 on the 1M-vertex graph) that still give 16,384 items
    if ((d == 16 && g->n >= kMfmaMinN) || ((d == 32 || d == 64 || d == 128) && g->n >= kMfmaWideMinN)) {
        for (int chunk : {32, 16, 8}) {
            const long long it = gempe_mfma_items(g->n, chunk);
            const long long grid = (it + kXcd - 1) / kXcd * kXcd;
            if ((it >= 16384 || chunk == 8) && grid * 256 < (1LL << 32)) {
                p.mfma = true;
                p.mfma_chunk = chunk;
                p.mfma_items = it;
                p.mfma_grid = grid;
                p.partials = std::max(p.items, it) + p.edge_blocks;
                break;
            }
        }
    }

    // fused-iteration plan: one workgroup per 64x64 tile, edge workgroups first
    p.persist = false;
    const long long t64 = tiles_for(g->n, 64);
    if (p.D <= 16 && t64 <= kPersistMaxTiles) {
        p.persist = true;
        p.nb64 = (g->n + 63) / 64;
        p.tiles64 = t64;
        p.units_edge = (g->nnz + 4 * kEdgesPerUnit - 1) / (4 * kEdgesPerUnit);
        p.units_sweep = t64;
        p.units = p.units_sweep + p.units_edge;
        p.iter_blocks = p.units + 1;
    }
    return p;
}

gempe_status gempe_check_plan(const SweepPlan &p, const char *who) {
    if (p.bf16) return GEMPE_OK;  // its launches are bounded by the n limit of BF16_GRAM
    // the FP32 sweeps launch one workgroup of 64 W threads per tile; HIP bounds a launch to
    // fewer than 2^32 work-items
    const long long threads = p.grid * 64LL * p.W;
    if (p.grid >= (1LL << 31) || threads >= (1LL << 32))
        return gempe_fail(GEMPE_ERR_UNSUPPORTED,
                          std::string(who) + ": n too large for one FP32 sweep launch at this d (" +
                              std::to_string(p.items) + " tiles of " + std::to_string(p.T) +
                              " rows; the limit is about n = 741,000 for d > 16, 2,960,000 for 5 <= d <= 16 and "
                              "5,930,000 for d <= 4)");
    return GEMPE_OK;
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
    L.zbuf = off;
    off = align256(off + sizeof(float) * (size_t)g->n);
    L.xbuf = off;
    off = align256(off + sizeof(float) * nd);
    L.gring = off;
    off = align256(off + sizeof(float) * 3 * nd);
    L.ppart = off;
    off = align256(off + sizeof(float) * 2 * (size_t)std::max<long long>(plan.units, 1));
    L.red = off;
    off = align256(off + sizeof(double) * kRed1Blocks);
    if (plan.bf16) {
        L.xb = off;
        off = align256(off + 2 * nd);
        L.nrm = off;
        off = align256(off + sizeof(float) * (size_t)g->n);
        L.snorm = off;
        off = align256(off + sizeof(float) * (size_t)g->n);
        L.smax128 = off;
        off = align256(off + sizeof(float) * (size_t)((g->n + 127) / 128));
        L.flags = off;
        off = align256(off + (size_t)plan.items);
        L.list = off;
        off = align256(off + sizeof(int) * (size_t)plan.items);
        L.dense = off;
        off = align256(off + (size_t)plan.items);
        L.chunks = off;
        off = align256(off + sizeof(int) * (size_t)(plan.items / 4096 + 1));
    }
    L.total = off;
    return L;
}

WsLayout gempe_ws_layout_eval(const gempe_graph_s *g, int d, const SweepPlan &plan) {
    (void)g;
    (void)d;
    WsLayout L;
    size_t off = 0;
    L.counters = off;
    off += 256;
    L.partials = off;
    off = align256(off + sizeof(float) * (size_t)plan.partials);
    L.red = off;
    off = align256(off + sizeof(double) * kRed1Blocks);
    L.total = off;
    return L;
}

GramCtx gempe_gram_ctx(const WsLayout &L, unsigned char *ws, const gempe_params *p) {
    GramCtx c;
    if (!L.xb) return c;
    c.xb = ws + L.xb;
    c.nrm = reinterpret_cast<float *>(ws + L.nrm);
    c.snorm = reinterpret_cast<float *>(ws + L.snorm);
    c.smax128 = reinterpret_cast<float *>(ws + L.smax128);
    c.flags = ws + L.flags;
    c.list = reinterpret_cast<int *>(ws + L.list);
    c.count = reinterpret_cast<int *>(ws + L.counters + 32);
    c.dense = ws + L.dense;
    c.chunks = reinterpret_cast<int *>(ws + L.chunks);
    c.all_dense = reinterpret_cast<int *>(ws + L.counters + 36);
    c.sample = reinterpret_cast<int *>(ws + L.counters + 40);
    c.theta0 = (float)(p->mu + p->near_k * p->sigma);
    return c;
}

PairParamsHost gempe_pair_params(const gempe_params *p) {
    PairParamsHost h;
    const double d1s = -1.0 / (p->sigma * 0.69314718055994530942);  // -1 / (sigma ln 2)
    h.mu_s = (float)(p->mu / p->sigma);
    h.inv_sigma = (float)(1.0 / p->sigma);
    h.c_neg = (float)(0.39894228040143267794 * d1s);  // sqrt(2/pi)/2
    h.c_pos = (float)(0.39894228040143267794 * d1s);  // 1/sqrt(2 pi)
    h.tk_scale = (float)(GEMPE_LTAB_INV_H / p->sigma);
    h.tk_off = (float)(-GEMPE_LTAB_INV_H * p->mu / p->sigma);
    h.slope_k = (float)(GEMPE_LTAB_INV_H * 0.69314718055994530942 / p->sigma);
    h.r_scale = (float)(-p->sigma * 0.69314718055994530942);
    h.w_scale = (float)(1.0 / (2.0 * p->sigma * p->sigma * 0.69314718055994530942));
    h.wk2 = (float)(-1.0 / (32.0 * p->sigma));
    // A non-edge has tau = (delta - mu) / sigma >= -mu / sigma; its table index
    // 16 tau - 16 GEMPE_LTAB_LO is then at least 1 when 16 mu / sigma <= 16 (-LO) - 1, a
    // margin of one segment over the FP32 rounding of the index arithmetic.
    h.table_full = (GEMPE_LTAB_INV_H * p->mu / p->sigma <= -GEMPE_LTAB_LO * GEMPE_LTAB_INV_H - 1.0) ? 1 : 0;
    h.reverse = (p->flags & GEMPE_F_REVERSE_TILES) ? 1 : 0;
    return h;
}

namespace {

template <int D, int R, int W, int EX>
void launch_small(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                  float *part, PairParams P) {
    long long per = pl.grid / kXcd;
    hipLaunchKernelGGL((k_sweep_small<D, R, W, EX>), dim3((unsigned)pl.grid), dim3(64 * W), 0, s, X, n, d,
                       pl.nt, pl.items, per, G, rl, part, P, pl.shard, pl.nshards);
}

template <int D, int EX>
void launch_small_rw(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                     float *part, PairParams P) {
    if (pl.R == 1 && pl.W == 1) return launch_small<D, 1, 1, EX>(pl, s, X, n, d, G, rl, part, P);
    if (pl.R == 1 && pl.W == 2) return launch_small<D, 1, 2, EX>(pl, s, X, n, d, G, rl, part, P);
    if (pl.R == 1 && pl.W == 4) return launch_small<D, 1, 4, EX>(pl, s, X, n, d, G, rl, part, P);
    if (pl.R == 2 && pl.W == 4) return launch_small<D, 2, 4, EX>(pl, s, X, n, d, G, rl, part, P);
    if constexpr (D <= 4) {
        if (pl.R == 4 && pl.W == 4) return launch_small<D, 4, 4, EX>(pl, s, X, n, d, G, rl, part, P);
    }
}

template <int D, int EX>
void launch_wide(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                 float *part, PairParams P) {
    long long per = pl.grid / kXcd;
    size_t lds = sizeof(float) * 4 * 64 * (D + 1);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sweep_wide<D, EX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sweep_wide<D, EX>), dim3((unsigned)pl.grid), dim3(64), lds, s, X, n, d, pl.nt,
                       pl.items, per, G, rl, part, P, pl.shard, pl.nshards);
}

template <int D, int EX>
void launch_wide_list(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, const GramCtx &gc,
                      float *G, float *rl, float *part, PairParams P) {
    size_t lds = sizeof(float) * 4 * 64 * (D + 1);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sweep_wide_list<D, EX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sweep_wide_list<D, EX>), dim3((unsigned)pl.grid), dim3(64), lds, s, X, n, d, pl.nt,
                       gc.list, gc.count, G, rl, part, P, gc.theta0 * gc.theta0, gc.dense, gc.all_dense);
}

template <int EX>
void launch_list(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, const GramCtx &gc, float *G,
                 float *rl, float *part, PairParams P) {
    switch (pl.D) {
        case 16: return launch_wide_list<16, EX>(pl, s, X, n, d, gc, G, rl, part, P);
        case 32: return launch_wide_list<32, EX>(pl, s, X, n, d, gc, G, rl, part, P);
        case 64: return launch_wide_list<64, EX>(pl, s, X, n, d, gc, G, rl, part, P);
        default: return launch_wide_list<128, EX>(pl, s, X, n, d, gc, G, rl, part, P);
    }
}

template <int EX>
void launch_sweep(const SweepPlan &pl, hipStream_t s, const float *X, int n, int d, float *G, float *rl,
                  float *part, PairParams P) {
    switch (pl.D) {
        case 1: return launch_small_rw<1, EX>(pl, s, X, n, d, G, rl, part, P);
        case 2: return launch_small_rw<2, EX>(pl, s, X, n, d, G, rl, part, P);
        case 3: return launch_small_rw<3, EX>(pl, s, X, n, d, G, rl, part, P);
        case 4: return launch_small_rw<4, EX>(pl, s, X, n, d, G, rl, part, P);
        case 8: return launch_small_rw<8, EX>(pl, s, X, n, d, G, rl, part, P);
        case 16: return launch_small_rw<16, EX>(pl, s, X, n, d, G, rl, part, P);
        case 32: return launch_wide<32, EX>(pl, s, X, n, d, G, rl, part, P);
        case 64: return launch_wide<64, EX>(pl, s, X, n, d, G, rl, part, P);
        default: return launch_wide<128, EX>(pl, s, X, n, d, G, rl, part, P);
    }
}

template <int D>
void launch_iters(const SweepPlan &pl, IterArgs &a, int K, int iters, hipStream_t s) {
    const unsigned grid = (unsigned)pl.iter_blocks;
    {
        TimedLaunches tl(kTkSweep, s, K);
        for (int k = 0; k < K; ++k) hipLaunchKernelGGL(k_iter<D>, dim3(grid), dim3(256), 0, s, a, k);
    }
    const long long nd = (long long)a.n * a.d;
    const unsigned fgrid = (unsigned)std::min<long long>(1024, std::max<long long>(1, (nd + 255) / 256));
    hipLaunchKernelGGL(k_iter_finish, dim3(fgrid), dim3(256), 0, s, a, K, iters);
}

}  // namespace

namespace {
// The BF16 path's route sample: at d = 16 the screen costs a tenth of the FP32 sweep it would
// spare, so a plain evaluation that may take the full matrix-core route screens a sample of
// its tiles first and skips the screen when most of the sample is flagged (the full sweep is
// exact for every pair, so only the time depends on the sample).  At d >= 32 the screen is
// under 2 % of that sweep and always runs.
bool route_sample(const SweepPlan &plan, int d, bool plain, const PairParamsHost &pph) {
    return plan.bf16 && plain && pph.table_full && plan.mfma_items > 0 && d == 16;
}

// The sweep (or BF16 screen + exact list pass) and the exact edge correction, with the
// per-vertex extra sum EX into `extra` (row loss or the weighted-majorization z).
template <int EX>
void launch_pass(const gempe_graph_s *g, int d, const SweepPlan &plan, const float *X, float *grad, float *extra,
                 float *partials, unsigned long long *hits, const PairParams &P, const PairParamsHost &pph,
                 hipStream_t s, const GramCtx &gc) {
    const int n = g->n;
    if (plan.bf16) {
        // The sparse pass evaluates the near pairs of sparsely flagged tiles exactly and marks
        // the dense ones.  At d = 16 the dense tiles of a plain evaluation go to the matrix
        // cores (FP32 Gram, the exact path for near pairs).  When most tiles are flagged, a
        // plain evaluation at d = 16 from n = 8,192 on, or at d = 32, 64, 128 from n = 4,096
        // on, leaves every pair to the full matrix-core sweep instead (chunk-major; at d = 16
        // four waves per SIMD against the list kernel's three) and the list kernel exits on
        // the sparse pass's flag.  Otherwise, and for per-vertex extras, the LDS tile pass.
        const bool mf16 = EX == kExNone && d == 16 && pph.table_full;
        const bool full = EX == kExNone && pph.table_full && plan.mfma_items > 0;
        {
            TimedLaunches tl(kTkExact, s);
            const int *sample = route_sample(plan, d, EX == kExNone, pph) ? gc.sample : nullptr;
            (void)gempe_launch_near_tiles(g, d, X, gc, pph, EX, grad, extra, partials, s, full ? 2 : mf16 ? 1 : 0,
                                          sample, (int)plan.mfma_items);
        }
        if (full) {
            TimedLaunches tf(kTkFull, s);
            SweepPlan pm = plan;
            pm.items = plan.mfma_items;
            pm.grid = plan.mfma_grid;
            if (d == 16)
                (void)gempe_launch_sweep_mfma16(pm, X, n, grad, partials, pph, s, gc.all_dense);
            else
                (void)gempe_launch_sweep_mfma_wide(pm, d, X, n, grad, partials, pph, s, gc.all_dense);
        }
        TimedLaunches tl(kTkExact, s);
        if (mf16)
            (void)gempe_launch_sweep_mfma16_list(plan, X, n, gc, grad, partials, pph, s);
        else
            launch_list<EX>(plan, s, X, n, d, gc, grad, extra, partials, P);
    } else if (plan.mfma) {
        TimedLaunches tl(kTkSweep, s);
        if (d == 16)
            (void)gempe_launch_sweep_mfma16(plan, X, n, grad, partials, pph, s);
        else
            (void)gempe_launch_sweep_mfma_wide(plan, d, X, n, grad, partials, pph, s);
    } else {
        TimedLaunches tl(kTkSweep, s);
        launch_sweep<EX>(plan, s, X, n, d, grad, extra, partials, P);
    }
    TimedLaunches tl(kTkEdges, s);
    float *epart = partials + plan.items;
    if (plan.D > 16 || plan.bf16) {
        // wide, and every BF16 plan: one wave per CSR row (also writes the partial of rows
        // without edges), with the squared distance (group16_sqdist) and the non-edge pair
        // function of the BF16 path's exact near-pair passes (the table at d = 16, the closed
        // form above), so a near edge's non-edge term cancels there bit for bit
#define GEMPE_EDGES_ROWS(DD)                                                                              \
    hipLaunchKernelGGL((k_edges_rows<DD, EX>), dim3(plan.edge_blocks), dim3(256), 0, s, X, n, d, g->row_ptr, \
                       g->col_idx, g->hash, (unsigned long long)g->hash_cap, grad, extra, epart, hits, P,    \
                       plan.T, plan.nt, plan.shard, plan.nshards)
        if (plan.D == 16)
            GEMPE_EDGES_ROWS(16);
        else if (plan.D == 32)
            GEMPE_EDGES_ROWS(32);
        else if (plan.D == 64)
            GEMPE_EDGES_ROWS(64);
        else
            GEMPE_EDGES_ROWS(128);
#undef GEMPE_EDGES_ROWS
    } else if (g->nnz > 0) {
        hipLaunchKernelGGL((k_edges<EX>), dim3(plan.edge_blocks), dim3(kEdgeBlock), 0, s, X, d, g->coo_row,
                           g->col_idx, (long long)g->nnz, g->hash, (unsigned long long)g->hash_cap, grad, extra,
                           epart, hits, P, plan.T, plan.nt, plan.shard, plan.nshards);
    } else {
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, epart, (long long)plan.edge_blocks, nullptr, 0LL,
                           nullptr, 0);
    }
}
}  // namespace

hipError_t gempe_launch_loss_grad(const gempe_graph_s *g, int d, const SweepPlan &plan_in, const float *X,
                                  float *grad, float *row_loss, float *partials, unsigned char *counters,
                                  double *loss, int64_t *hits_out, const PairParamsHost &pph,
                                  hipStream_t s, bool clear_status, const GramCtx &gc, double *red, float *wm_z) {
    const PairParams P = dev_params(pph);
    // the matrix-core sweep takes plain loss-and-gradient evaluations of the whole triangle
    // whose non-edges all lie in the pair table; the others run the vector sweep
    SweepPlan plan = plan_in;
    plan.mfma = plan_in.mfma && !row_loss && !wm_z && pph.table_full && plan_in.nshards <= 1;
    if (plan.mfma) {
        plan.items = plan_in.mfma_items;
        plan.grid = plan_in.mfma_grid;
    }
    const int n = g->n;
    const long long nd = (long long)n * d;
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(counters);
    unsigned *status = reinterpret_cast<unsigned *>(counters + 8);
    float *extra = wm_z ? wm_z : row_loss;
    {
        long long big = std::max<long long>(nd, extra ? n : 0);
        unsigned blocks = (unsigned)std::min<long long>(4096, std::max<long long>(1, (big + 255) / 256));
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, grad, nd, extra, extra ? (long long)n : 0, cnt,
                           clear_status ? 2 : 1);
    }
    if (plan.bf16) {
        const bool plain = !row_loss && !wm_z;
        hipError_t e = gempe_launch_gram_screen(g, d, X, gc.xb, gc.nrm, gc.snorm, gc.smax128, gc.flags, gc.list,
                                                gc.count, gc.theta0, gc.chunks, s,
                                                route_sample(plan, d, plain, pph) ? gc.sample : nullptr);
        if (e != hipSuccess) return e;
    }
    if (wm_z)
        launch_pass<kExZ>(g, d, plan, X, grad, wm_z, partials, hits_out ? cnt : nullptr, P, pph, s, gc);
    else if (row_loss)
        launch_pass<kExRowLoss>(g, d, plan, X, grad, row_loss, partials, hits_out ? cnt : nullptr, P, pph, s, gc);
    else
        launch_pass<kExNone>(g, d, plan, X, grad, nullptr, partials, hits_out ? cnt : nullptr, P, pph, s, gc);
    float *epart = partials + plan.items;
    // FP64 loss: sweep partials (for the BF16 screen only the flagged tiles' slots) + edge partials
    const long long total = plan.items + plan.edge_blocks;
    const int nb1 = (int)std::min<long long>(kRed1Blocks, std::max<long long>(1, (total + 4095) / 4096));
    const long long chunk = (total + nb1 - 1) / nb1;
    hipLaunchKernelGGL(k_reduce1, dim3(nb1), dim3(kFinBlock), 0, s, partials, plan.items,
                       plan.bf16 ? gc.count : nullptr, epart, (long long)plan.edge_blocks, chunk, red);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, s, red, nb1, loss, cnt, hits_out, status);
    return hipGetLastError();
}

hipError_t gempe_launch_wm_update(float *X, const float *G, const float *Z, int d, long long count, hipStream_t s) {
    unsigned blocks = (unsigned)std::max<long long>(1, (count + 255) / 256);
    hipLaunchKernelGGL(k_wm_update, dim3(blocks), dim3(256), 0, s, X, G, Z, d, count);
    return hipGetLastError();
}

hipError_t gempe_launch_axpy(float *X, const float *G, float eta, long long count, hipStream_t s) {
    unsigned blocks = (unsigned)std::max<long long>(1, (count + 255) / 256);
    hipLaunchKernelGGL(k_axpy, dim3(blocks), dim3(256), 0, s, X, G, eta, count);
    return hipGetLastError();
}

namespace {
IterArgs make_iter_args(const gempe_graph_s *g, int d, const SweepPlan &plan, float *X, float eta,
                        double *loss_hist, const WsLayout &L, unsigned char *ws, const PairParamsHost &pph) {
    IterArgs a;
    a.Xc = X;
    a.Xw = reinterpret_cast<float *>(ws + L.xbuf);
    a.G0 = reinterpret_cast<float *>(ws + L.gring);
    a.P0 = reinterpret_cast<float *>(ws + L.ppart);
    a.loss_hist = loss_hist;
    a.status = reinterpret_cast<unsigned *>(ws + L.counters + 8);
    a.coo_row = g->coo_row;
    a.col = g->col_idx;
    a.nnz = g->nnz;
    a.n = g->n;
    a.d = d;
    a.nb = (int)plan.nb64;
    a.epu = kEdgesPerUnit;
    a.units_edge = plan.units_edge;
    a.units = plan.units;
    a.neg_eta = -eta;
    a.P = dev_params(pph);
    return a;
}
}  // namespace

size_t gempe_batch_entry_bytes() { return sizeof(BatchEntry); }

void gempe_batch_entry_fill(void *dst, const gempe_graph_s *g, int d, const SweepPlan &plan, float *X,
                            int iters, float eta, double *loss_hist, const WsLayout &L, unsigned char *ws,
                            const PairParamsHost &pph, long long u0, int k0) {
    BatchEntry e{};
    e.a = make_iter_args(g, d, plan, X, eta, loss_hist, L, ws, pph);
    e.u0 = u0;
    e.blocks = plan.iter_blocks;
    e.k0 = k0;
    e.K = iters + (loss_hist ? 1 : 0);
    e.iters = iters;
    std::memcpy(dst, &e, sizeof(e));
}

hipError_t gempe_batch_prepare(const gempe_graph_s *g, int d, const WsLayout &L, unsigned char *ws,
                               hipStream_t s) {
    // gradient slot 0 and the status word start at zero (a fill kernel, no memset)
    const long long nd = (long long)g->n * d;
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(ws + L.counters);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<long long>(1024, std::max<long long>(1, (nd + 255) / 256))),
                       dim3(256), 0, s, reinterpret_cast<float *>(ws + L.gring), nd, nullptr, 0LL, cnt, 2);
    return hipGetLastError();
}

hipError_t gempe_launch_iter_batch(int D, const void *table, int njobs, long long blocks, int tick,
                                   hipStream_t s) {
    const BatchEntry *t = static_cast<const BatchEntry *>(table);
    const dim3 grid((unsigned)blocks), block(256);
    switch (D) {
        case 1: hipLaunchKernelGGL(k_iter_batch<1>, grid, block, 0, s, t, njobs, tick); break;
        case 2: hipLaunchKernelGGL(k_iter_batch<2>, grid, block, 0, s, t, njobs, tick); break;
        case 3: hipLaunchKernelGGL(k_iter_batch<3>, grid, block, 0, s, t, njobs, tick); break;
        case 4: hipLaunchKernelGGL(k_iter_batch<4>, grid, block, 0, s, t, njobs, tick); break;
        case 8: hipLaunchKernelGGL(k_iter_batch<8>, grid, block, 0, s, t, njobs, tick); break;
        case 16: hipLaunchKernelGGL(k_iter_batch<16>, grid, block, 0, s, t, njobs, tick); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t gempe_launch_embed_fused(const gempe_graph_s *g, int d, const SweepPlan &plan, float *X,
                                    int iters, float eta, double *loss_hist, const WsLayout &L,
                                    unsigned char *ws, const PairParamsHost &pph, hipStream_t s) {
    const long long nd = (long long)g->n * d;
    IterArgs a = make_iter_args(g, d, plan, X, eta, loss_hist, L, ws, pph);
    const int K = iters + (loss_hist ? 1 : 0);
    // clear gradient slot 0 and the status word (a fill kernel, no memset)
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(ws + L.counters);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<long long>(1024, std::max<long long>(1, (nd + 255) / 256))),
                       dim3(256), 0, s, a.G0, nd, nullptr, 0LL, cnt, 2);
    switch (plan.D) {
        case 1: launch_iters<1>(plan, a, K, iters, s); break;
        case 2: launch_iters<2>(plan, a, K, iters, s); break;
        case 3: launch_iters<3>(plan, a, K, iters, s); break;
        case 4: launch_iters<4>(plan, a, K, iters, s); break;
        case 8: launch_iters<8>(plan, a, K, iters, s); break;
        default: launch_iters<16>(plan, a, K, iters, s); break;
    }
    return hipGetLastError();
}
