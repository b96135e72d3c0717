// FP32 all-pairs sweep for d = 16 on the matrix cores (gfx950 v_mfma_f32_16x16x4_f32).
//
// At d = 16 the two O(d) parts of every pair are dense contractions over a tile of rows I
// and columns J:
//   squared distance   r2_ij = |x_i|^2 + |x_j|^2 - 2 x_i . x_j     (Gram block X_I X_J^T)
//   gradient           g_i += S_i x_i - sum_j cc_ij x_j,  S_i = sum_j cc_ij
//                      g_j += T_j x_j - sum_i cc_ij x_i,  T_j = sum_i cc_ij
// (cc_ij = (d dl/d delta)/delta, the coefficient of x_i - x_j in g_i).  Each of the three
// products X_I X_J^T, C^T X_I and C X_J runs on FP32 MFMA (full single-precision products,
// FP32 accumulation); the vector ALUs evaluate the pair function (the non-edge table of
// ltab.h) between them.  Per 16 x 16 block of pairs a wave issues 4 + 4 + 4 MFMAs:
//   - Gram: A = -2 x_I (lane (g, c) holds -2 x[i0 + c][4 kb + g], kb = 0..3), B = x_J; the
//     accumulator starts at |x_i|^2 + |x_j|^2, so it ends holding r2 of pair
//     (i0 + 4g + v, j0 + c) in register v of lane (g, c);
//   - column side: B = the cc register v itself (its rows i0 + 4g + v are the contraction
//     index), A = x_I in the layout lane (g, c) -> x[i0 + 4g + v][c];
//   - row side: the contraction runs over j, which the Gram layout keeps on the lanes, so the
//     cc block goes through LDS once (4 scalar writes, one 16-byte read per lane) to become
//     the B operand, with A = x_J in the layout lane (g, c) -> x[j0 + 4g + blk][c].
//
// Precision.  The Gram form loses accuracy where |x_i - x_j| is small against |x_i| and
// |x_j| (the error of r2 is a few single-precision units of |x_i|^2 + |x_j|^2, and the split
// gradient's terms are cc |x| instead of cc |x_i - x_j|).  A pair is therefore computed from
// the Gram only while r2 > kappa (|x_i|^2 + |x_j|^2), kappa = 1/16: its r2 then carries a
// relative error below about 16 (d + 3) 2^-24 (typically a few 2^-24) and its split terms
// are at most sqrt(2 / kappa) = 5.7 times the direct form's.  A pair at or below the bound
// (a "near" pair: at N(0, 1) coordinates in 16 dimensions about one pair in 10^4) is
// evaluated exactly instead: the difference-form squared distance and the pair function the
// edge correction uses, its gradient added directly, and its cc left out of the MFMA
// products.  A per-lane test of the smallest r2 of the lane's four pairs against
// kappa (max |x_i|^2 + |x_j|^2) gates that path with one compare per four pairs.
//
// Work decomposition: an item is a strip of 64 rows (four waves, 16 rows each) against a
// chunk of C column blocks of 64, C = 32, 16 or 8 (the largest that still gives the launch
// 16,384 items) (upper triangle: blocks b >= the strip's own block; the
// diagonal block and the tails are masked).  The workgroup stages each column block in LDS,
// every wave multiplies its 16 rows against it, the four waves' column partials meet in
// LDS and leave with one atomic per (column, coordinate) per block; the row partials leave
// at the end of the item.  Each item writes its FP32 loss partial to its own slot.  Items
// run chunk by chunk (all strips of a column chunk, then the next chunk), so the column data
// comes from L2 and each strip's 64 rows are read once per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "ltab_stage.h"
#include "pairfn.h"
#include "tiles.h"

namespace gempe {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMS = 20;                    // LDS stride of a staged column (floats)
constexpr float kNearKappa = 1.0f / 16.0f;  // Gram pairs need r2 > kappa (|x_i|^2 + |x_j|^2)
constexpr int kListSlots = 128;             // list slots per workgroup in the BF16 path's dense pass
// A Gram pair's dl and coefficient come from the staged table (c0 raised by kTabLogScale) as
// 2^32 times their values, so that far pairs (dl below 2^-126) stay normal; the coefficient
// block, the row and column sums and the loss are carried times 2^32 and scaled back
// (exactly) at the flushes.  The exact near pairs return unscaled values.
constexpr float kCScale = 0x1p32f, kCUnscale = kTabUnscale;

// Position of coordinate k in a staged column: lane (g, c) reads coordinates g, 4+g, 8+g,
// 12+g of column c as one 16-byte LDS load.
__device__ __forceinline__ int perm16(int k) { return (k & 3) * 4 + (k >> 2); }

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Item t -> column chunk J (C blocks of 64) and strip I (64 rows), chunk-major: chunk J is
// needed by strips 0 .. min(nb, (J + 1) C) - 1, so the items of one chunk are consecutive and
// the workgroups an XCD runs together (consecutive items, see xcd_item) share that chunk's
// columns in the XCD's L2.  Chunks J < Jf = floor(nb / C) have (J + 1) C strips, the rest nb.
__device__ inline void mfma_item(long long t, int nb, int nJ, int C, int &I, int &J) {
    const long long Jf = nb / C;
    auto start = [nb, C, Jf](long long j) -> long long {
        const long long m = j < Jf ? j : Jf;
        return C * m * (m + 1) / 2 + (j - m) * nb;
    };
    int lo = 0, hi = nJ - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start(mid) <= t) lo = mid; else hi = mid - 1;
    }
    J = lo;
    I = (int)(t - start(lo));
}

// row16_sum's combination of 16 partial sums (one per lane of a DPP row), in one lane:
// partial t meets t + 8, then t + 4, then t + 2, then t + 1.  Every add there pairs the same
// two values in both lanes, so this gives the bits every lane of the row ends with.
__device__ __forceinline__ float row16_order(const float (&a)[16]) {
    float b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) b[t] = a[t] + a[t + 8];
    const float c0 = b[0] + b[4], c1 = b[1] + b[5], c2 = b[2] + b[6], c3 = b[3] + b[7];
    return (c0 + c2) + (c1 + c3);
}

// The exact evaluation of one near pair, its gradient added directly to both ends, with the
// squared distance and non-edge value of the edge correction that runs beside the sweep, so
// that an edge among the near pairs cancels bit for bit: G16 = false (the FP32 evaluation,
// corrected by the COO edge pass) the difference form from FLT_MIN in coordinate order;
// G16 = true (the BF16 path, corrected by the row-wave pass) group16_sqdist's sum order plus
// FLT_MIN; the table in both.  Two passes over the coordinates (the differences recomputed
// for the gradient) keep only a few values live inside the sweep's register-heavy loop.
template <bool G16>
__device__ __forceinline__ float near_pair(const float *__restrict__ X, int i, int j, const float *__restrict__ ycolj,
                                           float *__restrict__ G, const PairParams &P, const float4 *ltab,
                                           float tko) {
    const float *xi = X + (size_t)i * 16;
    float dl, cc, w;
    if (G16) {
        float a[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float df = xi[k] - ycolj[perm16(k)];
            a[k] = __builtin_fmaf(df, df, 0.0f);
        }
        nonedge_eval<false, false, true>(row16_order(a) + kFltMin, P, ltab, tko, GEMPE_LTAB_SEGS, dl, cc, w);
    } else {
        float r2 = 1.17549435e-38f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float df = xi[k] - ycolj[perm16(k)];
            r2 = __builtin_fmaf(df, df, r2);
        }
        nonedge_eval<false, false, true>(r2, P, ltab, tko, GEMPE_LTAB_SEGS, dl, cc, w);
    }
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
        const float v = cc * (xi[k] - ycolj[perm16(k)]);
        atomicAdd(&G[(size_t)i * 16 + k], v);
        atomicAdd(&G[(size_t)j * 16 + k], -v);
    }
    return dl;
}

// One 64-column block against the wave's 16 rows.  MASK: the diagonal block or a tail (only
// pairs i < j < n, i < n count).  FLUSH: pairs with r2 >= far2 add exactly 0 (the BF16 path's
// far non-edges, flushed as its screen flushes them).
template <bool MASK, bool FLUSH, bool G16>
__device__ __forceinline__ void mfma_block(const float *__restrict__ X, int n, int r0, int j0, const float (&GA)[4],
                                           const float (&CA)[4], const float (&ni)[4], float nimax,
                                           const float *__restrict__ ycol, const float *__restrict__ ynrm,
                                           float *__restrict__ tb, float *__restrict__ cp, v4f &RT, float (&S)[4],
                                           float &loss, float *__restrict__ G, const PairParams &P,
                                           const float4 *ltab, float tko, float far2, int g, int c) {
    unsigned nearq = 0;  // column groups with near pairs (wave-uniform)
    // the Gram block of the next column group is issued before this group's pair function,
    // so the matrix core works on it while the vector ALUs evaluate; the loop over the four
    // groups stays rolled, which keeps the kernel within 128 VGPRs (four waves per SIMD)
    v4f accn;
    {
        const float4 gb = *reinterpret_cast<const float4 *>(ycol + c * kMS + 4 * g);
        const float nj0 = ynrm[c];
#pragma unroll
        for (int v = 0; v < 4; ++v) accn[v] = ni[v] + nj0;
        accn = mfma(GA[0], gb.x, accn);
        accn = mfma(GA[1], gb.y, accn);
        accn = mfma(GA[2], gb.z, accn);
        accn = mfma(GA[3], gb.w, accn);
    }
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const v4f acc = accn;
        if (q < 3) {
            const float4 gb = *reinterpret_cast<const float4 *>(ycol + (16 * (q + 1) + c) * kMS + 4 * g);
            const float nj1 = ynrm[16 * (q + 1) + c];
#pragma unroll
            for (int v = 0; v < 4; ++v) accn[v] = ni[v] + nj1;
            accn = mfma(GA[0], gb.x, accn);
            accn = mfma(GA[1], gb.y, accn);
            accn = mfma(GA[2], gb.z, accn);
            accn = mfma(GA[3], gb.w, accn);
        }
        float RA[4];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) RA[blk] = ycol[(16 * q + 4 * g + blk) * kMS + perm16(c)];
        const float nj = ynrm[16 * q + c];
        const int j = j0 + 16 * q + c;
        // pair function from the table (every non-edge tau of a Gram pair lies in it)
        float C[4], rinv[4], f[4], dl[4];
        unsigned off[4];
        bool valid[4];
        float mn = 3.0e38f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = r0 + 4 * g + v;
            valid[v] = !MASK || (j > i && j < n && i < n);
            const float r2 = acc[v];
            mn = valid[v] ? fminf(mn, r2) : mn;
            rinv[v] = hw_rsq(r2);
            const float delta = r2 * rinv[v];
            const float tk = __builtin_fmaf(delta, P.tk_scale, tko);
            f[v] = __builtin_amdgcn_fractf(tk);
            off[v] = min((unsigned)floor_to_int(tk), (unsigned)GEMPE_LTAB_SEGS) << 4;
        }
        float4 cf[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            cf[v] = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(ltab) + off[v]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float p = cf[v].w * f[v];
            const float qq = cf[v].z + p;
            const float L = __builtin_fmaf(__builtin_fmaf(qq, f[v], cf[v].y), f[v], cf[v].x);
            const float Lf = __builtin_fmaf(__builtin_fmaf(qq, 2.0f, p), f[v], cf[v].y);
            dl[v] = hw_exp2(L);
            C[v] = dl[v] * (Lf * (P.slope_k * rinv[v]));
            if (MASK) {
                dl[v] = valid[v] ? dl[v] : 0.0f;
                C[v] = valid[v] ? C[v] : 0.0f;
            }
            if (FLUSH) {
                const bool far = acc[v] >= far2;
                dl[v] = far ? 0.0f : dl[v];
                C[v] = far ? 0.0f : C[v];
            }
        }
        // near pairs (rare) are left out of the MFMA products here and evaluated exactly after
        // the four column groups (outside this register-heavy loop)
        if (__builtin_expect(__ballot(mn <= kNearKappa * (nimax + nj)) != 0ull, 0)) {
            nearq |= 1u << q;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const bool nr = valid[v] && acc[v] <= kNearKappa * (ni[v] + nj);
                dl[v] = nr ? 0.0f : dl[v];
                C[v] = nr ? 0.0f : C[v];
            }
        }
        float T = 0.0f;
        v4f CT = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            loss += dl[v];
            S[v] += C[v];
            T += C[v];
            CT = mfma(CA[v], C[v], CT);
        }
        // transpose the cc block through this wave's LDS slot for the row-side product
#pragma unroll
        for (int v = 0; v < 4; ++v) tb[(4 * g + v) * kMS + c] = C[v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float4 ct = *reinterpret_cast<const float4 *>(tb + c * kMS + 4 * g);
        RT = mfma(RA[0], ct.x, RT);
        RT = mfma(RA[1], ct.y, RT);
        RT = mfma(RA[2], ct.z, RT);
        RT = mfma(RA[3], ct.w, RT);
        __builtin_amdgcn_wave_barrier();
        // this wave's column partials of the 16 columns: Col^T[4g + v][c] and T over g
        T += __shfl_xor(T, 16, 64);
        T += __shfl_xor(T, 32, 64);
#pragma unroll
        for (int v = 0; v < 4; ++v) cp[(16 * q + c) * 17 + 4 * g + v] = CT[v];
        if (g == 0) cp[(16 * q + c) * 17 + 16] = T;
    }
    // the near pairs of the flagged column groups: the same Gram chain (same operands, same
    // order, so the same r2 and the same decisions), then the exact evaluation
    for (int q = 0; q < 4; ++q) {
        if (!(nearq & (1u << q))) continue;
        const float4 gb = *reinterpret_cast<const float4 *>(ycol + (16 * q + c) * kMS + 4 * g);
        const float nj = ynrm[16 * q + c];
        const int j = j0 + 16 * q + c;
        v4f acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = ni[v] + nj;
        acc = mfma(GA[0], gb.x, acc);
        acc = mfma(GA[1], gb.y, acc);
        acc = mfma(GA[2], gb.z, acc);
        acc = mfma(GA[3], gb.w, acc);
        for (int v = 0; v < 4; ++v) {
            const int i = r0 + 4 * g + v;
            const bool valid = !MASK || (j > i && j < n && i < n);
            if (valid && acc[v] <= kNearKappa * (ni[v] + nj))
                loss += near_pair<G16>(X, i, j, ycol + (16 * q + c) * kMS, G, P, ltab, tko) * kCScale;
        }
    }
}

// LDS of one matrix-core workgroup.
struct MfLds {
    float4 ltab[kLtabF4];
    __attribute__((aligned(16))) float ycol[64 * kMS];
    float ynrm[64];
    __attribute__((aligned(16))) float tr[4][16 * kMS];
    float colp[4][64 * 17];
    float lsum[4];
};

// Strip I (64 rows, four waves of 16) against column blocks [b0, b1): stage each block, the
// three products per 16 x 16 block, the column partials per block, the row partials at the
// end.  Returns the workgroup's FP32 loss in thread 0.
template <bool FLUSH, bool G16>
__device__ float mfma_strip(const float *__restrict__ X, int n, int I, int b0, int b1, float *__restrict__ G,
                            const PairParams &P, float tko, float far2, MfLds &L) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // the wave's 16 rows in the three register layouts, their squared norms
    const int r0 = I * 64 + wave * 16;
    float GA[4], CA[4], ni[4], S[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int i = r0 + c;
        GA[kb] = i < n ? -2.0f * X[(size_t)i * 16 + 4 * kb + g] : 0.0f;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = r0 + 4 * g + v;
        CA[v] = i < n ? X[(size_t)i * 16 + c] : 0.0f;
        ni[v] = row16_sum(CA[v] * CA[v]);
        S[v] = 0.0f;
    }
    const float nimax = fmaxf(fmaxf(ni[0], ni[1]), fmaxf(ni[2], ni[3]));
    v4f RT = {0.f, 0.f, 0.f, 0.f};
    float loss = 0.0f;

    for (int b = b0; b < b1; ++b) {
        const int j0 = b * 64;
        float lblk = 0.0f;  // two-level loss sums: per column block, then across blocks
        __syncthreads();  // the previous block's staged columns and partials are consumed
        {
            // thread t stages coordinates 4 (t % 4) .. + 3 of column t / 4 and its share of the norm
            const int col = threadIdx.x >> 2, part = threadIdx.x & 3, j = j0 + col;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < n) v = *reinterpret_cast<const float4 *>(X + (size_t)j * 16 + 4 * part);
            float *dst = L.ycol + col * kMS;
            dst[perm16(4 * part + 0)] = v.x;
            dst[perm16(4 * part + 1)] = v.y;
            dst[perm16(4 * part + 2)] = v.z;
            dst[perm16(4 * part + 3)] = v.w;
            float s = v.x * v.x;
            s = __builtin_fmaf(v.y, v.y, s);
            s = __builtin_fmaf(v.z, v.z, s);
            s = __builtin_fmaf(v.w, v.w, s);
            s += __shfl_xor(s, 1, 64);
            s += __shfl_xor(s, 2, 64);
            if (part == 0) L.ynrm[col] = s;
        }
        __syncthreads();
        const bool masked = (b == I) || (j0 + 64 > n) || (I * 64 + 64 > n);
        if (masked)
            mfma_block<true, FLUSH, G16>(X, n, r0, j0, GA, CA, ni, nimax, L.ycol, L.ynrm, L.tr[wave], L.colp[wave], RT, S,
                                    lblk, G, P, L.ltab, tko, far2, g, c);
        else
            mfma_block<false, FLUSH, G16>(X, n, r0, j0, GA, CA, ni, nimax, L.ycol, L.ynrm, L.tr[wave], L.colp[wave], RT,
                                     S, lblk, G, P, L.ltab, tko, far2, g, c);
        loss += lblk * kCUnscale;
        __syncthreads();
        // g_j += T_j x_j - sum_i cc_ij x_i, the four waves' partials summed in wave order (two
        // elements' LDS reads issued together; unrolled whole, the loop spills at 128 VGPRs)
#pragma unroll 2
        for (int it = 0; it < 4; ++it) {
            const int k = (int)threadIdx.x + 256 * it;
            const int col = k >> 4, kk = k & 15, j = j0 + col;
            const float cs = (L.colp[0][col * 17 + kk] + L.colp[1][col * 17 + kk]) +
                             (L.colp[2][col * 17 + kk] + L.colp[3][col * 17 + kk]);
            const float ts = (L.colp[0][col * 17 + 16] + L.colp[1][col * 17 + 16]) +
                             (L.colp[2][col * 17 + 16] + L.colp[3][col * 17 + 16]);
            if (j < n)
                atomicAdd(&G[(size_t)j * 16 + kk],
                          __builtin_fmaf(ts, L.ycol[col * kMS + perm16(kk)], -cs) * kCUnscale);
        }
    }
    // g_i += S_i x_i - sum_j cc_ij x_j: lane (g, c) holds coordinates 4g .. 4g+3 of row r0 + c
    // of the product; S of row r0 + 4g' + v' is the sum over the 16 lanes of DPP row g'
    float Srow[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Srow[v] = row16_sum(S[v]);
    const int src = (c >> 2) * 16;
    const float s0 = __shfl(Srow[0], src, 64), s1 = __shfl(Srow[1], src, 64), s2 = __shfl(Srow[2], src, 64),
                s3 = __shfl(Srow[3], src, 64);
    const float si = (c & 3) == 0 ? s0 : (c & 3) == 1 ? s1 : (c & 3) == 2 ? s2 : s3;
    const int i = r0 + c;
    if (i < n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = 4 * g + v;
            atomicAdd(&G[(size_t)i * 16 + k], __builtin_fmaf(si, X[(size_t)i * 16 + k], -RT[v]) * kCUnscale);
        }
    }
    const float ws = wave_sum(loss);
    if (lane == 0) L.lsum[wave] = ws;
    __syncthreads();
    return (L.lsum[0] + L.lsum[1]) + (L.lsum[2] + L.lsum[3]);
}


}  // namespace

// BF: the BF16 path's evaluation whose screen flagged most tiles; it runs only when the
// sparse pass set *gate (every pair exact in FP32, near pairs in that path's form).
template <bool BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sweep_mfma16(const float *__restrict__ X, int n, int nb, int nJ, int C,
                                                      long long items, long long per_xcd, float *__restrict__ G,
                                                      float *__restrict__ partials, PairParams P,
                                                      const int *__restrict__ gate) {
    __shared__ MfLds L;
    if (BF && *gate == 0) return;  // uniform over the grid
    long long t = xcd_item(blockIdx.x, per_xcd);
    if (t >= items) return;  // uniform over the workgroup
    if (P.reverse) t = items - 1 - t;
    stage_ltab(L.ltab);  // the strip's first barrier orders it before any use
    int I, J;
    mfma_item(t, nb, nJ, C, I, J);
    const float l = mfma_strip<false, BF>(X, n, I, max(J * C, I), min(J * C + C, nb), G, P,
                                          table_offset(P, kLtabZero), 0.0f, L);
    if (threadIdx.x == 0) partials[t] = l;
}

// The exact FP32 pass of the BF16 path at d = 16 over the densely flagged 64 x 64 tiles of
// its screen (list[0..*count) in increasing order, dense[q] set; partial slot q belongs to
// list[q]), on the matrix cores: the pairs at or beyond the far distance add 0 as the
// screen's unflagged pairs do, the near pairs take the exact path.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_sweep_mfma16_list(const float *__restrict__ X, int n, int nb,
                                                           const int *__restrict__ list,
                                                           const int *__restrict__ count,
                                                           const unsigned char *__restrict__ dense,
                                                           float *__restrict__ G, float *__restrict__ partials,
                                                           PairParams P, float far2, const int *__restrict__ all_dense) {
    __shared__ MfLds L;
    if (*all_dense) return;  // the full sweep took every tile (uniform over the grid)
    stage_ltab(L.ltab);
    const float tko = table_offset(P, kLtabZero);
    const int cnt = *count;
    // workgroup w owns slots [S w, S w + S), S = kListSlots (and the same range one grid further on); a
    // run of dense slots holding consecutive tiles of one strip is one strip call (rows loaded
    // and flushed once), its loss in the run's first slot and 0 in the others
    for (int base = blockIdx.x * kListSlots; base < cnt; base += gridDim.x * kListSlots) {
        const int end = min(base + kListSlots, cnt);
        for (int q = base; q < end;) {
            if (!dense[q]) {  // uniform: finished by the sparse pass
                ++q;
                continue;
            }
            int I, J;
            tile_of(list[q], nb, I, J);
            int r = q + 1;
            while (r < end && dense[r] && list[r] == list[r - 1] + 1 && J + (r - q) < nb) ++r;
            const float l = mfma_strip<true, true>(X, n, I, J, J + (r - q), G, P, tko, far2, L);
            if (threadIdx.x == 0) {
                partials[q] = l;
                for (int z = q + 1; z < r; ++z) partials[z] = 0.0f;
            }
            q = r;
        }
    }
}

// ------------------------------------------------------------------------------------
// The same decomposition for d = 32, 64, 128 (D = 16 M).  Per 16 x 16 block a wave issues
// D/4 MFMAs for the Gram and D/4 for each gradient side: the coordinates form M chunks of
// 16, each chunk one 16 x 16 output block of the column-side product (A = x_I in the layout
// lane (g, c) -> x[i0 + 4g + v][16m + c]) and of the row-side product (A = x_J in the layout
// lane (g, c) -> x[j0 + 4g + blk][16m + c]).  A staged column keeps its coordinates in
// chunks of 16, each in the perm16 order, so a lane's Gram operands of a chunk are one
// 16-byte load.  The four waves' column partials (D x 16 per column group) meet in LDS per
// column group and leave with one atomic per (column, coordinate) per 64-row strip.
// ------------------------------------------------------------------------------------
namespace {

template <int D>
struct MfLdsW {
    static constexpr int kS = D + 4;  // column stride (16-byte aligned rows)
    float4 ltab[kLtabF4];
    __attribute__((aligned(16))) float ycol[64 * kS];
    float ynrm[64];
    __attribute__((aligned(16))) float tr[4][16 * kMS];
    float colq[4][16 * (D + 1)];
    float lsum[4];
};

// The exact evaluation of one near pair at d = 32, 64, 128: the squared distance in
// difference form from FLT_MIN in coordinate order and the table.  It agrees with the wide
// edge correction (group16_sqdist and the closed form) to rounding, as the VALU wide sweep
// does; forming that pass's bits here (16 partial sums in its order, the closed form) costs
// these register-bound kernels 60 to 70 VGPRs.
template <int D>
__device__ __forceinline__ float near_pair_w(const float *__restrict__ X, int i, int j, const float *__restrict__ ycolj,
                                             float *__restrict__ G, const PairParams &P, const float4 *ltab,
                                             float tko) {
    const float *xi = X + (size_t)i * D;
    float r2 = 1.17549435e-38f;
#pragma unroll 8
    for (int k = 0; k < D; ++k) {
        const float df = xi[k] - ycolj[(k & ~15) + perm16(k & 15)];
        r2 = __builtin_fmaf(df, df, r2);
    }
    float dl, cc, w;
    nonedge_eval<false, false, true>(r2, P, ltab, tko, GEMPE_LTAB_SEGS, dl, cc, w);
#pragma unroll 4
    for (int k = 0; k < D; ++k) {
        const float v = cc * (xi[k] - ycolj[(k & ~15) + perm16(k & 15)]);
        atomicAdd(&G[(size_t)i * D + k], v);
        atomicAdd(&G[(size_t)j * D + k], -v);
    }
    return dl;
}

template <int D, bool MASK>
__device__ __forceinline__ void mfma_block_w(const float *__restrict__ X, int n, int r0, int j0,
                                             const float (&GA)[D / 4], const float (&CA)[D / 16][4],
                                             const float (&ni)[4], float nimax, MfLdsW<D> &L, int wave,
                                             v4f (&RT)[D / 16], float (&S)[4], float &loss, float *__restrict__ G,
                                             const PairParams &P, float tko, int g, int c) {
    constexpr int M = D / 16, kS = MfLdsW<D>::kS;
    float *tb = L.tr[wave];
    // the Gram block of the next column group is issued before this group's pair function, so
    // that the matrix core works while the vector ALUs evaluate (not at d = 64: the held block
    // would cost that kernel its third wave per SIMD)
    constexpr bool kAhead = D != 64;
    auto gram = [&](int qq) {
        const float *ycq = L.ycol + (16 * qq + c) * kS;
        const float njq = L.ynrm[16 * qq + c];
        v4f a;
#pragma unroll
        for (int v = 0; v < 4; ++v) a[v] = ni[v] + njq;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float4 gb = *reinterpret_cast<const float4 *>(ycq + 16 * m + 4 * g);
            a = mfma(GA[4 * m + 0], gb.x, a);
            a = mfma(GA[4 * m + 1], gb.y, a);
            a = mfma(GA[4 * m + 2], gb.z, a);
            a = mfma(GA[4 * m + 3], gb.w, a);
        }
        return a;
    };
    v4f accn;
    if (kAhead) accn = gram(0);
    for (int q = 0; q < 4; ++q) {
        const float *ycj = L.ycol + (16 * q + c) * kS;
        const float nj = L.ynrm[16 * q + c];
        const int j = j0 + 16 * q + c;
        const v4f acc = kAhead ? accn : gram(q);
        if (kAhead && q < 3) accn = gram(q + 1);
        float C[4], rinv[4], f[4], dl[4];
        unsigned off[4];
        bool valid[4];
        float mn = 3.0e38f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = r0 + 4 * g + v;
            valid[v] = !MASK || (j > i && j < n && i < n);
            const float r2 = acc[v];
            mn = valid[v] ? fminf(mn, r2) : mn;
            rinv[v] = hw_rsq(r2);
            const float delta = r2 * rinv[v];
            const float tk = __builtin_fmaf(delta, P.tk_scale, tko);
            f[v] = __builtin_amdgcn_fractf(tk);
            off[v] = min((unsigned)floor_to_int(tk), (unsigned)GEMPE_LTAB_SEGS) << 4;
        }
        float4 cf[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            cf[v] = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(L.ltab) + off[v]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float p = cf[v].w * f[v];
            const float qq = cf[v].z + p;
            const float Lv = __builtin_fmaf(__builtin_fmaf(qq, f[v], cf[v].y), f[v], cf[v].x);
            const float Lf = __builtin_fmaf(__builtin_fmaf(qq, 2.0f, p), f[v], cf[v].y);
            dl[v] = hw_exp2(Lv);
            C[v] = dl[v] * (Lf * (P.slope_k * rinv[v]));
            if (MASK) {
                dl[v] = valid[v] ? dl[v] : 0.0f;
                C[v] = valid[v] ? C[v] : 0.0f;
            }
        }
        // near pairs: exact, out of the MFMA products (rare at a spread start)
        if (__builtin_expect(__ballot(mn <= kNearKappa * (nimax + nj)) != 0ull, 0)) {
            for (int v = 0; v < 4; ++v) {
                if (valid[v] && acc[v] <= kNearKappa * (ni[v] + nj)) {
                    dl[v] = near_pair_w<D>(X, r0 + 4 * g + v, j, ycj, G, P, L.ltab, tko) * kCScale;
                    C[v] = 0.0f;
                }
            }
        }
        float T = 0.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            loss += dl[v];
            S[v] += C[v];
            T += C[v];
        }
        // column side: Col^T[16m + 4g + v][c] of this wave's 16 rows, into its LDS slot
        float *cq = L.colq[wave];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            v4f CT = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) CT = mfma(CA[m][v], C[v], CT);
#pragma unroll
            for (int v = 0; v < 4; ++v) cq[c * (D + 1) + 16 * m + 4 * g + v] = CT[v];
        }
        T += __shfl_xor(T, 16, 64);
        T += __shfl_xor(T, 32, 64);
        if (g == 0) cq[c * (D + 1) + D] = T;
        // row side: the cc block transposed through LDS, then one 16 x 16 output per chunk
#pragma unroll
        for (int v = 0; v < 4; ++v) tb[(4 * g + v) * kMS + c] = C[v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float4 ct = *reinterpret_cast<const float4 *>(tb + c * kMS + 4 * g);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float *ra = L.ycol + (16 * q + 4 * g) * kS + 16 * m + perm16(c);
            RT[m] = mfma(ra[0 * kS], ct.x, RT[m]);
            RT[m] = mfma(ra[1 * kS], ct.y, RT[m]);
            RT[m] = mfma(ra[2 * kS], ct.z, RT[m]);
            RT[m] = mfma(ra[3 * kS], ct.w, RT[m]);
        }
        __builtin_amdgcn_wave_barrier();
        // the four waves' partials of these 16 columns, summed in wave order:
        // g_j += T_j x_j - sum_i cc_ij x_i (the loop unrolled, so that each thread's LDS
        // reads are issued together instead of one iteration's at a time)
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 16 * D / 256; ++it) {
            const int k = (int)threadIdx.x + 256 * it;
            const int col = k / D, kk = k - col * D, jj = j0 + 16 * q + col;
            const int o = col * (D + 1);
            const float cs = (L.colq[0][o + kk] + L.colq[1][o + kk]) + (L.colq[2][o + kk] + L.colq[3][o + kk]);
            const float ts = (L.colq[0][o + D] + L.colq[1][o + D]) + (L.colq[2][o + D] + L.colq[3][o + D]);
            const float xj = L.ycol[(16 * q + col) * kS + (kk & ~15) + perm16(kk & 15)];
            if (jj < n) atomicAdd(&G[(size_t)jj * D + kk], __builtin_fmaf(ts, xj, -cs) * kCUnscale);
        }
        __syncthreads();  // the slots are rewritten by the next column group
    }
}

template <int D>
__device__ float mfma_strip_w(const float *__restrict__ X, int n, int I, int b0, int b1, float *__restrict__ G,
                              const PairParams &P, float tko, MfLdsW<D> &L) {
    constexpr int M = D / 16, kS = MfLdsW<D>::kS;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r0 = I * 64 + wave * 16;
    float GA[D / 4], CA[M][4], ni[4], S[4];
#pragma unroll
    for (int kb = 0; kb < D / 4; ++kb) {
        const int i = r0 + c;
        GA[kb] = i < n ? -2.0f * X[(size_t)i * D + 4 * kb + g] : 0.0f;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = r0 + 4 * g + v;
        float sq = 0.0f;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            CA[m][v] = i < n ? X[(size_t)i * D + 16 * m + c] : 0.0f;
            sq = __builtin_fmaf(CA[m][v], CA[m][v], sq);
        }
        ni[v] = row16_sum(sq);
        S[v] = 0.0f;
    }
    const float nimax = fmaxf(fmaxf(ni[0], ni[1]), fmaxf(ni[2], ni[3]));
    v4f RT[M];
#pragma unroll
    for (int m = 0; m < M; ++m) RT[m] = v4f{0.f, 0.f, 0.f, 0.f};
    float loss = 0.0f;
    for (int b = b0; b < b1; ++b) {
        const int j0 = b * 64;
        float lblk = 0.0f;
        __syncthreads();  // the previous block's staged columns are consumed
        // stage 64 columns: float4 f of column col goes to chunk f / 4, perm16 order
        for (int k = threadIdx.x; k < 64 * (D / 4); k += 256) {
            const int col = k / (D / 4), f4 = k - col * (D / 4), j = j0 + col;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < n) v = *reinterpret_cast<const float4 *>(X + (size_t)j * D + 4 * f4);
            float *dst = L.ycol + col * kS + 16 * (f4 >> 2);
            const int k0 = 4 * (f4 & 3);
            dst[perm16(k0 + 0)] = v.x;
            dst[perm16(k0 + 1)] = v.y;
            dst[perm16(k0 + 2)] = v.z;
            dst[perm16(k0 + 3)] = v.w;
        }
        __syncthreads();
        {  // squared norms of the staged columns: four quarter sums per column, combined in order
            const float *yc = L.ycol + (threadIdx.x >> 2) * kS + (threadIdx.x & 3) * (D / 4);
            float sq = 0.0f;
#pragma unroll 8
            for (int k = 0; k < D / 4; ++k) sq = __builtin_fmaf(yc[k], yc[k], sq);
            sq += __shfl_xor(sq, 1, 64);
            sq += __shfl_xor(sq, 2, 64);
            if ((threadIdx.x & 3) == 0) L.ynrm[threadIdx.x >> 2] = sq;
        }
        __syncthreads();
        const bool masked = (b == I) || (j0 + 64 > n) || (I * 64 + 64 > n);
        if (masked)
            mfma_block_w<D, true>(X, n, r0, j0, GA, CA, ni, nimax, L, wave, RT, S, lblk, G, P, tko, g, c);
        else
            mfma_block_w<D, false>(X, n, r0, j0, GA, CA, ni, nimax, L, wave, RT, S, lblk, G, P, tko, g, c);
        loss += lblk * kCUnscale;
    }
    // g_i += S_i x_i - sum_j cc_ij x_j: lane (g, c) holds coordinates 16m + 4g .. + 3 of row r0 + c
    float Srow[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Srow[v] = row16_sum(S[v]);
    const int src = (c >> 2) * 16;
    const float s0 = __shfl(Srow[0], src, 64), s1 = __shfl(Srow[1], src, 64), s2 = __shfl(Srow[2], src, 64),
                s3 = __shfl(Srow[3], src, 64);
    const float si = (c & 3) == 0 ? s0 : (c & 3) == 1 ? s1 : (c & 3) == 2 ? s2 : s3;
    const int i = r0 + c;
    if (i < n) {
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = 16 * m + 4 * g + v;
                atomicAdd(&G[(size_t)i * D + k], __builtin_fmaf(si, X[(size_t)i * D + k], -RT[m][v]) * kCUnscale);
            }
    }
    const float ws = wave_sum(loss);
    if (lane == 0) L.lsum[wave] = ws;
    __syncthreads();
    return (L.lsum[0] + L.lsum[1]) + (L.lsum[2] + L.lsum[3]);
}

}  // namespace

// d = 32 held to four waves per SIMD (128 VGPRs, a few spilled: 9.5 % faster than three
// waves without spills), d = 64 to three and d = 128 to two (the unrolled column flush would
// otherwise take the registers of a wave; a few values spill instead)
// BF: the BF16 path's evaluation whose screen flagged most tiles; it runs only when the
// sparse pass set *gate (every pair exact in FP32).
template <int D, bool BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 32 ? 4 : D == 64 ? 3 : 2))) void k_sweep_mfma_wide(const float *__restrict__ X, int n, int nb, int nJ, int C,
                                                         long long items, long long per_xcd, float *__restrict__ G,
                                                         float *__restrict__ partials, PairParams P,
                                                         const int *__restrict__ gate) {
    __shared__ MfLdsW<D> L;
    if (BF && *gate == 0) return;  // uniform over the grid
    long long t = xcd_item(blockIdx.x, per_xcd);
    if (t >= items) return;  // uniform over the workgroup
    if (P.reverse) t = items - 1 - t;
    stage_ltab(L.ltab);
    int I, J;
    mfma_item(t, nb, nJ, C, I, J);
    const float l = mfma_strip_w<D>(X, n, I, max(J * C, I), min(J * C + C, nb), G, P, table_offset(P, kLtabZero), L);
    if (threadIdx.x == 0) partials[t] = l;
}

}  // namespace gempe

using namespace gempe;

long long gempe_mfma_items(int n, int chunk) {
    const long long nb = (n + 63) / 64, nJ = (nb + chunk - 1) / chunk;
    const long long a = nb / chunk, r = nb - a * chunk;
    return nb * nJ - ((long long)chunk * a * (a - 1) / 2 + r * a);
}

hipError_t gempe_launch_sweep_mfma16(const SweepPlan &pl, const float *X, int n, float *G, float *partials,
                                     const PairParamsHost &pph, hipStream_t s, const int *gate) {
    const PairParams P{pph.mu_s,   pph.inv_sigma, pph.c_neg,   pph.c_pos,   pph.tk_scale,   pph.tk_off,
                       pph.slope_k, pph.r_scale,  pph.w_scale, pph.wk2,     pph.table_full, pph.reverse};
    const int nb = (n + 63) / 64;
    const int nJ = (nb + pl.mfma_chunk - 1) / pl.mfma_chunk;
    const long long per = pl.grid / kXcd;
    if (gate)
        hipLaunchKernelGGL(k_sweep_mfma16<true>, dim3((unsigned)pl.grid), dim3(256), 0, s, X, n, nb, nJ,
                           pl.mfma_chunk, pl.items, per, G, partials, P, gate);
    else
        hipLaunchKernelGGL(k_sweep_mfma16<false>, dim3((unsigned)pl.grid), dim3(256), 0, s, X, n, nb, nJ,
                           pl.mfma_chunk, pl.items, per, G, partials, P, gate);
    return hipGetLastError();
}

hipError_t gempe_launch_sweep_mfma16_list(const SweepPlan &pl, const float *X, int n, const GramCtx &gc, float *G,
                                          float *partials, const PairParamsHost &pph, hipStream_t s) {
    const PairParams P{pph.mu_s,   pph.inv_sigma, pph.c_neg,   pph.c_pos,   pph.tk_scale,   pph.tk_off,
                       pph.slope_k, pph.r_scale,  pph.w_scale, pph.wk2,     pph.table_full, pph.reverse};
    const int nb = (n + 63) / 64;
    const unsigned grid =
        (unsigned)std::max<long long>(1, std::min<long long>((pl.items + kListSlots - 1) / kListSlots, 8192));
    hipLaunchKernelGGL(k_sweep_mfma16_list, dim3(grid), dim3(256), 0, s, X, n, nb, gc.list, gc.count, gc.dense, G,
                       partials, P, gc.theta0 * gc.theta0, gc.all_dense);
    return hipGetLastError();
}

hipError_t gempe_launch_sweep_mfma_wide(const SweepPlan &pl, int d, const float *X, int n, float *G, float *partials,
                                        const PairParamsHost &pph, hipStream_t s, const int *gate) {
    const PairParams P{pph.mu_s,   pph.inv_sigma, pph.c_neg,   pph.c_pos,   pph.tk_scale,   pph.tk_off,
                       pph.slope_k, pph.r_scale,  pph.w_scale, pph.wk2,     pph.table_full, pph.reverse};
    const int nb = (n + 63) / 64;
    const int nJ = (nb + pl.mfma_chunk - 1) / pl.mfma_chunk;
    const long long per = pl.grid / kXcd;
    const dim3 grid((unsigned)pl.grid), block(256);
#define GEMPE_WIDE(DD)                                                                                          \
    if (gate)                                                                                                   \
        hipLaunchKernelGGL((k_sweep_mfma_wide<DD, true>), grid, block, 0, s, X, n, nb, nJ, pl.mfma_chunk, pl.items, \
                           per, G, partials, P, gate);                                                          \
    else                                                                                                        \
        hipLaunchKernelGGL((k_sweep_mfma_wide<DD, false>), grid, block, 0, s, X, n, nb, nJ, pl.mfma_chunk,          \
                           pl.items, per, G, partials, P, gate)
    switch (d) {
        case 32: GEMPE_WIDE(32); break;
        case 64: GEMPE_WIDE(64); break;
        case 128: GEMPE_WIDE(128); break;
        default: return hipErrorInvalidValue;
    }
#undef GEMPE_WIDE
    return hipGetLastError();
}
