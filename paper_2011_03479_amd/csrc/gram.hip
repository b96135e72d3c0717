// BF16 MFMA Gram screen for wide embeddings (d >= 16, d % 16 == 0).
//
// For d >= 64 the squared distance is a dense contraction: delta^2 = |x_i|^2 + |x_j|^2
// - 2 x_i.x_j.  The screen computes G~ = X~_I X~_J^T for 128 x 128 vertex tiles on MFMA
// (v_mfma_f32_32x32x16_bf16: BF16 operands, exact products, FP32 accumulation) from
// X~ = bf16(X), and decides per 64 x 64 sub-tile whether any pair (i < j) can be near:
//
//   bf16 rounding moves each point by at most 2^-8 |x_i|, so the distance between the
//   rounded points differs from the true one by at most 2^-8 (|x_i| + |x_j|); with
//   theta_ij = mu + near_k sigma + 2^-7 (|x_i| + |x_j|) (twice that bound, which also
//   covers the FP32 accumulation of G~ and of the norms), a pair whose computed
//   delta~^2 = n~_i + n~_j - 2 G~ is >= theta_ij^2 has true delta >= mu + near_k sigma.
//
// The test uses one theta per 128 x 128 tile (the largest |x| of its rows and columns),
// which only makes it stricter, and is evaluated as G~ - h_i > h_j with
// h = n~/2 - theta^2/4, two VALU operations per pair.  Flagged sub-tiles are compacted in
// tile order and recomputed exactly in FP32 by the LDS sweep (k_sweep_wide over the
// list); every other non-edge pair has delta >= mu + near_k sigma and is flushed: it
// contributes less than -log2 Phi(-near_k) bits (< 2e-19 at near_k = 9) and a gradient
// coefficient of the same order.  Edges are always recomputed exactly by the edge pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "pairfn.h"

namespace gempe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kXcdG = 8;

__device__ inline void tile_of_g(long long t, int nt, int &I, int &J) {
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

__device__ __forceinline__ long long upper_index(long long r, long long c, long long nt) {
    return r * nt - r * (r - 1) / 2 + (c - r);
}

__device__ __forceinline__ float wave_sum_g(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per vertex: X~ = bf16(X) (round to nearest even), n~ = |x~|^2 (FP32 from the
// rounded values), s = |x| (FP32, from the unrounded coordinates).
__global__ __launch_bounds__(256) void k_prep_bf16(const float *__restrict__ X, int n, int d,
                                                   __bf16 *__restrict__ Xb, float *__restrict__ nrm,
                                                   float *__restrict__ snorm) {
    const int lane = threadIdx.x & 63;
    const long long v = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    float sb = 0.0f, sx = 0.0f;
    for (int k = lane; k < d; k += 64) {
        float x = X[v * d + k];
        __bf16 b = (__bf16)x;
        Xb[v * d + k] = b;
        float xb = (float)b;
        sb = __builtin_fmaf(xb, xb, sb);
        sx = __builtin_fmaf(x, x, sx);
    }
    sb = wave_sum_g(sb);
    sx = wave_sum_g(sx);
    if (lane == 0) {
        nrm[v] = sb;
        snorm[v] = sqrtf(sx);
    }
}

// Screen of one 128 x 128 tile (I, J), I <= J, four waves of 64 x 64.  Writes flags[t64]
// (1: some pair of the 64 x 64 sub-tile may be near) for every sub-tile on or above the
// diagonal, so the flag array needs no clearing between calls.
template <int D>
__global__ __launch_bounds__(256) void k_gram_screen(const __bf16 *__restrict__ Xb,
                                                     const float *__restrict__ nrm,
                                                     const float *__restrict__ snorm, int n, int nt128,
                                                     long long items, long long per_xcd, long long nb64,
                                                     float theta0, unsigned char *__restrict__ flags) {
    constexpr int S = D + 8;  // padded LDS row stride (bf16): rows fall on different banks
    __shared__ __attribute__((aligned(16))) __bf16 As[128 * S];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[128 * S];
    __shared__ float hA[128], hB[128];
    __shared__ float red[2][4];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const long long t = (blockIdx.x % kXcdG) * per_xcd + blockIdx.x / kXcdG;
    if (t >= items) return;
    int I, J;
    tile_of_g(t, nt128, I, J);
    const int r0 = I * 128, c0 = J * 128;

    // stage the two 128-row slabs of X~ (16-byte chunks), zero beyond n
    constexpr int CH = D / 8;  // 16-byte chunks per row
    for (int q = tid; q < 128 * CH; q += 256) {
        int row = q / CH, ch = q - row * CH;
        bf16x8 va = {}, vb = {};
        if (r0 + row < n) va = *reinterpret_cast<const bf16x8 *>(Xb + (size_t)(r0 + row) * D + ch * 8);
        if (c0 + row < n) vb = *reinterpret_cast<const bf16x8 *>(Xb + (size_t)(c0 + row) * D + ch * 8);
        *reinterpret_cast<bf16x8 *>(As + row * S + ch * 8) = va;
        *reinterpret_cast<bf16x8 *>(Bs + row * S + ch * 8) = vb;
    }
    // theta of this tile from the largest |x| among its rows and among its columns
    float sa = 0.0f, sb = 0.0f;
    if (tid < 128) {
        sa = (r0 + tid < n) ? snorm[r0 + tid] : 0.0f;
    } else {
        sb = (c0 + tid - 128 < n) ? snorm[c0 + tid - 128] : 0.0f;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sa = fmaxf(sa, __shfl_xor(sa, off, 64));
        sb = fmaxf(sb, __shfl_xor(sb, off, 64));
    }
    if (lane == 0) red[0][wave] = sa, red[1][wave] = sb;
    __syncthreads();
    const float smaxA = fmaxf(red[0][0], red[0][1]);
    const float smaxB = fmaxf(red[1][2], red[1][3]);
    const float th = theta0 + 0.0078125f * (smaxA + smaxB);  // 2^-7
    const float q4 = 0.25f * th * th;
    if (tid < 128) {
        hA[tid] = (r0 + tid < n) ? 0.5f * nrm[r0 + tid] - q4 : INFINITY;
    } else {
        hB[tid - 128] = (c0 + tid - 128 < n) ? 0.5f * nrm[c0 + tid - 128] - q4 : INFINITY;
    }
    __syncthreads();

    const int wr = wave >> 1, wc = wave & 1;
    const long long R64 = 2LL * I + wr, C64 = 2LL * J + wc;
    if (R64 > C64 || C64 >= nb64) return;  // below the diagonal or past the last block

    floatx16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const int lrow = lane & 31, lk = (lane >> 5) * 8;
#pragma unroll
    for (int kk = 0; kk < D; kk += 16) {
        bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(As + (wr * 64 + lrow) * S + kk + lk);
        bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(As + (wr * 64 + 32 + lrow) * S + kk + lk);
        bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(Bs + (wc * 64 + lrow) * S + kk + lk);
        bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(Bs + (wc * 64 + 32 + lrow) * S + kk + lk);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    // accumulator r of lane l: row (r/4)*8 + (l/32)*4 + r%4, column l%32 of the 32 x 32 block
    const bool diag = (R64 == C64);
    bool near = false;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int jl = wc * 64 + b * 32 + (lane & 31);
        const float hj = hB[jl];
        const int jg = c0 + jl;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int il = wr * 64 + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                bool hit = (acc[a][b][r] - hA[il]) > hj;
                if (diag) hit = hit && (r0 + il < jg);
                near = near || hit;
            }
        }
    }
    const bool any = __ballot(near) != 0ull;
    if (lane == 0) flags[upper_index(R64, C64, nb64)] = any ? 1 : 0;
}

// Ordered compaction of the flags: list[0..count) = indices of flagged 64 x 64 tiles in
// increasing order (deterministic tile order for the exact pass and its loss partials).
// Thread t owns a contiguous range of 16-byte words; all-zero words (the common case) are
// skipped with one compare.  The flag region is 16-byte aligned; bytes past `total` are
// ignored.
constexpr int kCompactThreads = 1024;

__device__ __forceinline__ int flags_in_word(const uint4 &w, long long base, long long total) {
    int c = 0;
    const unsigned v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 16; ++q)
        c += (base + q < total && ((v[q >> 2] >> (8 * (q & 3))) & 0xffu)) ? 1 : 0;
    return c;
}

__global__ __launch_bounds__(kCompactThreads) void k_compact(const unsigned char *__restrict__ flags,
                                                             long long total, int *__restrict__ list,
                                                             int *__restrict__ count) {
    __shared__ int scan[kCompactThreads];
    const int tid = threadIdx.x;
    const uint4 *fw = reinterpret_cast<const uint4 *>(flags);
    const long long nw = (total + 15) / 16;
    const long long chunk = (nw + kCompactThreads - 1) / kCompactThreads;
    const long long lo = std::min<long long>(nw, (long long)tid * chunk);
    const long long hi = std::min<long long>(nw, lo + chunk);
    int c = 0;
    for (long long q = lo; q < hi; ++q) {
        uint4 w = fw[q];
        if (w.x | w.y | w.z | w.w) c += flags_in_word(w, q * 16, total);
    }
    scan[tid] = c;
    __syncthreads();
    for (int off = 1; off < kCompactThreads; off <<= 1) {  // inclusive Hillis-Steele scan
        int v = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    int pos = scan[tid] - c;
    for (long long q = lo; q < hi; ++q) {
        uint4 w = fw[q];
        if (!(w.x | w.y | w.z | w.w)) continue;
        const unsigned v[4] = {w.x, w.y, w.z, w.w};
        for (int b = 0; b < 16; ++b)
            if (q * 16 + b < total && ((v[b >> 2] >> (8 * (b & 3))) & 0xffu)) list[pos++] = (int)(q * 16 + b);
    }
    if (tid == kCompactThreads - 1) *count = scan[tid];
}

}  // namespace gempe

using namespace gempe;

hipError_t gempe_launch_gram_screen(const gempe_graph_s *g, int d, const float *X, void *Xb, float *nrm,
                                    float *snorm, unsigned char *flags, int *list, int *count, float theta0,
                                    hipStream_t s) {
    const int n = g->n;
    hipLaunchKernelGGL(k_prep_bf16, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, d,
                       reinterpret_cast<__bf16 *>(Xb), nrm, snorm);
    const int nt128 = (n + 127) / 128;
    const long long items = (long long)nt128 * (nt128 + 1) / 2;
    const long long per = (items + kXcdG - 1) / kXcdG;
    const long long nb64 = (n + 63) / 64;
    const __bf16 *xb = reinterpret_cast<const __bf16 *>(Xb);
    dim3 grid((unsigned)(per * kXcdG)), block(256);
    switch (d) {
        case 16: hipLaunchKernelGGL(k_gram_screen<16>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        case 32: hipLaunchKernelGGL(k_gram_screen<32>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        case 48: hipLaunchKernelGGL(k_gram_screen<48>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        case 64: hipLaunchKernelGGL(k_gram_screen<64>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        case 80: hipLaunchKernelGGL(k_gram_screen<80>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        case 96: hipLaunchKernelGGL(k_gram_screen<96>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        case 112: hipLaunchKernelGGL(k_gram_screen<112>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
        default: hipLaunchKernelGGL(k_gram_screen<128>, grid, block, 0, s, xb, nrm, snorm, n, nt128, items, per, nb64, theta0, flags); break;
    }
    const long long t64 = nb64 * (nb64 + 1) / 2;
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, s, flags, t64, list, count);
    return hipGetLastError();
}
