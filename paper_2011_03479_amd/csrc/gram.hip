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
// The test uses one theta per pair of 128-vertex blocks (the largest |x| of each block),
// which only makes it stricter, and is evaluated as G~ - n~_i/2 > n~_j/2 - theta^2/2,
// two VALU operations per pair.  Flagged sub-tiles are compacted in
// tile order and recomputed exactly in FP32 by the LDS sweep (k_sweep_wide over the
// list); every other non-edge pair has delta >= mu + near_k sigma and is flushed: it
// contributes less than -log2 Phi(-near_k) bits (< 2e-19 at near_k = 9) and a gradient
// coefficient of the same order.  Edges are always recomputed exactly by the edge pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "internal.h"
#include "ltab_stage.h"
#include "pairfn.h"
#include "tiles.h"

namespace gempe {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ long long upper_index(long long r, long long c, long long nt) {
    return r * nt - r * (r - 1) / 2 + (c - r);
}

__device__ __forceinline__ float wave_sum_g(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per vertex: X~ = bf16(X) (round to nearest even), n~ = |x~|^2 (FP32 from the
// rounded values), s = |x| (FP32, from the unrounded coordinates).  A vertex with a
// non-finite coordinate gets s = +inf: every tile it touches then counts as near, so the
// exact pass sees (and reports) the non-finite value instead of the screen flushing it.
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
        snorm[v] = isfinite(sx) ? sqrtf(sx) : INFINITY;
    }
}

// Largest |x| of every 128-vertex block (for the per-tile threshold of the screen).
__global__ __launch_bounds__(128) void k_blockmax(const float *__restrict__ snorm, int n,
                                                  float *__restrict__ smax128, int *__restrict__ sample) {
    __shared__ float w[2];
    if (sample && blockIdx.x == 0 && threadIdx.x < 2) sample[threadIdx.x] = 0;  // the route sample's counts
    const int v = blockIdx.x * 128 + threadIdx.x;
    float s = v < n ? snorm[v] : 0.0f;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s = fmaxf(s, __shfl_xor(s, off, 64));
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) smax128[blockIdx.x] = fmaxf(w[0], w[1]);
}

// Screen of a strip of 64 RW rows against column tiles of 64 CW columns (CW = 8 / RW):
// item I*Q + q takes the tiles J = J0 + q, J0 + q + Q, ... (J0: the first tile reaching the
// strip's diagonal).  Wave w owns the 64 x 64 sub-tile (w / CW, w % CW) of every step: it
// keeps the BF16 fragments of its 64 rows in registers for the whole item, and the column
// tiles stream through two LDS buffers, the next tile's global loads issued before the
// current tile's MFMAs.  A strip of 512 rows (RW = 8) reads each column tile once per 512
// rows, a quarter of the global traffic of 128-row strips (RW = 2), which is what keeps the
// MFMAs fed at large n; RW = 2 gives more workgroups when n is small.  Eight waves of up to
// 256 registers: two per SIMD, so one wave's MFMAs cover the other's waits.  Writes
// flags[t64] (1: some pair of the 64 x 64 sub-tile may be near) for every sub-tile on or
// above the diagonal, so the flags need no clearing between calls.
// The route sample runs the same kernel on every sstride-th strip, one item per strip (qb = 1)
// with a column step Q larger than the screen's and a phase that turns from strip to strip,
// and counts its sub-tiles and their flags into sample[0..1].  The screen after it returns at once when gate (those counts) shows more than
// half of the sampled sub-tiles flagged: the full matrix-core sweep then takes every pair.
constexpr int kScreenThreads = 512;

// More than half of the route sample's sub-tiles flagged (read by every kernel it gates).
__device__ __forceinline__ bool sample_dense(const int *sample) {
    return sample && 2LL * sample[0] > (long long)sample[1];
}

template <int D, int RW>
__global__ __launch_bounds__(kScreenThreads) void k_gram_screen(const __bf16 *__restrict__ Xb,
                                                     const float *__restrict__ nrm,
                                                     const float *__restrict__ smax128, int n, int ntile,
                                                     int Q, long long nb64, float theta0,
                                                     unsigned char *__restrict__ flags, int qb, int sstride,
                                                     const int *__restrict__ gate, int *__restrict__ sample) {
    if (sample_dense(gate)) return;  // uniform over the grid
    constexpr int CW = 8 / RW;
    constexpr int S = D + 8;   // padded LDS row stride (bf16): rows fall on different banks
    constexpr int CH = D / 8;  // 16-byte chunks per row
    constexpr int TC = 64 * CW;  // columns per tile
    constexpr int NT = kScreenThreads;
    constexpr int PER = (TC * CH + NT - 1) / NT;  // chunks each thread stages per tile
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TC * S];
    __shared__ float hN[2][TC], hS[2][TC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: branches stay scalar
    // the screen: qb = Q items per strip, phases q = 0 .. Q - 1; the sample: one item per
    // strip, its phase turning with the strip, so that every column tile is equally likely
    const int I = (int)(blockIdx.x / qb) * sstride, q = (int)(blockIdx.x % Q);
    int J = (I * RW) / CW + q;
    if (J >= ntile) return;  // uniform over the workgroup
    const int wr = wave / CW, wc = wave % CW;
    const long long R64 = (long long)I * RW + wr;  // this wave's row block (>= nb64: no rows)

    // Operands come in through raw buffer loads: the descriptor's record count is the n x D
    // matrix, so rows past n read as zero without a compare, the per-thread offset is one
    // register and the tile/chunk step goes into the scalar offset.
    const __amdgpu_buffer_rsrc_t xrs =
        __builtin_amdgcn_make_buffer_rsrc((void *)Xb, (short)0, n * D * (int)sizeof(__bf16), 0x00020000);
    const int voff = ((tid / CH) * D + (tid % CH) * 8) * (int)sizeof(__bf16);
    auto stage = [&](int Jt, bf16x8 (&regs)[PER]) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            if (tid + p * NT < TC * CH) {
                const int soff = (Jt * TC + p * (NT / CH)) * D * (int)sizeof(__bf16);
                const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(xrs, voff, soff, 0);
                regs[p] = __builtin_bit_cast(bf16x8, v);
            } else {
                regs[p] = bf16x8{};
            }
        }
    };
    auto commit = [&](int Jt, int buf, const bf16x8 (&regs)[PER]) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int c = tid + p * NT;
            const int row = c / CH, ch = c - row * CH;
            if (c < TC * CH) *reinterpret_cast<bf16x8 *>(&Bs[buf][row * S + ch * 8]) = regs[p];
        }
        if (tid < TC) {
            const int c = Jt * TC + tid;
            hN[buf][tid] = c < n ? nrm[c] : 0.0f;
            hS[buf][tid] = smax128[min(c, n - 1) / 128];
        }
    };

    // this wave's rows: fragments, row terms and the 128-row block's largest |x|
    const int lrow = lane & 31, lk = (lane >> 5) * 8;
    bf16x8 afr[D / 16][2];
#pragma unroll
    for (int kk = 0; kk < D / 16; ++kk)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int row = (int)R64 * 64 + a * 32 + lrow;
            const int off = (row * D + kk * 16 + lk) * (int)sizeof(__bf16);
            afr[kk][a] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(xrs, off, 0, 0));
        }
    // -n~_i / 2 in accumulator layout: the MFMA chains start from it, so they end at
    // G~_ij - n~_i / 2 (rows past n: -inf, never near)
    floatx16 nha[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const long long ig = R64 * 64 + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
            nha[a][r] = ig < n ? -(0.5f * nrm[ig]) : -INFINITY;
        }
    const float sI = R64 < nb64 ? smax128[R64 / 2] : 0.0f;
    // Per step a wave computes its 64 x 64 sub-tile of column tile Jt (LDS buffer cur) into
    // acc and reads the columns' thresholds from LDS (the buffer is refilled after the next
    // barrier); the epilogue reduces acc to the sub-tile's flag.  The first four waves run
    // the epilogue right after their MFMAs, the last four run it at the start of the next
    // step, before their MFMAs: the two waves that share a SIMD then reduce while the other
    // one multiplies, instead of both leaving the matrix core idle at the same time.
    // (wave w runs on SIMD w % 4; the 128-row strips of the widest rows keep one order, the
    // second copy of the loop would not fit in the registers)
    constexpr bool kDesync = RW == 8 || D <= 80;
    const bool late = kDesync && wave >= 4;
    // acc = G~ - n~_i/2 over the sub-tile (R64, Jt * CW + wc), B fragments from LDS buffer cur
    auto mma_tile = [&](int cur, floatx16 (&acc)[2][2]) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = nha[a];
        const __bf16 *Bc = Bs[cur];
#pragma unroll
        for (int kk = 0; kk < D / 16; ++kk) {
            bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(Bc + (wc * 64 + lrow) * S + kk * 16 + lk);
            bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(Bc + (wc * 64 + 32 + lrow) * S + kk * 16 + lk);
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[kk][0], b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[kk][0], b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[kk][1], b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[kk][1], b1, acc[1][1], 0, 0, 0);
        }
    };
    // near test G~ - n~_i/2 > n~_j/2 - theta^2/2  <=>  delta~^2 < theta^2, where theta
    // carries the 2^-7 (|x_i| + |x_j|) margin of the two 128-vertex blocks: the right side
    // for this lane's column of half b of the sub-tile column
    auto threshold = [&](int Jt, int cur, int b) __attribute__((always_inline)) {
        const int jl = wc * 64 + b * 32 + (lane & 31);
        const float th = theta0 + 0.0078125f * (sI + hS[cur][jl]);
        return Jt * TC + jl < n ? 0.5f * hN[cur][jl] - 0.5f * th * th : INFINITY;
    };
    // flag of sub-tile (R64, C64) of column tile Jt from its accumulators
    auto epilogue = [&](const floatx16 (&acc)[2][2], long long C64, int Jt, auto hb_of) __attribute__((always_inline)) {
        // accumulator r of lane l: row (r/4)*8 + (l/32)*4 + r%4, column l%32 of the block,
        // holding G~ - n~_i/2; the test is taken on the lane's largest value (one compare
        // per column)
        const bool diag = (R64 == C64);
        bool near = false;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int jg = Jt * TC + wc * 64 + b * 32 + (lane & 31);
            float m = -INFINITY;
            if (diag) {  // only pairs i < j of a diagonal sub-tile
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int ig = (int)R64 * 64 + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                        m = fmaxf(m, ig < jg ? acc[a][b][r] : -INFINITY);
                    }
            } else {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int r = 0; r < 16; ++r) m = fmaxf(m, acc[a][b][r]);
            }
            near = near || (m > hb_of(b));
        }
        const bool any = __ballot(near) != 0ull;
        if (lane == 0) {
            flags[upper_index(R64, C64, nb64)] = any ? 1 : 0;
            if (sample) {
                atomicAdd(&sample[0], any ? 1 : 0);
                atomicAdd(&sample[1], 1);
            }
        }
    };
    // the late waves' sub-tile held over to the next step, with its thresholds (its LDS
    // buffer is refilled after the next barrier)
    floatx16 hacc[2][2];
    float hb[2];
    long long hC64 = -1;  // -1: none
    int hJ = 0;
    auto held_epilogue = [&]() __attribute__((always_inline)) {
        if (hC64 >= 0) epilogue(hacc, hC64, hJ, [&](int b) { return hb[b]; });
        hC64 = -1;
    };
    // the step loop, compiled once per wave group so that each copy keeps only the
    // registers its own order needs
    auto run = [&](auto late_tag) __attribute__((always_inline)) {
        constexpr bool kLate = decltype(late_tag)::value;
        auto screen_tile = [&](int Jt, int cur) __attribute__((always_inline)) {
            const long long C64 = (long long)Jt * CW + wc;  // this wave's sub-tile column
            const bool live = R64 <= C64 && C64 < nb64;
            if constexpr (kLate) {
                held_epilogue();
                if (live) {
                    mma_tile(cur, hacc);
                    hb[0] = threshold(Jt, cur, 0);
                    hb[1] = threshold(Jt, cur, 1);
                    hC64 = C64;
                    hJ = Jt;
                }
            } else if (live) {
                floatx16 acc[2][2];
                mma_tile(cur, acc);
                epilogue(acc, C64, Jt, [&](int b) { return threshold(Jt, cur, b); });
            }
        };

        if constexpr (PER <= 2) {
            // global loads two steps ahead (two staging register sets): a load has a whole step
            // of MFMAs more to arrive before its commit
            bf16x8 ra[PER], rb[PER];
            stage(J, ra);
            commit(J, 0, ra);
            if (J + Q < ntile) stage(J + Q, ra);
            __syncthreads();
            for (;;) {
                // tile J in buffer 0, tile J + Q arriving in ra
                if (J + 2 * Q < ntile) stage(J + 2 * Q, rb);
                screen_tile(J, 0);
                if (J + Q < ntile) commit(J + Q, 1, ra);
                __syncthreads();
                J += Q;
                if (J >= ntile) break;
                // tile J in buffer 1, tile J + Q arriving in rb
                if (J + 2 * Q < ntile) stage(J + 2 * Q, ra);
                screen_tile(J, 1);
                if (J + Q < ntile) commit(J + Q, 0, rb);
                __syncthreads();
                J += Q;
                if (J >= ntile) break;
            }
        } else {
            {
                bf16x8 regs[PER];
                stage(J, regs);
                commit(J, 0, regs);
            }
            __syncthreads();
            for (int it = 0; J < ntile; ++it, J += Q) {
                const int cur = it & 1;
                const int Jn = J + Q;
                bf16x8 regs[PER];
                if (Jn < ntile) stage(Jn, regs);
                screen_tile(J, cur);
                // buffer cur ^ 1 was last read in the previous step, which every wave finished
                // before that step's closing barrier: commit into it without waiting
                if (Jn < ntile) commit(Jn, cur ^ 1, regs);
                __syncthreads();
            }
        }
        if constexpr (kLate) held_epilogue();  // the last sub-tile
    };
    if constexpr (kDesync) {
        if (late)
            run(std::true_type{});
        else
            run(std::false_type{});
    } else {
        run(std::false_type{});
    }
}

// Ordered compaction of the flags: list[0..count) = indices of flagged 64 x 64 tiles in
// increasing order (deterministic tile order for the exact pass and its loss partials).
// Thread t owns a contiguous range of 16-byte words; all-zero words (the common case) are
// skipped with one compare.  The flag region is 16-byte aligned; bytes past `total` are
// ignored.

__device__ __forceinline__ int flags_in_word(const uint4 &w, long long base, long long total) {
    int c = 0;
    const unsigned v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 16; ++q)
        c += (base + q < total && ((v[q >> 2] >> (8 * (q & 3))) & 0xffu)) ? 1 : 0;
    return c;
}

// Ordered compaction of the tile flags in three steps: per-chunk counts (one workgroup per
// 4,096 flags), an exclusive scan of the chunk counts, per-chunk writes at the chunk's offset.
// The list comes out in increasing tile order, so everything downstream is deterministic.
constexpr int kChunkFlags = 4096;  // 256 threads x 16 flags (one uint4 each)

__global__ __launch_bounds__(256) void k_flag_count(const unsigned char *__restrict__ flags, long long total,
                                                    int *__restrict__ chunk_count, const int *__restrict__ gate) {
    if (sample_dense(gate)) return;
    __shared__ int ws[4];
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;  // uint4 word index
    int c = 0;
    if (q * 16 < total) {
        const uint4 w = reinterpret_cast<const uint4 *>(flags)[q];
        if (w.x | w.y | w.z | w.w) c = flags_in_word(w, q * 16, total);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) chunk_count[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(1024) void k_flag_scan(int *__restrict__ chunk_count, int chunks, int *__restrict__ count,
                                                    const int *__restrict__ gate) {
    if (sample_dense(gate)) return;
    __shared__ int sc[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < chunks; base += 1024) {
        const int k = base + threadIdx.x;
        const int v = k < chunks ? chunk_count[k] : 0;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
            const int u = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
            __syncthreads();
            sc[threadIdx.x] += u;
            __syncthreads();
        }
        if (k < chunks) chunk_count[k] = carry + sc[threadIdx.x] - v;  // exclusive offset
        __syncthreads();
        if (threadIdx.x == 1023) carry += sc[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

__global__ __launch_bounds__(256) void k_flag_write(const unsigned char *__restrict__ flags, long long total,
                                                    const int *__restrict__ chunk_offset, int *__restrict__ list,
                                                    const int *__restrict__ gate) {
    if (sample_dense(gate)) return;
    __shared__ int sc[256];
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    uint4 w = {0u, 0u, 0u, 0u};
    int c = 0;
    if (q * 16 < total) {
        w = reinterpret_cast<const uint4 *>(flags)[q];
        if (w.x | w.y | w.z | w.w) c = flags_in_word(w, q * 16, total);
    }
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int u = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
        __syncthreads();
        sc[threadIdx.x] += u;
        __syncthreads();
    }
    if (!c) return;
    int pos = chunk_offset[blockIdx.x] + sc[threadIdx.x] - c;
    const unsigned v[4] = {w.x, w.y, w.z, w.w};
    for (int b = 0; b < 16; ++b)
        if (q * 16 + b < total && ((v[b >> 2] >> (8 * (b & 3))) & 0xffu)) list[pos++] = (int)(q * 16 + b);
}

// ------------------------------------------------------------------------------------
// The flagged tiles, one wave each in list order: the tile's BF16 Gram block is recomputed
// on MFMA with the screen's operands, starting values, accumulation order and threshold, so the near test
// picks exactly the pairs the screen saw.  A tile with at most kSparseNear near pairs is
// finished here: its near pairs are listed in a fixed order and evaluated exactly in FP32,
// four at a time, each by a group of 16 lanes (coordinates over lanes, group16_sqdist, the
// squared distance of the wide edge pass, so an edge among them gets bit-identical non-edge
// values there); the tile's loss goes to partial slot q.
// A denser tile is marked for the exact tile pass (k_sweep_wide_list), which writes slot q.
// ------------------------------------------------------------------------------------
constexpr int kSparseNear = 128;
constexpr int kNearTileGrid = 1024;

template <int D, int EX>
__global__ __launch_bounds__(256) void k_near_tiles(const __bf16 *__restrict__ Xb, const float *__restrict__ X,
                                                    const float *__restrict__ nrm,
                                                    const float *__restrict__ smax128, int n, long long nb64,
                                                    float theta0, const int *__restrict__ list,
                                                    int *__restrict__ count, gempe::PairParams P,
                                                    float *__restrict__ G, float *__restrict__ extra,
                                                    float *__restrict__ partials,
                                                    unsigned char *__restrict__ dense, int all_dense,
                                                    int *__restrict__ all_dense_flag, const int *__restrict__ sample,
                                                    int full_items) {
    if (sample_dense(sample)) {
        // the route sample found most tiles flagged and the screen did not run: the full
        // sweep writes loss slots [0, full_items), which the reduction then sums
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *all_dense_flag = 1;
            *count = full_items;
        }
        return;
    }
    __shared__ int near[4][kSparseNear];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lrow = lane & 31, lk = (lane >> 5) * 8;
    const int cnt = *count;
    // when the caller allows it (all_dense != 0) and most tiles are flagged (d = 16 from a
    // spread start, or a contracted embedding at any d: nearly every pair lies within the near
    // distance), no flagged tile is recomputed here only to be found dense: mode 1 hands each
    // to the dense list pass, mode 2 leaves every pair to the full matrix-core sweep
    if (all_dense && 2LL * cnt > nb64 * (nb64 + 1) / 2) {
        for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < cnt; q += (long long)gridDim.x * 256) {
            if (all_dense == 1)
                dense[q] = 1;
            else
                partials[q] = 0.0f;  // the full sweep writes its own slots below cnt
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) *all_dense_flag = all_dense == 2 ? 1 : 0;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *all_dense_flag = 0;
    // d = 16 takes the non-edge value from the table, as the dense pass and the edge pass do
    __shared__ float4 ltab[D == 16 ? gempe::kLtabF4 : 1];
    if (D == 16) {
        gempe::stage_ltab(ltab);
        __syncthreads();
    }
    for (int q = blockIdx.x * 4 + wave; q < cnt; q += gridDim.x * 4) {
        int R64, C64;
        gempe::tile_of(list[q], (int)nb64, R64, C64);
        floatx16 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ig = R64 * 64 + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                acc[a][0][r] = acc[a][1][r] = ig < n ? -(0.5f * nrm[ig]) : -INFINITY;
            }
#pragma unroll
        for (int kk = 0; kk < D / 16; ++kk) {
            bf16x8 a0 = {}, a1 = {}, b0 = {}, b1 = {};
            const int ra = R64 * 64 + lrow, rb = C64 * 64 + lrow;
            if (ra < n) a0 = *reinterpret_cast<const bf16x8 *>(Xb + (size_t)ra * D + kk * 16 + lk);
            if (ra + 32 < n) a1 = *reinterpret_cast<const bf16x8 *>(Xb + (size_t)(ra + 32) * D + kk * 16 + lk);
            if (rb < n) b0 = *reinterpret_cast<const bf16x8 *>(Xb + (size_t)rb * D + kk * 16 + lk);
            if (rb + 32 < n) b1 = *reinterpret_cast<const bf16x8 *>(Xb + (size_t)(rb + 32) * D + kk * 16 + lk);
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
        // the screen's threshold: strip of 128 rows I = R64 / 2, column block of 128
        const float sI = smax128[R64 / 2];
        float hb[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int c = C64 * 64 + b * 32 + lrow;
            const float th = theta0 + 0.0078125f * (sI + smax128[min(c, n - 1) / 128]);
            hb[b] = c < n ? 0.5f * nrm[c] - 0.5f * th * th : INFINITY;
        }
        // the decisions as bits (a, b, r) -> 32 a + 16 b + r of a per-lane mask
        unsigned long long dbits = 0ull;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ig = R64 * 64 + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int jg = C64 * 64 + b * 32 + lrow;
                    const bool nr = ig < jg && acc[a][b][r] > hb[b];
                    dbits |= (unsigned long long)nr << (32 * a + 16 * b + r);
                }
            }
        const int c = __popcll(dbits);
        int tot = c;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
        float loss = 0.0f;
        if (tot > kSparseNear) {
            if (lane == 0) dense[q] = 1;
        } else {
            if (lane == 0) dense[q] = 0;
            // list the near pairs as 6+6-bit local (row, column) codes, lane by lane (each
            // lane's decisions in bit order from its exclusive prefix count on); the list is
            // read back only by this wave
            int pos = c;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(pos, off, 64);
                if (lane >= off) pos += t;
            }
            pos -= c;
            const int npair = tot;
            while (dbits) {
                const int k = __builtin_ctzll(dbits);
                dbits &= dbits - 1ull;
                const int a = k >> 5, b = (k >> 4) & 1, r = k & 15;
                const int li = a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                near[wave][pos++] = (li << 6) | (b * 32 + lrow);
            }
            __builtin_amdgcn_wave_barrier();
            // four pairs at a time, one per group of 16 lanes
            const int grp = lane >> 4, sub = lane & 15;
            constexpr int C = D / 16;
            float lsum = 0.0f;
            for (int p0 = 0; p0 < npair; p0 += 4) {
                const bool valid = p0 + grp < npair;
                const int code = near[wave][valid ? p0 + grp : p0];
                const int i = R64 * 64 + (code >> 6), j = C64 * 64 + (code & 63);
                float xr[C], df[C];
#pragma unroll
                for (int k = 0; k < C; ++k) xr[k] = X[(size_t)i * D + sub + 16 * k];
                const float r2 = gempe::group16_sqdist<C>(xr, X + (size_t)j * D, sub, D, df);
                float dl, cc, w = 0.0f;
                if (D == 16)
                    gempe::nonedge_eval<EX == 2>(r2 + gempe::kFltMin, P, ltab, gempe::table_offset(P, gempe::kLtabZero),
                                                 gempe::kLtabSegs, dl, cc, w);
                else
                    gempe::pair_eval_t<EX == 2>(r2, 1.0f, P, dl, cc, w);
                if (valid) {
#pragma unroll
                    for (int k = 0; k < C; ++k) {
                        atomicAdd(&G[(size_t)i * D + sub + 16 * k], cc * df[k]);
                        atomicAdd(&G[(size_t)j * D + sub + 16 * k], -(cc * df[k]));
                    }
                    if (sub == 0) {
                        lsum += dl;
                        if (EX) {
                            const float ex = (EX == 2) ? w : dl;
                            atomicAdd(&extra[i], ex);
                            atomicAdd(&extra[j], ex);
                        }
                    }
                }
            }
            // the four groups' sums in a fixed order
            loss = ((lsum + __shfl(lsum, 16, 64)) + __shfl(lsum, 32, 64)) + __shfl(lsum, 48, 64);
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) partials[q] = loss;
    }
}

}  // namespace gempe

using namespace gempe;

hipError_t gempe_launch_gram_screen(const gempe_graph_s *g, int d, const float *X, void *Xb, float *nrm,
                                    float *snorm, float *smax128, unsigned char *flags, int *list, int *count,
                                    float theta0, int *chunk, hipStream_t s, int *sample) {
    const int n = g->n;
    hipLaunchKernelGGL(k_prep_bf16, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, d,
                       reinterpret_cast<__bf16 *>(Xb), nrm, snorm);
    const int nt128 = (n + 127) / 128;
    hipLaunchKernelGGL(k_blockmax, dim3((unsigned)nt128), dim3(128), 0, s, snorm, n, smax128, sample);
    const long long nb64 = (n + 63) / 64;
    const __bf16 *xb = reinterpret_cast<const __bf16 *>(Xb);
    // 512-row strips once there are enough of them to fill the chip with Q = 8 column
    // phases each, else 128-row strips; Q column tiles interleaved per strip
    const bool tall = (n + 511) / 512 >= 64;
    const int RW = tall ? 8 : 2, TC = 64 * (8 / RW);
    const int nstrip = (n + 64 * RW - 1) / (64 * RW), ntile = (n + TC - 1) / TC;
    const int Q = tall ? 8 : std::max(1, std::min(8, ntile / 2));
    // the route sample: about 32 strips spread over the matrix, each against every Qs-th
    // column tile right of its diagonal (phase k mod Qs for the k-th sampled strip)
    const int sstride = std::max(1, nstrip / 32);
    const int Qs = std::max(Q, std::min(16 * Q, ntile / 8));
#define GEMPE_SCREEN_GRID(DD, G, QQ, QB, SS, GATE, SAMPLE)                                                      \
    do {                                                                                                        \
        if (tall)                                                                                               \
            hipLaunchKernelGGL((k_gram_screen<DD, 8>), G, dim3(kScreenThreads), 0, s, xb, nrm, smax128, n, ntile, \
                               QQ, nb64, theta0, flags, QB, SS, GATE, SAMPLE);                                 \
        else                                                                                                    \
            hipLaunchKernelGGL((k_gram_screen<DD, 2>), G, dim3(kScreenThreads), 0, s, xb, nrm, smax128, n, ntile, \
                               QQ, nb64, theta0, flags, QB, SS, GATE, SAMPLE);                                 \
    } while (0)
#define GEMPE_SCREEN(DD)                                                                                        \
    do {                                                                                                        \
        if (sample) {                                                                                           \
            GEMPE_SCREEN_GRID(DD, dim3((unsigned)((nstrip + sstride - 1) / sstride)), Qs, 1, sstride,           \
                              (const int *)nullptr, sample);                                                    \
        }                                                                                                       \
        TimedLaunches tl(kTkGram, s);                                                                           \
        GEMPE_SCREEN_GRID(DD, dim3((unsigned)((long long)nstrip * Q)), Q, Q, 1, (const int *)sample,             \
                          (int *)nullptr);                                                                      \
    } while (0)
    {
        switch (d) {
            case 16: GEMPE_SCREEN(16); break;
            case 32: GEMPE_SCREEN(32); break;
            case 48: GEMPE_SCREEN(48); break;
            case 64: GEMPE_SCREEN(64); break;
            case 80: GEMPE_SCREEN(80); break;
            case 96: GEMPE_SCREEN(96); break;
            case 112: GEMPE_SCREEN(112); break;
            default: GEMPE_SCREEN(128); break;
        }
    }
#undef GEMPE_SCREEN
#undef GEMPE_SCREEN_GRID
    const long long t64 = nb64 * (nb64 + 1) / 2;
    const int chunks = (int)((t64 + kChunkFlags - 1) / kChunkFlags);
    const int *gate = sample;
    hipLaunchKernelGGL(k_flag_count, dim3(chunks), dim3(256), 0, s, flags, t64, chunk, gate);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, s, chunk, chunks, count, gate);
    hipLaunchKernelGGL(k_flag_write, dim3(chunks), dim3(256), 0, s, flags, t64, chunk, list, gate);
    return hipGetLastError();
}

namespace {
template <int EX>
void launch_near_tiles_ex(const gempe_graph_s *g, int d, const float *X, const GramCtx &gc, const gempe::PairParams &P,
                          float *G, float *extra, float *partials, hipStream_t s, int all_dense,
                          const int *sample, int full_items) {
    const long long nb64 = (g->n + 63) / 64;
    const __bf16 *xb = reinterpret_cast<const __bf16 *>(gc.xb);
    const dim3 grid(kNearTileGrid), block(256);
#define GEMPE_NEAR(DD)                                                                                     \
    hipLaunchKernelGGL((k_near_tiles<DD, EX>), grid, block, 0, s, xb, X, gc.nrm, gc.smax128, g->n, nb64,  \
                       gc.theta0, gc.list, gc.count, P, G, extra, partials, gc.dense, all_dense, gc.all_dense, \
                       sample, full_items)
    switch (d) {
        case 16: GEMPE_NEAR(16); break;
        case 32: GEMPE_NEAR(32); break;
        case 48: GEMPE_NEAR(48); break;
        case 64: GEMPE_NEAR(64); break;
        case 80: GEMPE_NEAR(80); break;
        case 96: GEMPE_NEAR(96); break;
        case 112: GEMPE_NEAR(112); break;
        default: GEMPE_NEAR(128); break;
    }
#undef GEMPE_NEAR
}
}  // namespace

hipError_t gempe_launch_near_tiles(const gempe_graph_s *g, int d, const float *X, const GramCtx &gc,
                                   const PairParamsHost &h, int ex, float *G, float *extra, float *partials,
                                   hipStream_t s, int all_dense, const int *sample, int full_items) {
    const gempe::PairParams P{h.mu_s,   h.inv_sigma, h.c_neg,   h.c_pos,   h.tk_scale,
                              h.tk_off, h.slope_k,   h.r_scale, h.w_scale, h.wk2, h.table_full, 0};
    if (ex == 2)
        launch_near_tiles_ex<2>(g, d, X, gc, P, G, extra, partials, s, all_dense, sample, full_items);
    else if (ex == 1)
        launch_near_tiles_ex<1>(g, d, X, gc, P, G, extra, partials, s, all_dense, sample, full_items);
    else
        launch_near_tiles_ex<0>(g, d, X, gc, P, G, extra, partials, s, all_dense, sample, full_items);
    return hipGetLastError();
}
