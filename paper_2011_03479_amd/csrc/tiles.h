// Device helpers shared by the sweeps, the edge passes, the sampled step and the distance
// histogram: the upper-triangle tile order, the XCD-aware workgroup mapping, the DPP wave
// rotation of the Latin-square schedule, segmented row sums, and the squared distances.
#pragma once

#include <hip/hip_runtime.h>

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

// Sharding of the upper triangle over several devices: strips p and nt-1-p (of rows p T and
// (nt-1-p) T, T the plan's tile edge) form strip pair min(p, nt-1-p), nt + 1 tiles together
// (the middle strip of an odd nt alone has nt - p); shard s of G owns the pairs p with
// p mod G == s, so every shard gets about the same number of pairs.
__device__ inline bool strip_owned(int I, int nt, int s, int G) {
    const int p = min(I, nt - 1 - I);
    return p % G == s;
}

// Tile (I, J) of item t: all upper-triangle tiles when G == 1 (tile_of), else the t-th tile
// of shard s (its strip pairs in increasing order, strip p's tiles first).
__device__ inline void item_tile(long long t, int nt, int s, int G, int &I, int &J) {
    if (G <= 1) {
        tile_of(t, nt, I, J);
        return;
    }
    const long long per = (long long)nt + 1;
    const long long q = t / per;
    const int p = s + (int)q * G;
    const int off = (int)(t - q * per);
    const int first = nt - p;  // tiles of strip p
    if (off < first) {
        I = p;
        J = p + off;
    } else {
        I = nt - 1 - p;
        J = I + (off - first);
    }
}

// Workgroup b -> tile index such that the workgroups one XCD receives (b = x, x+8, ...)
// take consecutive tiles (same row strip: x_I stays in that XCD's L2).
__device__ inline long long xcd_item(long long b, long long per_xcd) {
    return (b % kXcd) * per_xcd + b / kXcd;
}

__device__ __forceinline__ float rot1(float v) {
    // DPP wave rotation by one lane, in place (all rows and banks enabled)
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x134, 0xF, 0xF, false));
}

// The same rotation written so that the compiler folds it into the consuming add
// (v_add_f32_dpp): every source lane is valid for a wave rotation.
__device__ __forceinline__ float rot1_fold(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF, true));
}

// +1 if the rotation brings lane l+1's value to lane l, else -1.
__device__ __forceinline__ int rot_dir(int lane) {
    return (__float_as_int(rot1(__int_as_float(lane))) == ((lane + 1) & 63)) ? 1 : -1;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Lanes hold values keyed by a row id that is non-decreasing across the active lanes of the
// wave (CSR order; inactive lanes carry key -1).  Sums each run of equal keys into its first
// lane (segmented suffix sums, log2(64) shuffle steps) and returns true in those head
// lanes, so a hub row costs one atomic per wave instead of one per entry.
__device__ __forceinline__ bool seg_sum_to_head(int key, int lane, float &v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int ko = __shfl_down(key, off, 64);
        float vo = __shfl_down(v, off, 64);
        if (lane + off < 64 && ko == key) v += vo;
    }
    int kp = __shfl_up(key, 1, 64);
    return key >= 0 && (lane == 0 || kp != key);
}

// Sum over the 16 lanes of each DPP row, returned in all 16: rotations by 8 and 4 lanes, then
// exchanges within quads.  Each step adds two values that the partner lane adds in the
// other order, so every lane of the row ends with the same bits.  Call with the whole wave
// active.
__device__ __forceinline__ float row16_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, true));  // row_ror:8
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, true));  // row_ror:4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));   // quad 2,3,0,1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));   // quad 1,0,3,2
    return v;
}

// Squared distance of two rows by a group of 16 lanes (one DPP row): lane s of the group
// holds coordinates s, s+16, ..., s+16(C-1) of x_i in xi (zero past d), loads the same
// coordinates of x_j, sums its C squared differences in order with fused multiply-adds, and
// row16_sum combines the 16 partial sums.  The wide edge pass and the exact near-pair pass
// of the BF16 path both use it, so a pair they share gets the same bits in both.
template <int C>
__device__ __forceinline__ float group16_sqdist(const float (&xi)[C], const float *__restrict__ xj, int sub, int d,
                                                float (&df)[C]) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int c = sub + 16 * k;
        df[k] = xi[k] - (c < d ? xj[c] : 0.0f);
        s = __builtin_fmaf(df[k], df[k], s);
    }
    return row16_sum(s);
}

// The same sum started from FLT_MIN instead of 0: positive for coincident points (so the
// table pair function's rsq stays finite) and equal to sqdist wherever sqdist > 2^-101.
// The d <= 16 sweeps and their edge corrections use it, so both see the same bits.
template <int D>
__device__ __forceinline__ float sqdist_eps(const float (&a)[D], const float (&b)[D], float (&diff)[D]) {
    float r2 = 1.17549435e-38f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        diff[k] = a[k] - b[k];
        r2 = __builtin_fmaf(diff[k], diff[k], r2);
    }
    return r2;
}

// Squared distance, coordinates in order with fused multiply-adds (padding coordinates are
// zero on both sides and add exactly 0).
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

}  // namespace gempe
