// FP32 pair function of the GEMPE coding cost (device code).
//
// For a vertex pair at squared distance r2, with a = -1 for an edge and +1 otherwise,
//   tau = a (delta - mu) / sigma,  dl = -log2 Phi(tau)          (Sec. II-B, dl+/-)
//   d dl / d delta = -(a / (sigma ln 2)) R(tau),  R = phi / Phi
// and the coefficient of the gradient, cc = (d dl / d delta) / delta, so that the pair
// adds cc (x_i - x_j) to g_i; cc = 0 for a coincident pair (delta = 0), the convention
// of Eq. 5 for s_ij.
//
// Evaluation.  With u = |tau| / sqrt2, e = erfcx(u) = exp(u^2) erfc(u) and E = exp(-u^2),
//   Phi(-|tau|) = e E / 2,
//   tau <  0:  log2 Phi = log2(e / 2) - u^2 log2(e)   (log domain: no underflow for far
//                                                      edges),  R = sqrt(2/pi) / e
//   tau >= 0:  log2 Phi = log2(1 - e E / 2) (with the rounding of 1 - e E / 2 corrected),
//              R = E / (sqrt(2 pi) (1 - e E / 2))
// erfcx comes from one polynomial in y = (u - K)/(u + K) (Shepherd-Laframboise form,
// coefficients in erfcx_coef.h).  Both branches are evaluated without divergence: five
// hardware transcendentals (rsq, two rcp, exp2, log2) per pair.  All products and sums
// are explicit fmaf/mul/add so that the sweep and the exact edge pass, which both call
// this function, produce bit-identical values for the same pair.
#pragma once

#include <hip/hip_runtime.h>

#include "erfcx_coef.h"

namespace gempe {

struct PairParams {
    float mu;
    float inv_sigma;
    float d1_scale;  // -1 / (sigma ln 2)
};

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kSqrt1_2 = 0.70710678118654752f;
constexpr float kSqrt2OverPi = 0.79788456080286536f;   // sqrt(2/pi)
constexpr float kInvSqrt2Pi = 0.39894228040143268f;    // 1/sqrt(2 pi)
constexpr float kFltMin = 1.17549435e-38f;

__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// erfcx(u) for u >= 0 (u clamped to 1e18 so that (u + K)(1 + 2u) stays finite).
__device__ __forceinline__ float erfcx_pos(float u) {
    float uc = fminf(u, 1.0e18f);
    float A = uc + GEMPE_ERFCX_K;
    float B = __builtin_fmaf(2.0f, uc, 1.0f);
    float q = hw_rcp(A * B);
    float y = (uc - GEMPE_ERFCX_K) * B * q;
    float f = kErfcxCoef[GEMPE_ERFCX_NCOEF - 1];
#pragma unroll
    for (int k = GEMPE_ERFCX_NCOEF - 2; k >= 0; --k) f = __builtin_fmaf(f, y, kErfcxCoef[k]);
    return f * A * q;
}

// dl (bits) and cc for squared distance r2; a = +1 (non-edge) or -1 (edge).
__device__ __forceinline__ void pair_eval(float r2, float a, const PairParams &P, float &dl,
                                          float &cc) {
    float r2c = fmaxf(r2, kFltMin);
    float rinv = hw_rsq(r2c);
    float delta = r2c * rinv;
    float tau = a * ((delta - P.mu) * P.inv_sigma);
    float u = fabsf(tau) * kSqrt1_2;
    float e = erfcx_pos(u);
    float u2l = (tau * tau) * (0.5f * kLog2e);  // u^2 log2(e), two roundings
    float E = hw_exp2(-u2l);
    bool neg = tau < 0.0f;
    float half_e = 0.5f * e;
    float q_small = half_e * E;     // Phi(-|tau|)
    float one_m = 1.0f - q_small;   // Phi(|tau|), rounded
    float rq = hw_rcp(neg ? e : one_m);
    // tau >= 0: log2(1 - Q) = log2(one_m) + log2(1 + ((1 - one_m) - Q) / one_m); the
    // rounding error of one_m is recovered exactly ((1 - one_m) is exact), so far
    // non-edges keep full relative accuracy without a log1p.
    float corr = (((1.0f - one_m) - q_small) * rq) * kLog2e;
    float L = hw_log2(neg ? half_e : one_m) + (neg ? -u2l : corr);
    // r2 - r2 is 0 for finite r2 and NaN otherwise: a NaN or infinite coordinate reaches
    // the loss (and the status word) instead of being clamped away by fmaxf above.
    dl = (r2 - r2) - L;
    float R = (neg ? kSqrt2OverPi : E * kInvSqrt2Pi) * rq;
    float d1 = (a * R) * P.d1_scale;
    cc = (r2 > 0.0f) ? d1 * rinv : 0.0f;
}

// Non-edge specialisation used by the sweep (a = +1).
__device__ __forceinline__ void pair_nonedge(float r2, const PairParams &P, float &dl, float &cc) {
    pair_eval(r2, 1.0f, P, dl, cc);
}

}  // namespace gempe
