// FP32 pair function of the GEMPE coding cost (device code).
//
// For a vertex pair at squared distance r2, with a = -1 for an edge and +1 otherwise,
//   tau = a (delta - mu) / sigma,  dl = -log2 Phi(tau)          (Sec. II-B, dl+/-)
//   d dl / d delta = -(a / (sigma ln 2)) R(tau),  R = phi / Phi
// and the coefficient of the gradient, cc = (d dl / d delta) / delta, so that the pair
// adds cc (x_i - x_j) to g_i.  A coincident pair (r2 = 0) has diff = 0, so it adds 0 to the
// gradient, the convention of Eq. 5 for s_ij (cc stays finite: r2 is offset by FLT_MIN).
//
// Evaluation.  With u = |tau| / sqrt2, h = erfcx(u) / 2 and E = exp(-u^2),
//   Phi(-|tau|) = h E,
//   tau <  0:  log2 Phi = log2 h - u^2 log2(e)      (log domain: no underflow for far
//                                                      edges),  R = sqrt(2/pi) / (2 h)
//   tau >= 0:  log2 Phi = log2(1 - h E), with the rounding of 1 - h E recovered exactly,
//              R = E / (sqrt(2 pi) (1 - h E))
// erfcx comes from one polynomial in y = (u - K)/(u + K) (Shepherd-Laframboise form,
// coefficients in erfcx_coef.h).  Both branches are evaluated without divergence: five
// hardware transcendentals (rsq, two rcp, exp2, log2) per pair, one reciprocal and one
// logarithm shared by the two branches through a select of their argument.  All products
// and sums are explicit (no contraction) so that the sweep and the exact edge pass, which
// both call this function, produce bit-identical values for the same pair.
#pragma once

#include <hip/hip_runtime.h>

#include "erfcx_coef.h"

namespace gempe {

struct PairParams {
    float mu_s;       // mu / sigma
    float inv_sigma;  // 1 / sigma
    float c_neg;      // sqrt(2/pi)/2 * d1s,   d1s = -1 / (sigma ln 2)
    float c_pos;      // 1/sqrt(2 pi) * d1s
};

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kSqrt1_2 = 0.70710678118654752f;
constexpr float kSqrt2 = 1.41421356237309505f;
constexpr float kFltMin = 1.17549435e-38f;

__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// dl (bits) and cc for squared distance r2; a = +1 (non-edge) or -1 (edge).
__device__ __forceinline__ void pair_eval(float r2, float a, const PairParams &P, float &dl,
                                          float &cc) {
    // FLT_MIN keeps rsq finite at r2 = 0 and leaves every r2 > 2^-102 unchanged; NaN and
    // infinite r2 stay non-finite and reach the loss (and the status word).
    float r2c = r2 + kFltMin;
    float rinv = hw_rsq(r2c);
    float delta = r2c * rinv;
    float tau = a * __builtin_fmaf(delta, P.inv_sigma, -P.mu_s);
    // (u + K), (1 + 2u), (u - K) with u = |tau|/sqrt2 clamped so (u+K)(1+2u) stays finite
    float t = fminf(fabsf(tau), 1.0e18f);
    float A = __builtin_fmaf(t, kSqrt1_2, GEMPE_ERFCX_K);
    float B = __builtin_fmaf(t, kSqrt2, 1.0f);
    float Nm = __builtin_fmaf(t, kSqrt1_2, -GEMPE_ERFCX_K);
    float q = hw_rcp(A * B);
    float y = (Nm * B) * q;
    float f = kErfcxHalfCoef[GEMPE_ERFCX_NCOEF - 1];
#pragma unroll
    for (int k = GEMPE_ERFCX_NCOEF - 2; k >= 0; --k) f = __builtin_fmaf(f, y, kErfcxHalfCoef[k]);
    float h = f * (A * q);                          // erfcx(u) / 2
    float nu2l = tau * (tau * (-0.5f * kLog2e));    // -u^2 log2(e)
    float E = hw_exp2(nu2l);                        // exp(-u^2)
    float q_small = h * E;                          // Phi(-|tau|)
    float one_m = 1.0f - q_small;                   // Phi(|tau|), rounded
    bool neg = tau < 0.0f;
    float sel = neg ? h : one_m;
    float rq = hw_rcp(sel);
    // tau >= 0: log2(1 - Q) = log2(one_m) + log2(1 + ((1 - one_m) - Q) / one_m); (1 - one_m)
    // is exact, so far non-edges keep full relative accuracy without a log1p.
    float corr = (((1.0f - one_m) - q_small) * rq) * kLog2e;
    dl = -(hw_log2(sel) + (neg ? nu2l : corr));
    float Rf = neg ? P.c_neg : E * P.c_pos;
    cc = (a * (Rf * rq)) * rinv;
}

// Non-edge specialisation used by the sweep (a = +1).
__device__ __forceinline__ void pair_nonedge(float r2, const PairParams &P, float &dl, float &cc) {
    pair_eval(r2, 1.0f, P, dl, cc);
}

}  // namespace gempe
