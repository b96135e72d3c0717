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
#include "millsq_coef.h"

namespace gempe {

struct PairParams {
    float mu_s;       // mu / sigma
    float inv_sigma;  // 1 / sigma
    float c_neg;      // sqrt(2/pi)/2 * d1s,   d1s = -1 / (sigma ln 2)
    float c_pos;      // 1/sqrt(2 pi) * d1s
    float tk_scale;   // table index scale 16 / sigma   (16 tau = tk_scale delta + tk_off)
    float tk_off;     // -16 mu / sigma
    float slope_k;    // 16 ln 2 / sigma      (d dl/d delta = dl slope_k dL/df of the table)
    float r_scale;    // -sigma ln 2          (R = phi/Phi from the slope term)
    float w_scale;    // 1 / (2 sigma^2 ln 2) (w = dl''/2 = R (R + tau) w_scale)
    float wk2;        // -1 / (32 sigma)      (table form of w, see pair_nonedge_tab)
    int table_full;   // 1 when every non-edge tau >= -mu/sigma lies inside the table
                      // (16 mu / sigma <= 127), so the sweeps need no below-table fallback
    int reverse;      // 1: the FP32 sweeps take their tiles in reverse order (a schedule
                      // perturbation; each tile keeps its own loss-partial slot)
};

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kSqrt1_2 = 0.70710678118654752f;
constexpr float kSqrt2 = 1.41421356237309505f;
constexpr float kFltMin = 1.17549435e-38f;
// The hardware exp2 returns 0 for results below 2^-126 (FP32's smallest normal).  A far
// non-edge (tau beyond about 13.2; common at d = 128 from a spread start) has dl and cc in
// that range, and a vertex with only far pairs owes its whole gradient to them, so both
// pair functions evaluate exp2 on a range where its result is normal and scale back with a
// multiplication, which rounds into the subnormals as IEEE arithmetic does.  The staged
// one-gather table holds log2 dl + kTabLogScale (its c0 raised when it is staged).
constexpr float kTabLogScale = 32.0f;
constexpr float kTabUnscale = 0x1p-32f;

__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// dl (bits) and cc for squared distance r2; a = +1 (non-edge) or -1 (edge).  With W, also
// the weight of the weighted-majorization parabola (Sec. II-C, Eqs. 3-4: slope and curvature
// of the parabola match dl at the current distance), w = dl''/2 = R (R + tau) / (2 sigma^2
// ln 2).  For tau < 0, R + tau = R q(-tau) with q(t) = 1 - t M(t) (M the Mills ratio) from
// millsq_coef.h, so far edges (R + tau -> 1/|tau|) keep full relative accuracy.
// TAIL = false: exp(-u^2) below 2^-126 (tau beyond about 13.2) is taken as 0, for callers
// that give such pairs 0 anyway (the BF16 path's far flush); the bits of every other pair
// are the same for both values of TAIL.
template <bool W, bool TAIL = true>
__device__ __forceinline__ void pair_eval_t(float r2, float a, const PairParams &P, float &dl, float &cc,
                                            float &w) {
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
    float E;                                        // exp(-u^2)
    if (TAIL) {
        // below 2^-64 the exponent is raised by 64 (exactly: nu2l is then a multiple of its
        // ulp of at least 2^-17) and the result scaled back
        const bool tiny = nu2l < -64.0f;
        E = hw_exp2(tiny ? nu2l + 64.0f : nu2l) * (tiny ? 0x1p-64f : 1.0f);
    } else {
        E = hw_exp2(nu2l);
    }
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
    if (W) {
        const float R = (Rf * rq) * P.r_scale;      // phi(tau) / Phi(tau)
        float fq = kMillsQCoef[GEMPE_MILLSQ_NCOEF - 1];
#pragma unroll
        for (int k = GEMPE_MILLSQ_NCOEF - 2; k >= 0; --k) fq = __builtin_fmaf(fq, y, kMillsQCoef[k]);
        const float wn = (R * R) * (fq * hw_rcp(__builtin_fmaf(t, t, 1.0f)));
        const float wp = R * (R + tau);
        w = (neg ? wn : wp) * P.w_scale;
    }
}

__device__ __forceinline__ void pair_eval(float r2, float a, const PairParams &P, float &dl, float &cc) {
    float unused;
    pair_eval_t<false>(r2, a, P, dl, cc, unused);
}

// Non-edge specialisation (a = +1) with the closed-form evaluation above.
__device__ __forceinline__ void pair_nonedge(float r2, const PairParams &P, float &dl, float &cc) {
    pair_eval(r2, 1.0f, P, dl, cc);
}

// ------------------------------------------------------------------------------------
// Non-edge pair from the piecewise-cubic table of L = log2 dl(tau) (ltab.h), staged in LDS
// as one float4 {c0 + kTabLogScale, c1, c2, c3} per segment of width 1/16 in tau:
//   16 tau + zero = tk_scale delta + tko,  segment = floor of that,  f = its fraction
//   dl = 2^(c0 + f(c1 + f(c2 + f c3))),  d dl/d delta = dl slope_k (c1 + f(2 c2 + 3 c3 f))
// with the exp2 taken 2^32 times larger and the results scaled back (see kTabLogScale)
// (tko = tk_off + zero from table_offset, zero = the segment of tau = 0).  Two
// transcendentals (rsq, exp2) instead of five and one 16-byte LDS gather per pair.  r2
// must be positive: the sweeps' squared distances start from FLT_MIN (sqdist_eps), which
// keeps rsq finite for coincident points.  Returns false when tau is below the table
// (dl, cc unspecified); from the table's top on (dl < 2^-150) it returns dl = cc = 0.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int floor_to_int(float x) {
    int k;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(k) : "v"(x));
    return k;
}

// tk_off + zero, in a vector register: the index fma then reads a single scalar operand,
// which GFX9 encodings allow, instead of copying a second one into a VGPR for every pair.
__device__ __forceinline__ float table_offset(const PairParams &P, int zero) {
    float t = P.tk_off + (float)zero;
    asm("" : "+v"(t));
    return t;
}

template <bool W>
__device__ __forceinline__ bool pair_nonedge_tab(float r2, const PairParams &P, const float4 *__restrict__ tab,
                                                 float tko, unsigned segs, float &dl, float &cc, float &w) {
    float rinv = hw_rsq(r2);
    float delta = r2 * rinv;
    float tk = __builtin_fmaf(delta, P.tk_scale, tko);
    float f = __builtin_amdgcn_fractf(tk);
    const int k = floor_to_int(tk);
    const bool ok = k >= 0;
    // byte offset of the segment's float4; indices past the last segment (and, for lanes
    // that fall back, negative ones) read the all-zero segment `segs`
    const unsigned off = min((unsigned)k, segs) << 4;
    const float4 c = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tab) + off);
    // L and dL/df share p = c3 f, q = c2 + p:  L = c0 + f (c1 + f q),  dL/df = c1 + f (2q + p)
    const float p = c.w * f;
    const float q = c.z + p;
    const float L = __builtin_fmaf(__builtin_fmaf(q, f, c.y), f, c.x);  // log2 dl + kTabLogScale
    const float Lf = __builtin_fmaf(__builtin_fmaf(q, 2.0f, p), f, c.y);
    const float dls = hw_exp2(L);  // 2^32 dl, normal down to dl = 2^-158
    const float slope = P.slope_k * kTabUnscale;
    dl = dls * kTabUnscale;
    cc = dls * (Lf * (slope * rinv));  // (d dl / d delta) / delta, one multiply after the exp2
    // w = R (R + tau) / (2 sigma^2 ln 2) with R = -sigma ln2 c1:  w = c1 (ln2/2 c1 - tau/(2 sigma))
    if (W) {
        const float c1 = (dls * Lf) * slope;  // d dl / d delta
        w = c1 * __builtin_fmaf(0.34657359028f, c1, __builtin_fmaf(delta, P.tk_scale, P.tk_off) * P.wk2);
    }
    return ok;
}

// The same table staged as two float4 per segment, {n0 (int32 bits), r0, c1, c2} and
// {c3, d1, d2, d3} with n0 + r0 = c0 (n0 integer) and d = slope_k (c1, 2 c2, 3 c3):
//   dl = 2^n0 2^(r0 + f(c1 + f(c2 + f c3))),  d dl/d delta = dl (d1 + f(d2 + f d3)).
// Two gathers instead of one, but fewer dependent operations after them; the fused
// gradient-descent iteration, whose waves are few and short, runs faster with it (the long
// sweeps, bound by LDS bank conflicts, with the one-gather form).
template <bool W>
__device__ __forceinline__ bool pair_nonedge_tab2(float r2, const PairParams &P, const float4 *__restrict__ tab,
                                                  float tko, unsigned segs, float &dl, float &cc, float &w) {
    float rinv = hw_rsq(r2);
    float delta = r2 * rinv;
    float tk = __builtin_fmaf(delta, P.tk_scale, tko);
    float f = __builtin_amdgcn_fractf(tk);
    const int k = floor_to_int(tk);
    const bool ok = k >= 0;
    const unsigned off = min((unsigned)k, segs) << 5;
    const float4 *e = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tab) + off);
    const float4 A = e[0], B = e[1];
    const float r = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(B.x, f, A.w), f, A.z), f, A.y);
    const float D = __builtin_fmaf(__builtin_fmaf(B.w, f, B.z), f, B.y);
    dl = __builtin_amdgcn_ldexpf(hw_exp2(r), __float_as_int(A.x));
    const float c1 = dl * D;  // d dl / d delta
    cc = c1 * rinv;
    if (W) w = c1 * __builtin_fmaf(0.34657359028f, c1, __builtin_fmaf(delta, P.tk_scale, P.tk_off) * P.wk2);
    return ok;
}

// The non-edge value every sweep and edge correction of d <= 16 uses: the table for tau
// from its bottom up, else (per lane) the closed form.  A deterministic function of r2 for
// a given table form, so a sweep and its edge pass subtract exactly what the other added.
// CHK = false: the caller knows that no tau lies below the table (P.table_full), and the
// per-pair test and its branch go, which lets the gathers of several pairs issue together.
template <bool W, bool TWO = false, bool CHK = true>
__device__ __forceinline__ void nonedge_eval(float r2, const PairParams &P, const float4 *__restrict__ tab,
                                             float tko, unsigned segs, float &dl, float &cc, float &w) {
    const bool ok = TWO ? pair_nonedge_tab2<W>(r2, P, tab, tko, segs, dl, cc, w)
                        : pair_nonedge_tab<W>(r2, P, tab, tko, segs, dl, cc, w);
    if (CHK && __builtin_expect(__ballot(!ok) != 0ull, 0)) {
        float dl2, cc2, w2;
        pair_eval_t<W>(r2, 1.0f, P, dl2, cc2, w2);
        dl = ok ? dl : dl2;
        cc = ok ? cc : cc2;
        if (W) w = ok ? w : w2;
    }
}

}  // namespace gempe
