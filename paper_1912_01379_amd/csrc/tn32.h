// Float32 truncated-normal draw by inversion for the batched sampler (Sec. IV.B: a data
// mode's coordinate is redrawn from N(c/d, 1/d^2) truncated to the interval of
// Eq. (modeLimits)).
//
// In standard units a = d lo - c, b = d hi - c, w = b - a, the draw is x = F^-1(F(a) +
// u (F(b) - F(a))) for the normal CDF F.  Every case is mapped onto one path that evaluates
// the upper tail Q = 1 - F twice and its inverse once:
//   a >= 0 (interval above the mean):   p = Q(a) - u (Q(a) - Q(a + w)), x = Q^-1(p);
//   b <= 0 (interval below the mean):   the mirror image, with u and 1 - u exchanged;
//   a < 0 < b:                          p = F(a) + u mass, x = -Q^-1(p) when p <= 1/2, else
//                                       x = Q^-1(Q(b) + (1 - u) mass), mass = 1 - Q(-a) - Q(b);
// each tail probability is formed from the end where it is small, so nothing cancels.
// Q and Q^-1 are the polynomial fits of tn32_coef.h on the hardware exp2/log2/rcp/sqrt,
// with one Newton step on Q^-1; they carry about 1e-7 relative error.
// Two rare cases leave this path: intervals much narrower than the Gaussian (the density
// is then an exponential tilt across the interval, drawn in closed form), and one-sided
// intervals more than 10 standard deviations from the mean (the tail path on the Mills
// ratio).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "tn32_coef.h"

namespace asmk {

__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// exp(-x^2/2) for 0 <= x < 14, carrying the rounding of x^2 and of the scaling to base 2
__device__ __forceinline__ float exp_half_sq(float x) {
    constexpr float kL2eHalf = 0.72134752f;           // log2(e) / 2, rounded
    constexpr float kL2eHalfLo = 9.6298141e-09f;      // log2(e) / 2 - kL2eHalf
    constexpr float kLn2 = 0.69314718f;
    const float x2 = x * x;
    const float x2lo = fmaf(x, x, -x2);               // x^2 = x2 + x2lo exactly
    const float e = -x2 * kL2eHalf;
    const float elo = fmaf(-x2, kL2eHalf, -e) - fmaf(x2, kL2eHalfLo, x2lo * kL2eHalf);
    return hw_exp2(e) * fmaf(elo, kLn2, 1.0f);
}

// Q(x) = P(Z > x) for x >= 0 (+inf allowed)
__device__ __forceinline__ float q_upper32(float x) {
    using namespace tn32c;
    const float r = hw_rcp(kQK + x);
    const float v = fmaf(kQAlpha, r, kQBeta);
    float h = kQ[kQDeg];
#pragma unroll
    for (int j = kQDeg - 1; j >= 0; --j) h = fmaf(h, v, kQ[j]);
    const float q = (kQK * r) * h * exp_half_sq(x);
    return x < kQXmax ? q : 0.0f;
}

// z >= 0 with Q(z) = p, for 1e-33 <= p <= 1/2
__device__ __forceinline__ float q_inv32(float p) {
    using namespace tn32c;
    constexpr float kLn2 = 0.69314718f;
    constexpr float kSqrt2Pi = 2.5066283f;
    p = fmaxf(p, 1e-33f);
    const float y = fmaf(-2.0f, p, 1.0f);
    const float w = -kLn2 * hw_log2(4.0f * p * (1.0f - p));
    // centre: z = y P_c((w - wcut/2) / (wcut/2)); tail: z = s P_t(a s + b), s = sqrt(w)
    const float vc = fmaf(w, 2.0f / kInvWcut, -1.0f);
    float hc = kInvC[kInvDegC];
#pragma unroll
    for (int j = kInvDegC - 1; j >= 0; --j) hc = fmaf(hc, vc, kInvC[j]);
    const float s = hw_sqrt(w);
    const float vt = fmaf(kInvTa, s, kInvTb);
    float ht = kInvT[kInvDegT];
#pragma unroll
    for (int j = kInvDegT - 1; j >= 0; --j) ht = fmaf(ht, vt, kInvT[j]);
    float z = w < kInvWcut ? y * hc : s * ht;
    // Newton on Q(z) = p: z += (Q(z) - p) / phi(z), Q(z) = E t H, phi(z) = E / sqrt(2 pi)
    const float r = hw_rcp(kQK + z);
    const float v = fmaf(kQAlpha, r, kQBeta);
    float h = kQ[kQDeg];
#pragma unroll
    for (int j = kQDeg - 1; j >= 0; --j) h = fmaf(h, v, kQ[j]);
    // the step is about 1e-5 of z, so exp(-z^2/2) needs no compensation here
    const float E = hw_exp2(-0.72134752f * z * z);
    const float step = kSqrt2Pi * fmaf(-p, hw_rcp(E), (kQK * r) * h);
    return E > 0.0f ? z + step : z;
}

// 1 - e^-X for X >= 0: the Taylor series to X^8 below 1/2 (the first omitted term is
// below 2e-8 of the value there), the hardware exp2 above (no cancellation: 1 - e^-X > 0.39)
__device__ __forceinline__ float one_minus_exp_neg(float X) {
    constexpr float kL2e = 1.44269504f;
    float p = -1.0f / 40320.0f;
    p = fmaf(p, X, 1.0f / 5040.0f);
    p = fmaf(p, X, -1.0f / 720.0f);
    p = fmaf(p, X, 1.0f / 120.0f);
    p = fmaf(p, X, -1.0f / 24.0f);
    p = fmaf(p, X, 1.0f / 6.0f);
    p = fmaf(p, X, -0.5f);
    p = fmaf(p, X, 1.0f);
    return X < 0.5f ? X * p : 1.0f - hw_exp2(-X * kL2e);
}

// -log(1 - y) for 0 <= y < 1: 2 atanh(t) = 2 (t + t^3/3 + ... + t^13/13), t = y / (2 - y)
// <= 1/3, for y <= 1/2 (first omitted term below 2e-8 of the value); the hardware log2 of
// 1 - y (exact there) above
__device__ __forceinline__ float neg_log1m(float y) {
    constexpr float kLn2 = 0.69314718f;
    const float t = y * hw_rcp(2.0f - y);
    const float t2 = t * t;
    float p = 1.0f / 13.0f;
    p = fmaf(p, t2, 1.0f / 11.0f);
    p = fmaf(p, t2, 1.0f / 9.0f);
    p = fmaf(p, t2, 1.0f / 7.0f);
    p = fmaf(p, t2, 1.0f / 5.0f);
    p = fmaf(p, t2, 1.0f / 3.0f);
    p = fmaf(p, t2, 1.0f);
    const float lg = -kLn2 * hw_log2(1.0f - y);   // both forms are computed: no branch
    return y <= 0.5f ? 2.0f * t * p : lg;
}

// t in [0, w] with density proportional to exp(-lam t) (lam of either sign), by inversion:
// the distance s from the end where the density is largest is
// s = -log(1 - v (1 - e^-|lam| w)) / |lam|, with v = u from the lower end (lam > 0) and
// v = 1 - u from the upper end (lam < 0)
__device__ __forceinline__ float tilt_draw32(float lam, float w, float u, float uc) {
    const float X = fabsf(lam * w);
    const float v = lam > 0.0f ? u : uc;
    const float s = neg_log1m(v * one_minus_exp_neg(X)) * hw_rcp(fabsf(lam));
    const float sd = X < 1e-6f ? v * w : s;   // also covers w = 0 and lam = 0
    return lam > 0.0f ? sd : w - sd;
}

// Mills ratio m(x) = Q(x) / phi(x) for x >= 0: the fit of Q below 14, the asymptotic
// series 1/x (1 - 1/x^2 + 3/x^4 - 15/x^6) above (its first omitted term is 7e-11 there);
// both are formed and one is selected, so no branch splits a wavefront
__device__ __forceinline__ float mills32(float x) {
    using namespace tn32c;
    constexpr float kSqrt2Pi = 2.5066283f;
    const float r = hw_rcp(kQK + x);
    const float v = fmaf(kQAlpha, r, kQBeta);
    float h = kQ[kQDeg];
#pragma unroll
    for (int j = kQDeg - 1; j >= 0; --j) h = fmaf(h, v, kQ[j]);
    const float fit = kSqrt2Pi * (kQK * r) * h;
    const float ix = hw_rcp(x), i2 = ix * ix;
    const float asym = ix * fmaf(i2, fmaf(i2, fmaf(i2, -15.0f, 3.0f), -1.0f), 1.0f);
    return x < kQXmax ? fit : asym;
}

// t in [0, w] with density proportional to exp(-a t - t^2/2) for a > 10, where Q(a + t)
// underflows: solve log Q(a + t) - log Q(a) = log(1 - u (1 - Q(a + w) / Q(a))) for t with
// log Q(a + t) - log Q(a) = -t (a + t/2) + log(m(a + t) / m(a)), by Newton from t = -target/a
// (d/dt log Q(a + t) = -1 / m(a + t)).  The logarithms of Mills-ratio quotients are small
// corrections to t (a + t/2) > 10 t and take the hardware log2; the target is formed by the
// series helpers above, which keep 1 - e^lr and log(1 - y) accurate near zero.
__device__ __forceinline__ float tail_draw32(float a, float w, float u) {
    constexpr float kLn2 = 0.69314718f;
    const float rma = hw_rcp(mills32(a));
    // log of Q(a + w) / Q(a) (-inf for a one-sided interval: w = +inf)
    const float lr = fmaf(-w, fmaf(0.5f, w, a), kLn2 * hw_log2(mills32(a + w) * rma));
    const float target = -neg_log1m(u * one_minus_exp_neg(w < INFINITY ? -lr : INFINITY));
    float t = -target * hw_rcp(a);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float mt = mills32(a + t);
        const float g = fmaf(-t, fmaf(0.5f, t, a), fmaf(kLn2, hw_log2(mt * rma), -target));
        t = fmaf(g, mt, t);
    }
    return fminf(fmaxf(t, 0.0f), w);
}

// The draw in parameter units: delta in [lo, hi], lo <= 0 <= hi, d > 0, u in (0, 1).
// Lanes 2j and 2j + 1 must carry the same draw (the samplers give every lane of a chain the
// same arguments): the two tail probabilities of the inversion are evaluated once, one on
// each lane of the pair, and exchanged.
__device__ __forceinline__ float tn_draw32(float c, float d, float lo, float hi, float u) {
    const float uc = 1.0f - u;
    const float a = fmaf(d, lo, -c);
    const float b = fmaf(d, hi, -c);
    const float w = d * (hi - lo);
    const float rd = hw_rcp(d);
    const float far = fmaxf(fabsf(a), fabsf(b));
    // The tilt errs by about w^2/16 of the interval (the curvature it drops), the inversion
    // by about 1.5e-7 max(1, |a|, |b|) / w (the float32 resolution of p and x): take the tilt
    // where it is the more accurate of the two (lo = hi gives w = 0 and delta = lo).
    const bool narrow = w * w * w < 2.4e-6f * fmaxf(1.0f, far);
    // narrow interval: exponential tilt at the slope of the midpoint, computed without
    // branches by every lane (most draws of the samplers take it)
    const float lam = fmaf(0.5f, w, a);
    float delta = fmaf(tilt_draw32(lam, w, u, uc), rd, lo);
    if (!narrow) {
        const bool lower = b <= 0.0f;                   // interval below the mean
        const bool one = lower || a >= 0.0f;
        const float a1 = lower ? -b : a;
        const float u1 = lower ? uc : u;
        const float uc1 = lower ? u : uc;
        if (one && a1 > 10.0f) {
            const float t = tail_draw32(a1, w, u1);
            delta = lower ? hi - t * rd : lo + t * rd;
        } else {
            const bool odd = (__lane_id() & 1) != 0;
            const float e1 = one ? a1 : -a, e2 = one ? a1 + w : b;
            const float qm = q_upper32(odd ? e2 : e1);
            const float qo = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(qm), 0xB1, 0xF, 0xF, false));
            const float q1 = odd ? qo : qm;
            const float q2 = odd ? qm : qo;
            const float dq = q1 - q2;
            const float mass = (1.0f - q1) - q2;
            const float plo = fmaf(u, mass, q1);
            const float p1 = u1 <= 0.5f ? fmaf(-u1, dq, q1) : fmaf(uc1, dq, q2);
            const float p2 = plo <= 0.5f ? plo : fmaf(uc, mass, q2);
            const float p = one ? p1 : p2;
            const float sg = (one || plo > 0.5f) ? 1.0f : -1.0f;
            const float x = sg * q_inv32(p);
            const float t = fminf(fmaxf(x - a1, 0.0f), w);
            const float d1 = lower ? hi - t * rd : lo + t * rd;
            delta = one ? d1 : (x + c) * rd;
        }
    }
    return __builtin_amdgcn_fmed3f(delta, lo, hi);
}

}  // namespace asmk
