// Device primitives of a single move: counter-based uniforms and the inverse-CDF
// truncated normal of Sec. IV.B (a mode with d_i > 0 is redrawn from a Gaussian of width
// 1/d_i centred on the best fit, truncated to the interval of Eq. (modeLimits)).
//
// The truncated normal is reduced to one primitive: draw t in [0, w] with density
// proportional to exp(-a t - t^2/2), a >= 0.  With the Mills ratio m(x) = Q(x)/phi(x),
//   E(a, t) = int_0^t exp(-a s - s^2/2) ds = m(a) - m(a + t) exp(-t (a + t/2)),
// and for small t (where the difference cancels) the series
//   E(a, t) = sum_j (-1/2)^j / j! t^(2j+1) M_2j(a t),  M_k(z) = int_0^1 v^k e^(-z v) dv.
// It is solved by Newton's method to full float64 precision (the float64 sampler is held to
// trajectory parity with the CPU reference); the float32 samplers use tn32.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asmk {

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the maps from its words to (0,1)
// ------------------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// float64 uniform of move (chain, sweep, block, mode): ((w0>>6) 2^26 + (w1>>6) + 1/2) 2^-52;
// tag 0 for the move's draw, 3 for its acceptance test under a gamma prior
__device__ __forceinline__ double move_u64(uint64_t seed, uint32_t problem, uint32_t chain,
                                           uint32_t sweep, uint32_t block, uint32_t mode,
                                           uint32_t tag = 0u) {
    U4 c{chain, sweep, (block << 16) | mode, tag};
    U4 o = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32) ^ problem);
    const uint64_t j = ((uint64_t)(o.x >> 6) << 26) | (uint64_t)(o.y >> 6);
    return ((double)j + 0.5) * 0x1.0p-52;
}

// the hierarchy level sampled in a sweep, the same for every chain of the problem (tag 2 in
// the last word, chain field 2^32 - 1): floor(w0 L / 2^32), uniform over the L levels
__host__ __device__ __forceinline__ uint32_t sweep_level(uint64_t seed, uint32_t problem, uint32_t sweep,
                                                         uint32_t levels) {
    const U4 c{0xFFFFFFFFu, sweep, 0u, 2u};
    const U4 o = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32) ^ problem);
    return (uint32_t)(((uint64_t)o.x * levels) >> 32);
}

// float32 uniforms: one Philox call serves four consecutive modes (tag 1 in the last word;
// tag 4 for the acceptance tests of a gamma prior)
__device__ __forceinline__ U4 move_words32(uint64_t seed, uint32_t problem, uint32_t chain,
                                           uint32_t sweep, uint32_t block, uint32_t quad,
                                           uint32_t tag = 1u) {
    U4 c{chain, sweep, (block << 16) | quad, tag};
    return philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32) ^ problem);
}

__device__ __forceinline__ float word_u32(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * 0x1.0p-23f;   // (2J+1) 2^-24, open interval
}

// ------------------------------------------------------------------------------------
// math wrappers of the float64 draw
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ double m_log1p(double x) { return log1p(x); }
__device__ __forceinline__ double m_erfcx(double x) { return erfcx(x); }
__device__ __forceinline__ double m_erf(double x) { return erf(x); }
__device__ __forceinline__ double m_erfc(double x) { return erfc(x); }
__device__ __forceinline__ double m_abs(double x) { return fabs(x); }
__device__ __forceinline__ bool m_isinf(double x) { return __builtin_isinf(x); }

template <typename T>
struct TnCfg;
template <>
struct TnCfg<double> {
    static constexpr double series_max = 0.25;   // series for t <= this
    static constexpr int terms = 10;             // terms of the series
    static constexpr int max_iter = 100;
    static constexpr double tol = 4e-16;
};

// Mills ratio Q(x)/phi(x) = sqrt(pi/2) erfcx(x/sqrt 2), x >= 0
template <typename T>
__device__ __forceinline__ T mills(T x) {
    return T(1.2533141373155002512) * m_erfcx(x * T(0.70710678118654752440));
}

// M_k(z) = int_0^1 v^k exp(-z v) dv for even k, z >= 0
template <typename T>
__device__ T moment_k(int k, T z) {
    if (k == 0) return (z == T(0)) ? T(1) : -m_expm1(-z) / z;
    if (z <= T(50)) {
        // e^-z sum_j z^j / ((k+1)(k+2)...(k+1+j)), all terms positive
        T term = T(1) / T(k + 1), sum = term;
        for (int j = 1; j < 400; ++j) {
            term *= z / T(k + 1 + j);
            sum += term;
            if (term < T(1e-18) * sum) break;
        }
        return m_exp(-z) * sum;
    }
    // k!/z^(k+1) (1 - e^-z sum_{j<=k} z^j/j!)
    T fact = T(1), poly = T(1), zj = T(1), zk = z;
    for (int j = 1; j <= k; ++j) {
        fact *= T(j);
        zj *= z / T(j);
        poly += zj;
        zk *= z;
    }
    return fact / zk * (T(1) - m_exp(-z) * poly);
}

// E(a, t) = int_0^t exp(-a s - s^2/2) ds, a >= 0, t >= 0 (t may be +inf)
template <typename T>
__device__ T tn_mass(T a, T t) {
    if (!(t > T(0))) return T(0);
    if (m_isinf(t)) return mills(a);
    if (t <= TnCfg<T>::series_max) {
        const T z = a * t;
        T coef = t, sum = T(0);
        for (int j = 0; j < TnCfg<T>::terms; ++j) {
            sum += coef * moment_k<T>(2 * j, z);
            coef *= -(t * t) / T(2 * (j + 1));
        }
        return sum;
    }
    return mills(a) - mills(a + t) * m_exp(-t * (a + T(0.5) * t));
}

// t in [0, w] with density prop. to exp(-a t - t^2/2) at uniform u (uc = 1 - u, exact)
template <typename T>
__device__ T tn_onesided(T a, T w, T u, T uc) {
    const T Ew = tn_mass(a, w);
    T tl = T(0), th, t;
    const bool lower = (u <= T(0.5));
    th = lower ? (w < T(1) ? w : T(1)) : (w < T(40) ? w : T(40));
    t = T(0.5) * (tl + th);
    if (a > T(0)) {
        const T ts = -m_log1p(u * m_expm1(-a * w)) / a;   // exponential-tilt start
        if (ts > tl && ts < th) t = ts;
    } else if (w < T(1)) {
        t = u * w;
    }
    if (lower) {
        const T target = u * Ew;
        for (int it = 0; it < TnCfg<T>::max_iter; ++it) {
            const T f = tn_mass(a, t) - target;
            if (f == T(0)) break;   // exact root
            if (f < T(0)) tl = t; else th = t;
            const T fp = m_exp(-t * (a + T(0.5) * t));
            T tn = t - f / fp;
            if (!(tn >= tl && tn <= th)) tn = T(0.5) * (tl + th);
            const T dt = m_abs(tn - t);
            t = tn;
            if (dt <= TnCfg<T>::tol * t || th - tl <= TnCfg<T>::tol * th) break;
        }
    } else {
        const T lstar = m_log(uc) + m_log(Ew);
        for (int it = 0; it < TnCfg<T>::max_iter; ++it) {
            const T tail = tn_mass(a + t, w - t);
            const T h = -t * (a + T(0.5) * t) + m_log(tail) - lstar;
            if (h == T(0)) break;   // exact root
            if (h > T(0)) tl = t; else th = t;
            T tn = t + h * tail;
            if (!(tn >= tl && tn <= th)) tn = T(0.5) * (tl + th);
            const T dt = m_abs(tn - t);
            t = tn;
            if (dt <= TnCfg<T>::tol * t || th - tl <= TnCfg<T>::tol * th) break;
        }
    }
    return t;
}

// delta ~ N(c/d, 1/d^2) truncated to [lo, hi], lo <= 0 <= hi, d > 0, by inversion at u
template <typename T>
__device__ T tn_draw(T c, T d, T lo, T hi, T u) {
    if (lo == hi) return lo;
    const T uc = T(1) - u;
    const T a = d * lo - c;        // standardised ends x = d delta - c
    const T b = d * hi - c;
    const T w = d * (hi - lo);
    T delta;
    if (a >= T(0)) {
        delta = lo + tn_onesided<T>(a, w, u, uc) / d;
    } else if (b <= T(0)) {
        delta = hi - tn_onesided<T>(-b, w, uc, u) / d;
    } else {
        const T pl = tn_mass(T(0), -a);
        const T pr = tn_mass(T(0), b);
        const T tot = pl + pr;
        const T q = u * tot;
        if (q < pl) {
            delta = (c - tn_onesided<T>(T(0), -a, (pl - q) / pl, q / pl)) / d;
        } else {
            delta = (c + tn_onesided<T>(T(0), b, (q - pl) / pr, (uc * tot) / pr)) / d;
        }
    }
    delta = delta < lo ? lo : delta;
    delta = delta > hi ? hi : delta;
    return delta;
}

}  // namespace asmk
