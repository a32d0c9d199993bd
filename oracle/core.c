/*
 * Plain FP64 CPU oracle for blocked modes sampling (Ghanem & Koch, arXiv:1912.01379).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference the
 * GPU library is checked against.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the GPU library.
 *
 * What it computes (the paper's notation):
 *   - whitened problem chi^2(f) = ||g~ - K~ f||^2 (Sec. IV, whitening after Eq. (chi2));
 *   - per-block SVD factors K~_b = U_b D_b V_b^T are inputs (computed by the Python
 *     driver with LAPACK);
 *   - a random walk over f >= 0 that updates one blocked mode e_i at a time (Sec. IV.B
 *     "Modes Sampling", Sec. IV.C "Blocked Modes Sampling"): for d_i > 0 the new value
 *     is drawn from a Gaussian of width 1/d_i centred on the best fit, for d_i = 0 from
 *     a flat distribution, both truncated to the interval of Eq. (modeLimits);
 *   - the estimate of Eq. (MCint) as the average of f over the post-burn-in samples.
 *
 * Readings where the paper is silent (each stated once more in the design notes):
 *   - the truncated Gaussian is drawn by inversion of its distribution function with
 *     one uniform number per move, not by rejection;
 *   - uniform numbers come from Philox4x32-10 (Salmon et al., SC'11) on the counter
 *     (chain, sweep, block<<16 | mode, 0) with key (seed_lo, seed_hi ^ problem);
 *   - components that round below zero after a move are set to +0;
 *   - modes of a block are visited in the order given (data modes by descending
 *     singular value, then the zero modes), blocks in increasing order;
 *   - with a hierarchy of partitions (Fig. 2, Sec. IV.C), every sweep samples all blocks of
 *     one level, the same for all chains, chosen by Philox on the counter
 *     (2^32 - 1, sweep, 0, 2): level = floor(w0 L / 2^32); the uniforms of a move keep the
 *     block's index within its level;
 *   - the residual is recomputed from scratch every `refresh_every` sweeps;
 *   - under a linear constraint c . A = F (Sec. IV.E), a block's modes span the part of the
 *     block orthogonal to its share of c (nm = Nb - 1 modes), so every move keeps c . A;
 *   - with gamma-prior weights prod_n A_n^(w_n - 1) (Sec. V.C, Eq. (compat), the limit of
 *     vanishing scale), each move's draw is a proposal accepted when
 *     log u' < sum_q (w_q - 1) log(A'_q / A_q), u' the uniform of counter
 *     (chain, sweep, block << 16 | mode, 3); a rejected move leaves the state unchanged.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EUNBOUNDED (-4)

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as      */
/* 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with the key added      */
/* into the high halves and a Weyl-sequence key schedule.                               */
/* ------------------------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on the open interval (0,1): 52 random bits plus one half, times 2^-52. */
static double u01_from_words(uint32_t w0, uint32_t w1) {
    uint64_t j = ((uint64_t)(w0 >> 6) << 26) | (uint64_t)(w1 >> 6);
    return ((double)j + 0.5) * 0x1.0p-52;
}

/* The hierarchy level of a sweep, shared by all chains of the problem. */
static int64_t sweep_level(uint64_t seed, int64_t problem, int64_t sweep, int64_t L) {
    if (L <= 1) return 0;
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu),
                       (uint32_t)(seed >> 32) ^ (uint32_t)problem};
    uint32_t ctr[4] = {0xffffffffu, (uint32_t)sweep, 0u, 2u};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    return (int64_t)(((uint64_t)w[0] * (uint64_t)L) >> 32);
}

/* tag 0: the move's draw; tag 3: its acceptance test under a gamma prior */
static double move_uniform_tag(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep,
                               int64_t block, int64_t mode, uint32_t tag) {
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu),
                       (uint32_t)(seed >> 32) ^ (uint32_t)problem};
    uint32_t ctr[4] = {(uint32_t)chain, (uint32_t)sweep,
                       ((uint32_t)block << 16) | (uint32_t)mode, tag};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    return u01_from_words(w[0], w[1]);
}

static double move_uniform(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep,
                           int64_t block, int64_t mode) {
    return move_uniform_tag(seed, problem, chain, sweep, block, mode, 0u);
}

/* (w - 1) log(a_new / a_old): one component's share of the log ratio of the gamma-prior
   weights prod_n A_n^(w_n - 1) (Eq. (gammadist), Eq. (compat)) between two states. */
static double prior_log_ratio(double a_new, double a_old, double wm1) {
    if (wm1 == 0.0 || a_new == a_old) return 0.0;
    if (a_old == 0.0) return wm1 > 0.0 ? INFINITY : -INFINITY;
    if (a_new == 0.0) return wm1 > 0.0 ? -INFINITY : INFINITY;
    return wm1 * log(a_new / a_old);
}

/* ------------------------------------------------------------------------------------ */
/* One-dimensional truncated normal, by inversion of its distribution function          */
/* (Sec. IV.B: a data mode is redrawn from a Gaussian of width 1/d centred on the best  */
/* fit, cut to the interval of Eq. (modeLimits)).                                       */
/*                                                                                      */
/* In standard units x = d delta - c the step is the u-quantile of a standard normal    */
/* restricted to [a, b], a = d lo - c, b = d hi - c: the x at which                     */
/*     F(x) = P(a <= X <= x) / P(a <= X <= b)                                           */
/* equals u.  It is found by plain bisection of F, nothing else.                        */
/*                                                                                      */
/* An interval below the centre (b <= 0) is first reflected (x -> -x, u -> 1 - u), so   */
/* the interval either lies above the centre (a >= 0) or contains it.  Masses are then  */
/* measured relative to the density at a reference point r0 (r0 = a above the centre,  */
/* 0 around it), in the offset tau = x - r0, so that no tail underflows:                */
/*     S(t1, t2) = int_{t1}^{t2} g(tau) dtau,   g(tau) = exp(-tau (2 r0 + tau) / 2).    */
/* Over a short stretch (where g changes by at most a factor e^2) S is a Gauss-Legendre */
/* sum, exact to rounding there.  Over a longer stretch it is a difference of upper     */
/* tails T(tau) = int_tau^inf g = Q(r0 + tau) / phi(r0), Q the normal upper tail, which */
/* then cancels by at most the factor 1 - e^-2.  Q / phi is taken from erfc below 8 and */
/* from the Laplace continued fraction above.                                           */
/* For u <= 1/2 the bisection solves S(ta, tau) = u S(ta, tb); above, it solves the     */
/* complementary S(tau, tb) = (1 - u) S(ta, tb), so both tails keep relative accuracy.  */
/* ------------------------------------------------------------------------------------ */
static const double SQRT_2PI = 2.5066282746310002416;

/* Gauss-Legendre nodes and weights on [-1, 1], set by the Python driver from numpy's
   leggauss before any draw. */
#define GL_MAX 32
static int gl_n = 0;
static double gl_x[GL_MAX], gl_w[GL_MAX];

void orc_set_quadrature(int n, const double *x, const double *w) {
    if (n > GL_MAX) n = GL_MAX;
    for (int i = 0; i < n; ++i) { gl_x[i] = x[i]; gl_w[i] = w[i]; }
    gl_n = n;
}

/* Mills ratio Q(x) / phi(x), x >= 0. */
static double mills(double x) {
    if (x < 8.0) {
        /* Q(x) = erfc(x / sqrt2) / 2; 1 / phi(x) = sqrt(2 pi) exp(x^2 / 2), with x^2 split
           exactly into hi + lo so that the exponential keeps its accuracy */
        double hi = x * x;
        double lo = fma(x, x, -hi);
        return 0.5 * erfc(x * 0.70710678118654752440) * SQRT_2PI * exp(0.5 * hi) * exp(0.5 * lo);
    }
    /* m(x) = 1 / (x + 1 / (x + 2 / (x + 3 / (x + ...)))), evaluated from deep down */
    double f = x;
    for (int k = 200; k >= 1; --k) f = x + (double)k / f;
    return 1.0 / f;
}

/* T(tau) = int_tau^inf g for r0 + tau >= 0: Q(r0 + tau) / phi(r0). */
static double tail_T(double r0, double tau) {
    if (isinf(tau)) return 0.0;
    return mills(r0 + tau) * exp(-0.5 * tau * (2.0 * r0 + tau));
}

/* S(t1, t2) = int_{t1}^{t2} g, t1 <= t2 (either may be infinite); r0 >= 0, and r0 > 0
   only with t1 >= 0 (an interval above the centre). */
static double mass_S(double r0, double t1, double t2) {
    if (!(t2 > t1)) return 0.0;
    if (isfinite(t1) && isfinite(t2)) {
        /* the change of log g over the stretch */
        double vmax = 0.5 * t2 * (2.0 * r0 + t2), vmin = 0.5 * t1 * (2.0 * r0 + t1);
        double v;
        if (r0 > 0.0 || t1 >= 0.0) v = vmax - vmin;
        else if (t2 <= 0.0) v = vmin - vmax;
        else v = fmax(vmin, vmax);
        if (v <= 2.0) {
            double h = 0.5 * (t2 - t1), m = 0.5 * (t1 + t2), s = 0.0;
            for (int i = 0; i < gl_n; ++i) {
                double tau = m + h * gl_x[i];
                s += gl_w[i] * exp(-0.5 * tau * (2.0 * r0 + tau));
            }
            return h * s;
        }
    }
    if (r0 > 0.0 || t1 >= 0.0) return tail_T(r0, t1) - tail_T(r0, t2);
    /* r0 = 0 and the stretch starts below the centre: g is even */
    if (t2 <= 0.0) return tail_T(0.0, -t2) - tail_T(0.0, -t1);
    return SQRT_2PI - tail_T(0.0, -t1) - tail_T(0.0, t2);
}

/* The offset tau in [ta, tb] of the u-quantile, by bisection (uc = 1 - u exactly). */
static double bisect_quantile(double r0, double ta, double tb, double u, double uc) {
    const double tot = mass_S(r0, ta, tb);
    /* a finite bracket: beyond 40 standard units of the reference nothing is left */
    double lo = isinf(ta) ? -40.0 : ta;
    double hi = isinf(tb) ? 40.0 : tb;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;   /* the bracket is two adjacent doubles */
        double f = (u <= 0.5) ? mass_S(r0, ta, mid) - u * tot : uc * tot - mass_S(r0, mid, tb);
        if (f < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Draw delta from N(c/d, 1/d^2) restricted to [lo, hi] (lo <= 0 <= hi, d > 0) at u. */
double orc_tn_draw(double c, double d, double lo, double hi, double u) {
    if (lo == hi) return lo;
    const double uc = 1.0 - u;   /* exact: u is a multiple of 2^-53 in (0, 1) */
    const double a = d * lo - c, b = d * hi - c;
    /* the interval's length in standard units, taken from hi - lo rather than b - a, which
       carries the rounding of both ends */
    const double w = d * (hi - lo);
    double delta;
    if (!(w > 0.0)) {
        /* too short for the Gaussian to vary across it at all: flat */
        delta = lo + u * (hi - lo);
    } else if (a >= 0.0) {
        delta = lo + bisect_quantile(a, 0.0, w, u, uc) / d;
    } else if (b <= 0.0) {
        /* reflected: the upper end becomes the reference, and the quantile 1 - u */
        delta = hi - bisect_quantile(-b, 0.0, w, uc, u) / d;
    } else {
        delta = (c + bisect_quantile(0.0, a, b, u, uc)) / d;
    }
    if (delta < lo) delta = lo;
    if (delta > hi) delta = hi;
    return delta;
}

/* the pieces, for the pins */
double orc_mills(double x) { return mills(x); }
double orc_mass(double r0, double t1, double t2) { return mass_S(r0, t1, t2); }
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    philox4x32_10(ctr, key, out);
}
int64_t orc_sweep_level(uint64_t seed, int64_t problem, int64_t sweep, int64_t L) {
    return sweep_level(seed, problem, sweep, L);
}
double orc_move_uniform(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep,
                        int64_t block, int64_t mode) {
    return move_uniform(seed, problem, chain, sweep, block, mode);
}

/* ------------------------------------------------------------------------------------ */
/* The sampler.                                                                         */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int64_t M, N, B;        /* B: blocks of all levels together                          */
    const double *Kt;       /* M x N whitened kernel, row-major                          */
    const double *gt;       /* M whitened data                                           */
    const int64_t *bn0;     /* B first grid points                                       */
    const int64_t *bnb;     /* B block sizes                                             */
    int64_t L;              /* levels of the hierarchy (1: one partition)                */
    const int64_t *lfirst;  /* L: first block of each level                              */
    const int64_t *lcount;  /* L: blocks of each level                                   */
    const int32_t *kb;      /* data modes per block                                      */
    const double *d;        /* concatenated data singular values (sum kb)                */
    const double *U;        /* concatenated U_b, each M x kb row-major                   */
    const double *V;        /* concatenated V_b, each Nb x Nb row-major, column = mode   */
    const double *shape_m1; /* N: w_n - 1 of the gamma prior weights, or NULL (flat)      */
    const int64_t *bnm;     /* B modes per block (Nb, or Nb - 1 under a linear constraint),
                               or NULL (Nb); V_b is then Nb x nm row-major               */
} orc_problem;

typedef struct {
    int64_t chains, burnin, sweeps;
    uint64_t seed;
    int64_t problem_index;
    int64_t refresh_every;
    int64_t groups;
    int64_t want_cross;
    int64_t threads;
    int64_t traj_chain;     /* chain whose A is recorded after every sweep, or -1        */
    const double *init;     /* N start vector (shared by all chains), >= 0               */
    const double *vjp_v;    /* N cotangent for per-group VJP moments, or NULL            */
} orc_options;

typedef struct {
    double *sumA;        /* groups x N                                                  */
    double *sumA2;       /* groups x N                                                  */
    int64_t *count;      /* groups                                                      */
    double *sumR;        /* M              (want_cross)                                 */
    double *sumRA;       /* M x N          (want_cross)                                 */
    double *final_A;     /* chains x N                                                  */
    double *final_r;     /* chains x M                                                  */
    double *final_chi2;  /* chains                                                      */
    double *traj_A;      /* (burnin+sweeps) x N, or NULL                                */
    double *traj_chi2;   /* (burnin+sweeps), or NULL                                    */
    double *drift_max;   /* 1                                                           */
    int64_t *n_frozen;   /* 1                                                           */
    int64_t *n_clamped;  /* 1                                                           */
    int32_t *status;     /* 1                                                           */
    int64_t *n_rejected; /* 1: moves rejected by the gamma-prior acceptance test         */
    double *gRv;         /* groups x M: sum r (A . v)       (vjp_v)                      */
    double *gR;          /* groups x M: sum r               (vjp_v)                      */
    double *gAv;         /* groups: sum A . v               (vjp_v)                      */
} orc_out;

typedef struct {
    const orc_problem *p;
    const orc_options *o;
    orc_out *out;
    int64_t c0, c1;
    /* per-thread accumulators */
    double *sumA, *sumA2, *sumR, *sumRA;
    double *gRv, *gR, *gAv;
    int64_t *count;
    double drift;
    int64_t frozen, clamped, rejected;
    int32_t status;
} worker;

static void refresh(const orc_problem *p, const double *A, double *r, double *chi2) {
    double s = 0.0;
    for (int64_t m = 0; m < p->M; ++m) {
        double acc = p->gt[m];
        const double *row = p->Kt + m * p->N;
        for (int64_t n = 0; n < p->N; ++n) acc -= row[n] * A[n];
        r[m] = acc;
        s += acc * acc;
    }
    *chi2 = s;
}

static void *run_chains(void *arg) {
    worker *wk = (worker *)arg;
    const orc_problem *p = wk->p;
    const orc_options *o = wk->o;
    const int64_t M = p->M, N = p->N, B = p->B;
    const int64_t total = o->burnin + o->sweeps;
    double *A = (double *)malloc(sizeof(double) * N);
    double *r = (double *)malloc(sizeof(double) * M);

    /* offsets of each block's factors */
    int64_t *offd = (int64_t *)malloc(sizeof(int64_t) * (B + 1));
    int64_t *offU = (int64_t *)malloc(sizeof(int64_t) * (B + 1));
    int64_t *offV = (int64_t *)malloc(sizeof(int64_t) * (B + 1));
    offd[0] = offU[0] = offV[0] = 0;
    for (int64_t b = 0; b < B; ++b) {
        int64_t nb = p->bnb[b], nm = p->bnm ? p->bnm[b] : nb;
        offd[b + 1] = offd[b] + p->kb[b];
        offU[b + 1] = offU[b] + M * p->kb[b];
        offV[b + 1] = offV[b] + nb * nm;
    }

    for (int64_t c = wk->c0; c < wk->c1; ++c) {
        for (int64_t n = 0; n < N; ++n) A[n] = o->init[n];
        double chi2;
        refresh(p, A, r, &chi2);
        for (int64_t s = 0; s < total; ++s) {
            const int64_t lvl = sweep_level(o->seed, o->problem_index, s, p->L);
            for (int64_t b = 0; b < p->lcount[lvl]; ++b) {
                const int64_t gb = p->lfirst[lvl] + b;   /* the block among all levels */
                const int64_t n0 = p->bn0[gb], nb = p->bnb[gb];
                const int64_t nm = p->bnm ? p->bnm[gb] : nb;   /* modes of the block */
                const int64_t kb = p->kb[gb];
                const double *Vb = p->V + offV[gb];
                const double *Ub = p->U + offU[gb];
                const double *db = p->d + offd[gb];
                for (int64_t i = 0; i < nm; ++i) {
                    /* Eq. (modeLimits): f + delta V_i >= 0 */
                    double lo = -INFINITY, hi = INFINITY;
                    for (int64_t q = 0; q < nb; ++q) {
                        double v = Vb[q * nm + i];
                        if (v > 0.0) {
                            double t = -A[n0 + q] / v;
                            if (t > lo) lo = t;
                        } else if (v < 0.0) {
                            double t = -A[n0 + q] / v;
                            if (t < hi) hi = t;
                        }
                    }
                    double u = move_uniform(o->seed, o->problem_index, c, s, b, i);
                    double delta, cdot = 0.0, dd = 0.0;
                    if (i < kb) {
                        dd = db[i];
                        for (int64_t m = 0; m < M; ++m) cdot += Ub[m * kb + i] * r[m];
                        delta = orc_tn_draw(cdot, dd, lo, hi, u);
                    } else {
                        if (isinf(lo) || isinf(hi)) {
                            wk->status = ORC_EUNBOUNDED;
                            delta = 0.0;
                        } else {
                            delta = lo + u * (hi - lo);
                        }
                    }
                    if (lo == hi) wk->frozen++;
                    if (p->shape_m1) {
                        /* Sec. V.C: the target along the mode carries the weights
                           prod_q A_q^(w_q - 1); the draw above (the Gaussian or flat
                           conditional of the flat-prior posterior) is an independence proposal,
                           accepted with probability min(1, R(delta) / R(0)) */
                        double lr = 0.0;
                        for (int64_t q = 0; q < nb; ++q) {
                            double an = A[n0 + q] + delta * Vb[q * nm + i];
                            if (an < 0.0) an = 0.0;
                            lr += prior_log_ratio(an, A[n0 + q], p->shape_m1[n0 + q]);
                        }
                        double ua = move_uniform_tag(o->seed, o->problem_index, c, s, b, i, 3u);
                        if (!(log(ua) < lr)) {
                            delta = 0.0;
                            wk->rejected++;
                        }
                    }
                    for (int64_t q = 0; q < nb; ++q) {
                        double an = A[n0 + q] + delta * Vb[q * nm + i];
                        if (an < 0.0) {
                            an = 0.0;
                            wk->clamped++;
                        }
                        A[n0 + q] = an;
                    }
                    if (i < kb) {
                        double e = delta * dd;
                        for (int64_t m = 0; m < M; ++m) r[m] -= e * Ub[m * kb + i];
                        chi2 += e * (e - 2.0 * cdot);
                    }
                }
            }
            if (o->refresh_every > 0 && (s + 1) % o->refresh_every == 0) {
                double chi2_ref;
                refresh(p, A, r, &chi2_ref);
                double dr = fabs(chi2 - chi2_ref) / (chi2_ref > 0.0 ? chi2_ref : 1.0);
                if (dr > wk->drift) wk->drift = dr;
                chi2 = chi2_ref;
            }
            if (c == o->traj_chain && wk->out->traj_A) {
                memcpy(wk->out->traj_A + s * N, A, sizeof(double) * N);
                if (wk->out->traj_chi2) wk->out->traj_chi2[s] = chi2;
            }
            if (s >= o->burnin) {
                int64_t g;
                if (o->chains >= o->groups)
                    g = c * o->groups / o->chains;
                else
                    g = (s - o->burnin) * o->groups / o->sweeps;
                double *sa = wk->sumA + g * N, *sa2 = wk->sumA2 + g * N;
                for (int64_t n = 0; n < N; ++n) {
                    sa[n] += A[n];
                    sa2[n] += A[n] * A[n];
                }
                wk->count[g]++;
                if (o->vjp_v) {
                    /* the moments of one group's covariance Cov(r~, A) v (Sec. II, Eq. (PI)
                       differentiated in the data) */
                    double av = 0.0;
                    for (int64_t n = 0; n < N; ++n) av += A[n] * o->vjp_v[n];
                    for (int64_t m = 0; m < M; ++m) {
                        wk->gRv[g * M + m] += r[m] * av;
                        wk->gR[g * M + m] += r[m];
                    }
                    wk->gAv[g] += av;
                }
                if (o->want_cross) {
                    for (int64_t m = 0; m < M; ++m) {
                        wk->sumR[m] += r[m];
                        double *row = wk->sumRA + m * N;
                        for (int64_t n = 0; n < N; ++n) row[n] += r[m] * A[n];
                    }
                }
            }
        }
        memcpy(wk->out->final_A + c * N, A, sizeof(double) * N);
        memcpy(wk->out->final_r + c * M, r, sizeof(double) * M);
        wk->out->final_chi2[c] = chi2;
    }
    free(A); free(r); free(offd); free(offU); free(offV);
    return NULL;
}

int orc_run(const orc_problem *p, const orc_options *o, orc_out *out) {
    int64_t nt = o->threads > 0 ? o->threads : 1;
    if (nt > o->chains) nt = o->chains;
    const int64_t N = p->N, M = p->M, G = o->groups;
    worker *wk = (worker *)calloc((size_t)nt, sizeof(worker));
    pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
    for (int64_t t = 0; t < nt; ++t) {
        wk[t].p = p; wk[t].o = o; wk[t].out = out;
        wk[t].c0 = o->chains * t / nt;
        wk[t].c1 = o->chains * (t + 1) / nt;
        wk[t].sumA = (double *)calloc((size_t)(G * N), sizeof(double));
        wk[t].sumA2 = (double *)calloc((size_t)(G * N), sizeof(double));
        wk[t].count = (int64_t *)calloc((size_t)G, sizeof(int64_t));
        if (o->want_cross) {
            wk[t].sumR = (double *)calloc((size_t)M, sizeof(double));
            wk[t].sumRA = (double *)calloc((size_t)(M * N), sizeof(double));
        }
        if (o->vjp_v) {
            wk[t].gRv = (double *)calloc((size_t)(G * M), sizeof(double));
            wk[t].gR = (double *)calloc((size_t)(G * M), sizeof(double));
            wk[t].gAv = (double *)calloc((size_t)G, sizeof(double));
        }
        pthread_create(&th[t], NULL, run_chains, &wk[t]);
    }
    int32_t status = ORC_OK;
    double drift = 0.0;
    int64_t frozen = 0, clamped = 0, rejected = 0;
    for (int64_t t = 0; t < nt; ++t) {
        pthread_join(th[t], NULL);
        for (int64_t i = 0; i < G * N; ++i) {
            out->sumA[i] += wk[t].sumA[i];
            out->sumA2[i] += wk[t].sumA2[i];
        }
        for (int64_t g = 0; g < G; ++g) out->count[g] += wk[t].count[g];
        if (o->vjp_v) {
            for (int64_t i = 0; i < G * M; ++i) {
                out->gRv[i] += wk[t].gRv[i];
                out->gR[i] += wk[t].gR[i];
            }
            for (int64_t g = 0; g < G; ++g) out->gAv[g] += wk[t].gAv[g];
            free(wk[t].gRv); free(wk[t].gR); free(wk[t].gAv);
        }
        if (o->want_cross) {
            for (int64_t m = 0; m < M; ++m) out->sumR[m] += wk[t].sumR[m];
            for (int64_t i = 0; i < M * N; ++i) out->sumRA[i] += wk[t].sumRA[i];
            free(wk[t].sumR); free(wk[t].sumRA);
        }
        if (wk[t].status != ORC_OK) status = wk[t].status;
        if (wk[t].drift > drift) drift = wk[t].drift;
        frozen += wk[t].frozen;
        clamped += wk[t].clamped;
        rejected += wk[t].rejected;
        free(wk[t].sumA); free(wk[t].sumA2); free(wk[t].count);
    }
    *out->drift_max = drift;
    *out->n_frozen = frozen;
    *out->n_clamped = clamped;
    if (out->n_rejected) *out->n_rejected = rejected;
    *out->status = status;
    free(wk); free(th);
    return status;
}
