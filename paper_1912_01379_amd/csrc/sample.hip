// The two samplers of blocked modes sampling (Sec. IV.B-C).
//
// A sweep moves every mode of every block of one partition, blocks in increasing order; with
// a hierarchy of partitions (Fig. 2) the partition is the sweep's level, drawn for all chains
// of the problem at once.  One move of mode i of block b (data modes, d_i > 0, first; then
// the zero modes):
//   1. interval of the step delta along V_i that keeps the block non-negative,
//      Eq. (modeLimits): lo = max_{V_qi>0} -A_q/V_qi, hi = min_{V_qi<0} -A_q/V_qi;
//   2. a uniform number of the counter-based generator keyed by (chain, sweep, b, i);
//   3. data mode: c = U_i . r (r = g~ - K~ A, the whitened residual), and delta from the
//      Gaussian N(c/d_i, 1/d_i^2) truncated to [lo, hi]; zero mode: delta uniform on
//      [lo, hi] (the flat distribution of Sec. IV.B);
//   4. A_b += delta V_i (components rounding below zero are set to +0);
//   5. data mode: r -= delta d_i U_i (K~_b V_i = d_i U_i), chi^2 += e (e - 2c), e = delta d_i.
//
// sample64: one wavefront per chain, float64 state (the plain sampler; reproduces the CPU
// reference trajectory).  The batched float32 sampler is in sample32.h.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "rng_tn.h"
#include "tn32.h"

namespace asmk {

// ------------------------------------------------------------------------------------
// float64 sampler: one 64-lane wavefront per chain
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double wsum64(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wmax64(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wmin64(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// (w - 1) log(a_new / a_old): one component's share of the log ratio of the gamma-prior
// weights prod_n A_n^(w_n - 1) (Sec. V.C) between the proposed and the current state
__device__ __forceinline__ double prior_term(double a_new, double a_old, double wm1) {
    if (wm1 == 0.0 || a_new == a_old) return 0.0;
    if (a_old == 0.0) return wm1 > 0.0 ? INFINITY : -INFINITY;
    if (a_new == 0.0) return wm1 > 0.0 ? -INFINITY : INFINITY;
    return wm1 * log(a_new / a_old);
}

__global__ __launch_bounds__(64) void k_sample64(SampleArgs a, const int32_t *chain_problem,
                                                 const int32_t *chain_local) {
    extern __shared__ double sm64[];
    const int lane = threadIdx.x;
    const int p = chain_problem[blockIdx.x];
    const int64_t c = chain_local[blockIdx.x];
    const ProbDesc pd = a.probs[p];
    const int64_t M = pd.M, N = pd.N;
    double *A = sm64;        // N
    double *r = sm64 + N;    // M
    double *Ag = a.A64 + pd.off_A + c * N;
    double *rg = a.r64 + pd.off_r + c * M;
    for (int64_t n = lane; n < N; n += 64) A[n] = Ag[n];
    for (int64_t m = lane; m < M; m += 64) r[m] = rg[m];
    double chi2 = a.chi2[pd.off_c + c];
    double drift = a.drift[pd.off_c + c];
    const double *Kc = a.Kt + pd.off_K;
    const double *gc = a.gt + pd.off_m;
    unsigned long long clamped = 0, frozen = 0, rejected = 0;
    const double *wsh = pd.has_prior ? a.shape + pd.off_n : nullptr;
    int unbounded = 0;
    __syncthreads();
    const int64_t s0 = *a.sweep;
    for (int64_t s = s0; s < s0 + a.nsw; ++s) {
        // the sweep's level of the hierarchy (Fig. 2): its blocks are [lf, lf + lc); the
        // moves are keyed by the block's index within the level
        int64_t lf = 0, lc = pd.B;
        if (pd.levels > 1) {
            const int64_t l = sweep_level(a.seed, pd.index, (uint32_t)s, (uint32_t)pd.levels);
            lf = a.lvl[2 * (pd.off_lvl + l)];
            lc = a.lvl[2 * (pd.off_lvl + l) + 1];
        }
        for (int64_t b = 0; b < lc; ++b) {
            const BlockDesc bd = a.blocks[pd.off_blk + lf + b];
            const int64_t nb = bd.nb, kb = bd.kb;
            const double *V = a.V64 + bd.off_V;
            const double *U = a.U64 + bd.off_U;
            const double *dv = a.d64 + bd.off_d;
            double *Ab = A + bd.n0;
            for (int64_t i = 0; i < bd.nm; ++i) {   // modes: nb, or nb - 1 under a constraint
                const double *Vi = V + i * nb;
                double lo = -INFINITY, hi = INFINITY;
                for (int64_t q = lane; q < nb; q += 64) {
                    const double v = Vi[q];
                    if (v > 0.0) lo = fmax(lo, -Ab[q] / v);
                    else if (v < 0.0) hi = fmin(hi, -Ab[q] / v);
                }
                lo = wmax64(lo);
                hi = wmin64(hi);
                const double u = move_u64(a.seed, pd.index, (uint32_t)c, (uint32_t)s, (uint32_t)b,
                                          (uint32_t)i);
                double delta, cdot = 0.0, dd = 0.0;
                if (i < kb) {
                    const double *Ui = U + i * M;
                    for (int64_t m = lane; m < M; m += 64) cdot += Ui[m] * r[m];
                    cdot = wsum64(cdot);
                    dd = dv[i];
                    delta = tn_draw<double>(cdot, dd, lo, hi, u);
                } else if (__builtin_isinf(lo) || __builtin_isinf(hi)) {
                    unbounded = 1;
                    delta = 0.0;
                } else {
                    delta = __dadd_rn(lo, __dmul_rn(u, __dadd_rn(hi, -lo)));
                }
                frozen += (lo == hi);
                if (wsh) {
                    // gamma prior (Sec. V.C): the draw is a proposal along the mode, accepted
                    // with probability min(1, R(delta) / R(0)), R = prod_q A_q^(w_q - 1)
                    double lr = 0.0;
                    for (int64_t q = lane; q < nb; q += 64) {
                        double an = __dadd_rn(Ab[q], __dmul_rn(delta, Vi[q]));
                        if (an < 0.0) an = 0.0;
                        lr += prior_term(an, Ab[q], wsh[bd.n0 + q] - 1.0);
                    }
                    lr = wsum64(lr);
                    const double ua = move_u64(a.seed, pd.index, (uint32_t)c, (uint32_t)s, (uint32_t)b,
                                               (uint32_t)i, 3u);
                    if (!(log(ua) < lr)) {
                        delta = 0.0;
                        rejected += (lane == 0);
                    }
                }
                for (int64_t q = lane; q < nb; q += 64) {
                    double an = __dadd_rn(Ab[q], __dmul_rn(delta, Vi[q]));
                    if (an < 0.0) {
                        an = 0.0;
                        ++clamped;
                    }
                    Ab[q] = an;
                }
                if (i < kb) {
                    const double *Ui = U + i * M;
                    const double e = __dmul_rn(delta, dd);
                    for (int64_t m = lane; m < M; m += 64) r[m] = __dadd_rn(r[m], -__dmul_rn(e, Ui[m]));
                    chi2 = __dadd_rn(chi2, __dmul_rn(e, __dadd_rn(e, -2.0 * cdot)));
                }
            }
        }
        if (a.refresh_every > 0 && (s + 1) % a.refresh_every == 0) {
            __syncthreads();
            double ss = 0.0;
            for (int64_t m = lane; m < M; m += 64) {
                double acc = gc[m];
                const double *row = Kc + m * N;
                for (int64_t n = 0; n < N; ++n) acc = __dadd_rn(acc, -__dmul_rn(row[n], A[n]));
                r[m] = acc;
                ss += acc * acc;
            }
            ss = wsum64(ss);
            const double dr = fabs(chi2 - ss) / (ss > 0.0 ? ss : 1.0);
            drift = fmax(drift, dr);
            chi2 = ss;
            __syncthreads();
        }
        if (a.accumulate && s >= a.burnin) {
            int64_t slot = c * pd.batches;
            if (pd.batches > 1) slot += (s - a.burnin) * pd.batches / a.sweeps;
            double *s1 = a.accA + pd.off_slot + slot * N;
            double *s2 = a.accA2 + pd.off_slot + slot * N;
            for (int64_t n = lane; n < N; n += 64) {
                const double x = A[n];
                s1[n] += x;
                s2[n] += x * x;
            }
        }
    }
    __syncthreads();
    for (int64_t n = lane; n < N; n += 64) Ag[n] = A[n];
    for (int64_t m = lane; m < M; m += 64) rg[m] = r[m];
    if (clamped) atomicAdd(&a.counters[0], clamped);
    if (lane == 0) {
        a.chi2[pd.off_c + c] = chi2;
        a.drift[pd.off_c + c] = drift;
        if (frozen) atomicAdd(&a.counters[1], frozen);
        if (rejected) atomicAdd(&a.counters[2], rejected);
        if (unbounded) atomicOr(a.flags, 1);
    }
}

hipError_t launch_sample64_grid(const SampleArgs &a, int64_t total_chains, const int32_t *chain_problem,
                                const int32_t *chain_local, size_t lds_bytes, hipStream_t s) {
    if (total_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample64, dim3((unsigned)total_chains), dim3(64), lds_bytes, s, a,
                       chain_problem, chain_local);
    return hipGetLastError();
}

hipError_t set_sample64_lds_limit() {
    return hipFuncSetAttribute((const void *)k_sample64, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

// ------------------------------------------------------------------------------------
// small kernels: sweep counter, tile queue, and test entry points
// ------------------------------------------------------------------------------------
// the float32 samplers' tile queue: kTileQueues range counters
constexpr int kTileQueues = 8;

__global__ void k_bump(int64_t *sweep, int64_t by, int *queue) {
    if (threadIdx.x == 0) *sweep += by;
    if (queue && threadIdx.x < kTileQueues) queue[threadIdx.x] = 0;
}

__global__ void k_reset_queue(int *queue) {
    if (threadIdx.x < kTileQueues) queue[threadIdx.x] = 0;
}

hipError_t launch_bump(int64_t *sweep, int64_t by, int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, sweep, by, queue);
    return hipGetLastError();
}

hipError_t launch_reset_queue(int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, queue);
    return hipGetLastError();
}

__global__ void k_tn_draw(const double *c, const double *d, const double *lo, const double *hi,
                          const double *u, double *out, int64_t n, int precision) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (precision == ASM_FP64) {
        if (t >= n) return;
        out[t] = tn_draw<double>(c[t], d[t], lo[t], hi[t], u[t]);
    } else {
        // the float32 draw runs on a pair of lanes with the same arguments, as in the sampler
        const int64_t i = t / 2;
        if (i >= n) return;
        const float v = tn_draw32((float)c[i], (float)d[i], (float)lo[i], (float)hi[i], (float)u[i]);
        if ((t & 1) == 0) out[i] = (double)v;
    }
}

hipError_t launch_tn_draw(const double *c, const double *d, const double *lo, const double *hi,
                          const double *u, double *out, int64_t n, int precision, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t threads = precision == ASM_FP64 ? n : 2 * n;
    hipLaunchKernelGGL(k_tn_draw, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, c, d, lo, hi, u,
                       out, n, precision);
    return hipGetLastError();
}

__global__ void k_uniforms(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep0,
                           int64_t nsweeps, int64_t nblocks, int64_t nmodes, double *out) {
    const int64_t total = nsweeps * nblocks * nmodes;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i % nmodes, b = (i / nmodes) % nblocks, s = i / (nmodes * nblocks);
        out[i] = move_u64(seed, (uint32_t)problem, (uint32_t)chain, (uint32_t)(sweep0 + s),
                          (uint32_t)b, (uint32_t)m);
    }
}

hipError_t launch_uniforms(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep0,
                           int64_t nsweeps, int64_t nblocks, int64_t nmodes, double *out,
                           hipStream_t s) {
    const int64_t total = nsweeps * nblocks * nmodes;
    if (total <= 0) return hipSuccess;
    int grid = (int)((total + 255) / 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_uniforms, dim3(grid), dim3(256), 0, s, seed, problem, chain, sweep0,
                       nsweeps, nblocks, nmodes, out);
    return hipGetLastError();
}

}  // namespace asmk
