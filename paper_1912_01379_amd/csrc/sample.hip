// The two samplers of blocked modes sampling (Sec. IV.B-C).
//
// One move of mode i of block b (data modes, d_i > 0, first; then the zero modes):
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
// reference trajectory).  sample32: many chains per workgroup, `L` lanes per chain, float32
// state, the block's (V, -1/V) staged in LDS and shared by all chains of the workgroup.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "rng_tn.h"

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
    unsigned long long clamped = 0, frozen = 0;
    int unbounded = 0;
    __syncthreads();
    const int64_t s0 = *a.sweep;
    for (int64_t s = s0; s < s0 + a.nsw; ++s) {
        for (int64_t b = 0; b < pd.B; ++b) {
            const BlockDesc bd = a.blocks[pd.off_blk + b];
            const int64_t nb = bd.nb, kb = bd.kb;
            const double *V = a.V64 + bd.off_V;
            const double *U = a.U64 + bd.off_U;
            const double *dv = a.d64 + bd.off_d;
            double *Ab = A + bd.n0;
            for (int64_t i = 0; i < nb; ++i) {
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

// ------------------------------------------------------------------------------------
// float32 batched sampler
// ------------------------------------------------------------------------------------
// Reductions over the L lanes of one chain (the lanes are contiguous and L divides 16 for
// the DPP steps); every lane ends with the same bits.  `update_dpp` with the identity of
// the operation as the old value lets the compiler fold each move into the min/add.
template <int L>
__device__ __forceinline__ uint32_t seg_umin(uint32_t x) {
    if constexpr (L >= 2) x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, 0xB1, 0xF, 0xF, false));
    if constexpr (L >= 4) x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, 0x4E, 0xF, 0xF, false));
    if constexpr (L >= 8) x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, 0x141, 0xF, 0xF, false));
    if constexpr (L >= 16) x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, 0x140, 0xF, 0xF, false));
    if constexpr (L >= 32) x = min(x, (uint32_t)__shfl_xor((int)x, 16));
    if constexpr (L >= 64) x = min(x, (uint32_t)__shfl_xor((int)x, 32));
    return x;
}

template <int L>
__device__ __forceinline__ float seg_sum(float x) {
    if constexpr (L >= 2) x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
    if constexpr (L >= 4) x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
    if constexpr (L >= 8) x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));
    if constexpr (L >= 16) x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));
    if constexpr (L >= 32) x += __shfl_xor(x, 16);
    if constexpr (L >= 64) x += __shfl_xor(x, 32);
    return x;
}

// Interval of Eq. (modeLimits) for one mode from the lane's EPT components.  With
// x_q = A_q * (-1/V_qi) and A_q >= +0, the sign bit of x_q is set exactly when V_qi > 0,
// so the lower limit is -min over those |x_q| and the upper limit the min over the rest;
// both are unsigned minima of the bit patterns.  Padding entries carry a NaN ratio, whose
// patterns lie above +inf in either search, so they never win.
template <int L, int EPT>
__device__ __forceinline__ void interval32(const float2 (&vw)[EPT], const float (&Ar)[EPT], float &lo,
                                           float &hi) {
    uint32_t hb = 0xFFFFFFFFu, lb = 0xFFFFFFFFu;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const uint32_t bits = __float_as_uint(Ar[t] * vw[t].y);
        hb = min(hb, bits);
        lb = min(lb, bits ^ 0x80000000u);
    }
    hb = seg_umin<L>(hb);
    lb = seg_umin<L>(lb);
    hi = hb >= 0x7F800000u ? INFINITY : __uint_as_float(hb);
    lo = lb >= 0x7F800000u ? -INFINITY : -__uint_as_float(lb);
}

// Kept out of line: the inverse-CDF draw is long and only data modes need it, so its
// registers are not added to those of the move loop.
__device__ __noinline__ float tn_draw32(float c, float d, float lo, float hi, float u) {
    return tn_draw_fast32(c, d, lo, hi, u);
}

// L lanes per chain; every lane owns EPT components of the current block (q = lane + L t)
// and RPT residual entries (m = lane + L t).  Block rows are padded to EPT*L with the
// neutral pair (0, NaN), U rows to RPT*L with zeros, so no lane ever branches on a size.
template <int L, int EPT, int RPT>
__global__ __launch_bounds__(512) void k_sample32(SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem32[];
    constexpr int ROW = EPT * L;
    constexpr int MP = RPT * L;
    const int tid = threadIdx.x;
    const int lane = tid % L;
    const int slotc = tid / L;
    float2 *sVW = reinterpret_cast<float2 *>(smem32);
    float *sUnif = reinterpret_cast<float *>(sVW + a.lds_vw);   // chains x ROW
    __shared__ int s_tile;
    const int64_t s0 = *a.sweep;
    const int64_t nsw = a.nsw;

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(a.queue, 1);
        __syncthreads();
        const int tile = s_tile;
        __syncthreads();
        if (tile >= a.ntiles) break;
        const TileDesc td = a.tiles[tile];
        const ProbDesc pd = a.probs[td.problem];
        const int M = (int)pd.M;
        const int64_t N = pd.N;
        const bool active = slotc < td.nchains;
        const int64_t chain = td.chain0 + (active ? slotc : 0);
        float *Ag = a.A32 + pd.off_A + chain * N;
        float *rg = a.r32 + pd.off_r + chain * (int64_t)M;
        float rr[RPT];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int m = lane + L * t;
            rr[t] = (m < M && active) ? rg[m] : 0.0f;
        }
        bool unbounded = false;
        float *urow = sUnif + slotc * ROW;

        for (int64_t s = s0; s < s0 + nsw; ++s) {
            for (int64_t b = 0; b < pd.B; ++b) {
                const BlockDesc bd = a.blocks[pd.off_blk + b];
                const int nb = (int)bd.nb, kb = (int)bd.kb;
                __syncthreads();
                {   // stage the block's (V, -1/V) rows
                    const float4 *src = reinterpret_cast<const float4 *>(a.VW32 + bd.off_VW);
                    float4 *dst = reinterpret_cast<float4 *>(sVW);
                    const int n4 = nb * ROW / 2;
                    for (int i = tid; i < n4; i += blockDim.x) dst[i] = src[i];
                }
                // this block's uniforms: one Philox call per four modes
                for (int g = lane; 4 * g < nb; g += L) {
                    const U4 w = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s,
                                              (uint32_t)b, (uint32_t)g);
                    float *d = urow + 4 * g;
                    d[0] = word_u32(w.x);
                    d[1] = word_u32(w.y);
                    d[2] = word_u32(w.z);
                    d[3] = word_u32(w.w);
                }
                __syncthreads();
                float Ar[EPT];
#pragma unroll
                for (int t = 0; t < EPT; ++t) {
                    const int q = lane + L * t;
                    Ar[t] = (q < nb && active) ? Ag[bd.n0 + q] : 0.0f;
                }
                const float *U = a.U32 + bd.off_U32;
                const float *dv = a.d32 + bd.off_d32;
                float2 vw[EPT];
#pragma unroll
                for (int t = 0; t < EPT; ++t) vw[t] = sVW[lane + L * t];
                for (int i = 0; i < nb; ++i) {
                    // next row, loaded while this move is computed
                    const float2 *nrow = sVW + (i + 1 < nb ? i + 1 : i) * ROW;
                    float2 vn[EPT];
#pragma unroll
                    for (int t = 0; t < EPT; ++t) vn[t] = nrow[lane + L * t];
                    float lo, hi;
                    interval32<L, EPT>(vw, Ar, lo, hi);
                    const float u = urow[i];
                    float delta;
                    if (i < kb) {
                        const float *Ui = U + i * MP;
                        float cp = 0.0f;
#pragma unroll
                        for (int t = 0; t < RPT; ++t) cp = fmaf(Ui[lane + L * t], rr[t], cp);
                        const float cdot = seg_sum<L>(cp);
                        const float dd = dv[i];
                        delta = tn_draw32(cdot, dd, lo, hi, u);
                        const float e = delta * dd;
#pragma unroll
                        for (int t = 0; t < RPT; ++t) rr[t] = fmaf(-e, Ui[lane + L * t], rr[t]);
                    } else {
                        const bool inf = __builtin_isinf(lo) || __builtin_isinf(hi);
                        unbounded |= inf;
                        delta = inf ? 0.0f : fmaf(u, hi - lo, lo);
                    }
#pragma unroll
                    for (int t = 0; t < EPT; ++t) {
                        Ar[t] = fmaxf(fmaf(delta, vw[t].x, Ar[t]), 0.0f);
                        vw[t] = vn[t];
                    }
                }
#pragma unroll
                for (int t = 0; t < EPT; ++t) {
                    const int q = lane + L * t;
                    if (active && q < nb) Ag[bd.n0 + q] = Ar[t];
                }
                if (a.accumulate && s >= a.burnin) {
                    // per-tile sums over the tile's chains, float64, owned by this workgroup
#pragma unroll
                    for (int t = 0; t < EPT; ++t) urow[lane + L * t] = active ? Ar[t] : 0.0f;
                    __syncthreads();
                    int64_t slot = td.slot;
                    if (pd.batches > 1) slot += (s - a.burnin) * pd.batches / a.sweeps;
                    double *s1 = a.accA + pd.off_slot + slot * N + bd.n0;
                    double *s2 = a.accA2 + pd.off_slot + slot * N + bd.n0;
                    for (int q = tid; q < nb; q += blockDim.x) {
                        double x1 = 0.0, x2 = 0.0;
                        for (int cs = 0; cs < td.nchains; ++cs) {
                            const double x = (double)sUnif[cs * ROW + q];
                            x1 += x;
                            x2 += x * x;
                        }
                        s1[q] += x1;
                        s2[q] += x2;
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int m = lane + L * t;
            if (active && m < M) rg[m] = rr[t];
        }
        if (unbounded) atomicOr(a.flags, 1);
    }
}

// The compiled instances: (lanes per chain, components per lane, residual entries per lane).
struct Inst32 {
    int L, EPT, RPT;
};
static const Inst32 kInst32[] = {{16, 7, 16}, {16, 8, 32}, {16, 2, 4}, {8, 13, 32}, {8, 16, 64},
                                 {4, 32, 32}, {32, 4, 16}};

int sample32_pick(int lanes, int64_t max_nb, int64_t max_m, int *ept, int *rpt) {
    int best = -1;
    for (int k = 0; k < (int)(sizeof kInst32 / sizeof kInst32[0]); ++k) {
        const Inst32 &c = kInst32[k];
        if (c.L != lanes || (int64_t)c.EPT * c.L < max_nb || (int64_t)c.RPT * c.L < max_m) continue;
        if (best < 0 || c.EPT * 4 + c.RPT < kInst32[best].EPT * 4 + kInst32[best].RPT) best = k;
    }
    if (best < 0) return -1;
    *ept = kInst32[best].EPT;
    *rpt = kInst32[best].RPT;
    return 0;
}

template <int L, int EPT, int RPT>
static hipError_t launch_one(const SampleArgs &a, int threads, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_sample32<L, EPT, RPT>), dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_sample32_inst(const SampleArgs &a, int lanes, int ept, int rpt, int chains_per_wg,
                                int grid, size_t lds_bytes, hipStream_t s) {
    const int threads = lanes * chains_per_wg;
    if (threads % 64 != 0 || threads > 512) return hipErrorInvalidValue;
#define INST(L_, E_, R_) \
    if (lanes == L_ && ept == E_ && rpt == R_) return launch_one<L_, E_, R_>(a, threads, grid, lds_bytes, s);
    INST(16, 7, 16)
    INST(16, 8, 32)
    INST(16, 2, 4)
    INST(8, 13, 32)
    INST(8, 16, 64)
    INST(4, 32, 32)
    INST(32, 4, 16)
#undef INST
    return hipErrorInvalidValue;
}

hipError_t set_sample32_lds_limit() {
    // allow up to 160 KB of LDS per workgroup on gfx950 (best effort)
#define ATTR(L_, E_, R_) \
    (void)hipFuncSetAttribute((const void *)k_sample32<L_, E_, R_>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    ATTR(16, 7, 16)
    ATTR(16, 8, 32)
    ATTR(16, 2, 4)
    ATTR(8, 13, 32)
    ATTR(8, 16, 64)
    ATTR(4, 32, 32)
    ATTR(32, 4, 16)
#undef ATTR
    return hipFuncSetAttribute((const void *)k_sample64, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

// ------------------------------------------------------------------------------------
// small kernels: sweep counter, tile queue, and test entry points
// ------------------------------------------------------------------------------------
__global__ void k_bump(int64_t *sweep, int64_t by, int *queue) {
    if (threadIdx.x == 0) {
        *sweep += by;
        if (queue) *queue = 0;
    }
}

__global__ void k_reset_queue(int *queue) {
    if (threadIdx.x == 0) *queue = 0;
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
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (precision == ASM_FP64) {
        out[i] = tn_draw<double>(c[i], d[i], lo[i], hi[i], u[i]);
    } else {
        out[i] = (double)tn_draw_fast32((float)c[i], (float)d[i], (float)lo[i], (float)hi[i],
                                        (float)u[i]);
    }
}

hipError_t launch_tn_draw(const double *c, const double *d, const double *lo, const double *hi,
                          const double *u, double *out, int64_t n, int precision, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tn_draw, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, c, d, lo, hi, u,
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
