// Batched float32 sampler of blocked modes sampling (Sec. IV.B-C).
//
// L lanes of one wavefront carry one chain; a workgroup carries `cpw` chains of one problem
// (a tile) and walks the blocks of that problem in order.  For each block the workgroup
// stages the block's factors in LDS, shared by all its chains, by copying the block's packed
// chunk (setup.hip), which is the image of the staging area:
//   (V_qi, w_qi) pairs, w ~ -1/V, mode-major rows of ROW = EPT L entries (padding (0, NaN)),
//   the singular values, and U_i rows of MP = RPT L entries (padding 0) when they fit,
// and each chain draws the block's uniforms into its own LDS row.  A lane owns components
// q = lane + L t (t < EPT) of the block, in registers, and residual entries m = lane + L t
// (t < RPT), in registers for the whole launch.
//
// One move of mode i (the oracle's order: data modes i < k_b first, then the zero modes):
//   1. interval of Eq. (modeLimits): x_q = A_q (-1/V_qi); x_q <= 0 (sign bit set) exactly
//      when V_qi > 0, so lo is the signed-integer minimum of the bit patterns (the negative
//      x closest to zero) and hi their unsigned minimum (the smallest non-negative x);
//      padding and V_qi = 0 give a NaN x, which neither minimum can select;
//   2. data mode: c = U_i . r and delta from the truncated normal (tn32.h); zero mode:
//      delta = lo + u (hi - lo);
//   3. A_q += delta V_qi (non-negative by construction, see zero_move); data mode:
//      r -= delta d_i U_i.
// Sums over the L lanes of a chain use DPP row operations (L <= 16) or lane shuffles.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <utility>

#include "internal.h"
#include "rng_tn.h"
#include "tn32.h"

namespace asmk {

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
__device__ __forceinline__ int32_t seg_imin(int32_t x) {
    if constexpr (L >= 2) x = min(x, __builtin_amdgcn_update_dpp(0x7FFFFFFF, x, 0xB1, 0xF, 0xF, false));
    if constexpr (L >= 4) x = min(x, __builtin_amdgcn_update_dpp(0x7FFFFFFF, x, 0x4E, 0xF, 0xF, false));
    if constexpr (L >= 8) x = min(x, __builtin_amdgcn_update_dpp(0x7FFFFFFF, x, 0x141, 0xF, 0xF, false));
    if constexpr (L >= 16) x = min(x, __builtin_amdgcn_update_dpp(0x7FFFFFFF, x, 0x140, 0xF, 0xF, false));
    if constexpr (L >= 32) x = min(x, __shfl_xor(x, 16));
    if constexpr (L >= 64) x = min(x, __shfl_xor(x, 32));
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

// Interval [lo, hi] of the step along one mode (Eq. (modeLimits)) from the lane's EPT
// components; every lane of the chain ends with the same values.  Without `bounded` an
// unsigned minimum at or above the pattern of +inf means no finite non-negative x (hi =
// +inf), and a signed minimum at or above the pattern of -inf means no finite negative x
// nor -0 (lo = -inf).  Zero modes are `bounded`: both ends are finite by construction.
template <int L, int EPT, bool bounded>
__device__ __forceinline__ void interval32(const float2 (&vw)[EPT], const float (&Ar)[EPT], float &lo,
                                           float &hi) {
    // two partial minima of each kind (even and odd t), so that the chains of dependent
    // minimum instructions are half as long; the minimum is exact in any order
    uint32_t hb = 0xFFFFFFFFu, hb1 = 0xFFFFFFFFu;
    int32_t lb = 0x7FFFFFFF, lb1 = 0x7FFFFFFF;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const uint32_t bits = __float_as_uint(Ar[t] * vw[t].y);
        if (t & 1) {
            hb1 = min(hb1, bits);
            lb1 = min(lb1, (int32_t)bits);
        } else {
            hb = min(hb, bits);
            lb = min(lb, (int32_t)bits);
        }
    }
    hb = min(hb, hb1);
    lb = min(lb, lb1);
    hb = seg_umin<L>(hb);
    lb = seg_imin<L>(lb);
    if (!bounded) {
        hb = min(hb, 0x7F800000u);
        lb = min(lb, (int32_t)0xFF800000u);
    }
    hi = __uint_as_float(hb);
    lo = __int_as_float(lb);
}

// One zero-mode move (d_i = 0: flat on [lo, hi]).  The packed ratios are shrunk by 2^-21
// relative to -1/V, so the computed interval lies inside the exact one; with delta clamped
// into it, every A_q + delta V_q is non-negative before rounding, hence after it, and no
// component needs clamping.  Every zero mode has a finite interval: a mode whose V has
// entries of only one sign makes the posterior improper and is rejected before sampling.
// Gamma-prior weights prod_q A_q^(w_q - 1) (Sec. V.C): per lane the exponents w_q - 1 of its
// components (0 on padding) and their log2, kept current so that a move needs one logarithm
// per component; rejections are counted on the chain's first lane.
template <int EPT>
struct PriorRegs {
    float W[EPT];
    float Lg[EPT];
    unsigned rej;
};

// The acceptance test of a proposed step: log2 u' < sum_q (w_q - 1) log2(A'_q / A_q), a term
// being 0 where w_q = 1 or A'_q = A_q (the infinite cases at A = 0 follow the signs).
// Returns the step, or 0 when rejected; every lane of the chain takes the same decision.
template <int L, int EPT>
__device__ __forceinline__ float prior_accept(const float2 (&vw)[EPT], const float (&Ar)[EPT],
                                              PriorRegs<EPT> &pr, float delta, float ua, int lane) {
    float Ln[EPT];
    float lr = 0.0f;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const float an = fmaf(delta, vw[t].x, Ar[t]);
        Ln[t] = __log2f(an);
        lr += (pr.W[t] == 0.0f || an == Ar[t]) ? 0.0f : pr.W[t] * (Ln[t] - pr.Lg[t]);
    }
    lr = seg_sum<L>(lr);
    const bool acc = __log2f(ua) < lr;
#pragma unroll
    for (int t = 0; t < EPT; ++t) pr.Lg[t] = acc ? Ln[t] : pr.Lg[t];
    pr.rej += (!acc && lane == 0) ? 1u : 0u;
    return acc ? delta : 0.0f;
}

template <int L, int EPT, bool P = false>
__device__ __forceinline__ void zero_move(const float2 (&vw)[EPT], float (&Ar)[EPT], float u,
                                          PriorRegs<EPT> *pr = nullptr, float ua = 0.0f, int lane = 0) {
    float lo, hi;
    interval32<L, EPT, true>(vw, Ar, lo, hi);
    float delta = __builtin_amdgcn_fmed3f(fmaf(u, hi - lo, lo), lo, hi);
    if constexpr (P) delta = prior_accept<L, EPT>(vw, Ar, *pr, delta, ua, lane);
#pragma unroll
    for (int t = 0; t < EPT; ++t) Ar[t] = fmaf(delta, vw[t].x, Ar[t]);
}

template <int EPT>
__device__ __forceinline__ void load_row(float2 (&vw)[EPT], const float2 *row, int lane, int L) {
#pragma unroll
    for (int t = 0; t < EPT; ++t) vw[t] = row[lane + L * t];
}

// Data modes by the projection identity (Sec. IV.B-C): a data move of mode j changes r by a
// multiple of U_j, and U_i . U_j = 0 for i != j, so the Gaussian centre c_i = U_i . r of every
// other data mode of the block is the same before and after it.  The block's centres are
// therefore formed once as it is entered (c = U_b^T r), and r takes the block's steps
// e_i = delta_i d_i in one update as it is left (r -= U_b e).  Between the two passes a move is
// the interval, the truncated-normal draw and the update of A: the residual leaves the chain of
// dependent instructions of the moves.  sc is the chain's LDS row: c_0..c_{kb-1}, then the steps
// e_0..e_{kb-1} at sc + KCE.

template <int L, int RPT>
__device__ __forceinline__ void load_u(float (&Ui)[RPT], const float *U, int row, int lane) {
    constexpr int MP = RPT * L;
#pragma unroll
    for (int t = 0; t < RPT; ++t) Ui[t] = U[row * MP + lane + L * t];
}

// c_i = U_i . r for i < kb, written to sc[i] by the chain's first lane; the next row is loaded
// while the current one is reduced
template <int L, int RPT>
__device__ __forceinline__ void centres(int kb, const float *U, const float (&rr)[RPT], int lane, float *sc) {
    if (kb <= 0) return;
    float Ua[RPT];
    load_u<L, RPT>(Ua, U, 0, lane);
    for (int i = 0; i < kb; ++i) {
        float Ub[RPT];
        load_u<L, RPT>(Ub, U, i + 1 < kb ? i + 1 : i, lane);
        float c0 = 0.0f, c1 = 0.0f;   // two partial sums for a shorter dependence chain
#pragma unroll
        for (int t = 0; t < RPT; t += 2) c0 = fmaf(Ua[t], rr[t], c0);
#pragma unroll
        for (int t = 1; t < RPT; t += 2) c1 = fmaf(Ua[t], rr[t], c1);
        const float c = seg_sum<L>(c0 + c1);
        if (lane == 0) sc[i] = c;
#pragma unroll
        for (int t = 0; t < RPT; ++t) Ua[t] = Ub[t];
    }
}

// r -= sum_i e_i U_i over the block's data modes (the steps from sc)
template <int L, int RPT>
__device__ __forceinline__ void residual_update(int kb, const float *U, const float *se, int lane, float (&rr)[RPT]) {
    if (kb <= 0) return;
    float Ua[RPT];
    load_u<L, RPT>(Ua, U, 0, lane);
    for (int i = 0; i < kb; ++i) {
        float Ub[RPT];
        load_u<L, RPT>(Ub, U, i + 1 < kb ? i + 1 : i, lane);
        const float e = se[i];
#pragma unroll
        for (int t = 0; t < RPT; ++t) rr[t] = fmaf(-e, Ua[t], rr[t]);
#pragma unroll
        for (int t = 0; t < RPT; ++t) Ua[t] = Ub[t];
    }
}

// One data-mode move: interval, the truncated-normal step about the centre c, the update of A;
// the step e = delta d goes to se (by the chain's first lane) for the residual update.
template <int L, int EPT, bool P = false>
__device__ __forceinline__ void data_move(const float2 (&vw)[EPT], float c, float u, float dd, float (&Ar)[EPT],
                                          float *se, int lane, PriorRegs<EPT> *pr = nullptr, float ua = 0.0f) {
    float lo, hi;
    interval32<L, EPT, false>(vw, Ar, lo, hi);
    float delta = tn_draw32(c, dd, lo, hi, u);
    if constexpr (P) delta = prior_accept<L, EPT>(vw, Ar, *pr, delta, ua, lane);
    if (lane == 0) *se = delta * dd;
#pragma unroll
    for (int t = 0; t < EPT; ++t) Ar[t] = fmaf(delta, vw[t].x, Ar[t]);
}

// The data-mode moves of one block (d_i > 0, modes 0..kb-1): the centres, the moves two per
// iteration with the next (V, w) row loaded one move ahead, the residual update.  On entry vw
// holds row 0; on return row kb.  U is the block's U rows (LDS or global memory).
template <int L, int EPT, int RPT, bool P = false>
__device__ __forceinline__ void data_moves(int kb, const float2 *sVW, const float *sD, const float *U,
                                           const float *urow, float *sc, int kce, int lane, float2 (&vw)[EPT],
                                           float (&Ar)[EPT], float (&rr)[RPT], PriorRegs<EPT> *pr = nullptr,
                                           const float *urowA = nullptr) {
    constexpr int ROW = EPT * L;
    if (kb <= 0) return;
    centres<L, RPT>(kb, U, rr, lane, sc);
    float *se = sc + kce;
    int i = 0;
    for (; i + 2 <= kb; i += 2) {
        float2 vb[EPT];
        load_row<EPT>(vb, sVW + (i + 1) * ROW, lane, L);
        const float u0 = urow[i], u1 = urow[i + 1], d0 = sD[i], d1 = sD[i + 1], c0 = sc[i], c1 = sc[i + 1];
        float a0 = 0.0f, a1 = 0.0f;
        if constexpr (P) {
            a0 = urowA[i];
            a1 = urowA[i + 1];
        }
        data_move<L, EPT, P>(vw, c0, u0, d0, Ar, se + i, lane, pr, a0);
        load_row<EPT>(vw, sVW + (i + 2) * ROW, lane, L);
        data_move<L, EPT, P>(vb, c1, u1, d1, Ar, se + i + 1, lane, pr, a1);
    }
    if (i < kb) {
        float a0 = 0.0f;
        if constexpr (P) a0 = urowA[i];
        data_move<L, EPT, P>(vw, sc[i], urow[i], sD[i], Ar, se + i, lane, pr, a0);
        load_row<EPT>(vw, sVW + (i + 1) * ROW, lane, L);
    }
    residual_update<L, RPT>(kb, U, se, lane, rr);
}

// The zero modes of one block (modes kb..nm-1) with the gamma-prior test, three per iteration,
// each row loaded two moves ahead, as in the sampler's own loop.  On entry vw holds row kb.
template <int L, int EPT, bool P>
__device__ __forceinline__ void zero_moves(int kb, int nm, const float2 *sVW, const float *urow,
                                           const float *urowA, int lane, float2 (&vw)[EPT],
                                           float (&Ar)[EPT], PriorRegs<EPT> *pr) {
    constexpr int ROW = EPT * L;
    int i = kb;
    float2 vb[EPT], vc[EPT];
    load_row<EPT>(vb, sVW + (i + 1) * ROW, lane, L);
    auto ua = [&](int j) { return P ? urowA[j] : 0.0f; };
    for (; i + 3 <= nm; i += 3) {
        load_row<EPT>(vc, sVW + (i + 2) * ROW, lane, L);
        const float u0 = urow[i], u1 = urow[i + 1], u2 = urow[i + 2];
        zero_move<L, EPT, P>(vw, Ar, u0, pr, ua(i), lane);
        load_row<EPT>(vw, sVW + (i + 3) * ROW, lane, L);
        zero_move<L, EPT, P>(vb, Ar, u1, pr, ua(i + 1), lane);
        load_row<EPT>(vb, sVW + (i + 4) * ROW, lane, L);
        zero_move<L, EPT, P>(vc, Ar, u2, pr, ua(i + 2), lane);
    }
    if (i < nm) zero_move<L, EPT, P>(vw, Ar, urow[i], pr, ua(i), lane);
    if (i + 1 < nm) zero_move<L, EPT, P>(vb, Ar, urow[i + 1], pr, ua(i + 1), lane);
}

// The sums of A and A^2 over the measured sweeps (Eq. (MCint)), kept in float64.  A block's
// components at the end of its visit in sweep s are the chain's state after sweep s (the
// partition's blocks are disjoint), so each visit adds its components to the sums of its sweep.
// The chains of one wavefront are summed by a butterfly over the lanes that hold the same
// component (float64, the squares exact), and the groups of L lanes then split the
// read-modify-writes of the wavefront's accumulator slot, which no other wavefront touches: no
// atomics, and a fixed order of additions.  The read of each read-modify-write is issued ahead
// (acc_read_ahead, before the block's zero modes, which touch no global memory), so its latency
// is hidden behind them; acc_block adds and stores.
template <int L, int EPT>
struct AccAhead {
    static constexpr int GW = 64 / L;                 // chains per wavefront
    static constexpr int KA = (EPT + GW - 1) / GW;    // components t = grp + GW j a lane updates
    double a[KA], a2[KA];
};

// The slot entries the lane updates.  The loads are unconditional (clamped into the block) so
// that no branch leaves the compiler's wait counts inexact; the values of lanes that store
// nothing are never used.  The slot's previous update was stored a block visit earlier by the
// same wavefront.
template <int L, int EPT>
__device__ __forceinline__ void acc_read_ahead(AccAhead<L, EPT> &h, const double *accA, const double *accA2,
                                               int64_t n0, int nb, int wlane) {
    constexpr int GW = 64 / L;
    const int lane = wlane % L, grp = wlane / L;
#pragma unroll
    for (int j = 0; j < AccAhead<L, EPT>::KA; ++j) {
        const int t = min(grp + GW * j, EPT - 1);
        const int64_t q = n0 + min(lane + L * t, nb - 1);
        h.a[j] = accA[q];
        h.a2[j] = accA2[q];
    }
}

template <int L, int EPT>
__device__ __forceinline__ void acc_block(double *accA, double *accA2, int64_t n0, int nb, int wlane, bool active,
                                          const float (&Ar)[EPT], const AccAhead<L, EPT> &h) {
    constexpr int GW = 64 / L;
    double s1[EPT], s2[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        // the empty chain slots of a partial tile carry no chain: they add nothing
        const double x = active ? (double)Ar[t] : 0.0;
        s1[t] = x;
        s2[t] = x * x;
    }
    constexpr int STEPS = (L == 64) ? 0 : (L == 32) ? 1 : (L == 16) ? 2 : (L == 8) ? 3 : (L == 4) ? 4 : 5;
#pragma unroll
    for (int k = 0; k < STEPS; ++k) {
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            s1[t] += __shfl_xor(s1[t], L << k);
            s2[t] += __shfl_xor(s2[t], L << k);
        }
    }
    const int lane = wlane % L, grp = wlane / L;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int q = lane + L * t;
        if (t % GW == grp && q < nb) {
            accA[n0 + q] = h.a[t / GW] + s1[t];
            accA2[n0 + q] = h.a2[t / GW] + s2[t];
        }
    }
}

// The sums of A and A^2 from a chain's whole state after a sweep (read back from memory), in
// chunks of 4 L components: as acc_block, for every component of the grid.
template <int L>
__device__ __forceinline__ void acc_state(double *accA, double *accA2, const float *Ag, int64_t N, int wlane,
                                          bool active) {
    constexpr int GW = 64 / L;
    constexpr int STEPS = (L == 64) ? 0 : (L == 32) ? 1 : (L == 16) ? 2 : (L == 8) ? 3 : (L == 4) ? 4 : 5;
    const int lane = wlane % L, grp = wlane / L;
    for (int64_t q0 = 0; q0 < N; q0 += 4 * L) {
        double s1[4], s2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t q = q0 + lane + L * t;
            const double x = (active && q < N) ? (double)Ag[q] : 0.0;
            s1[t] = x;
            s2[t] = x * x;
        }
#pragma unroll
        for (int k = 0; k < STEPS; ++k) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                s1[t] += __shfl_xor(s1[t], L << k);
                s2[t] += __shfl_xor(s2[t], L << k);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t q = q0 + lane + L * t;
            if (t % GW == grp && q < N) {
                accA[q] += s1[t];
                accA2[q] += s2[t];
            }
        }
    }
}

// The accumulator slot of a wavefront for sweep s, or -1 when s is not measured: one slot per
// (tile, wavefront), or per (tile, wavefront, batch of sweeps) for batch means.
__device__ __forceinline__ int64_t acc_slot(const SampleArgs &a, const ProbDesc &pd, const TileDesc &td,
                                            int wave, int64_t s) {
    if (!a.accumulate || s < a.burnin || s >= a.burnin + a.sweeps) return -1;
    const int64_t bt = pd.batches > 1 ? (s - a.burnin) * pd.batches / a.sweeps : 0;
    return td.slot + (int64_t)wave * pd.batches + bt;
}

// Copy a block's factor chunk (the image of the staging area) to LDS with all threads,
// eight words in flight per thread.
__device__ __forceinline__ void stage_sync(float4 *dst, const float4 *src, int n, int tid, int nthr) {
    int i = tid;
    for (; i + 7 * nthr < n; i += 8 * nthr) {
        float4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = src[i + k * nthr];
#pragma unroll
        for (int k = 0; k < 8; ++k) dst[i + k * nthr] = v[k];
    }
    for (; i < n; i += nthr) dst[i] = src[i];
}

// The prefetch registers: PF words per thread, addressed with constant indices only (a fold
// over an index sequence instead of a loop) and of the compiler's native vector type, so that
// they stay in registers.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The plan's descriptor tables are written before any sampler launch and never during one:
// read through the constant address space, their uniform loads become scalar loads, which
// keep out of the vector-memory wait counts.
template <typename T>
__device__ __forceinline__ T cload(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
    typedef const __attribute__((address_space(4))) uint32_t cword;
    cword *src = (cword *)p;
    T v;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return v;
}

// The tile queue: the tile list (problem by problem, chain groups in order) is cut into
// kQueues equal ranges, each with its own counter.  Workgroup b starts on range b mod kQueues,
// which is the XCD the dispatcher places it on, so the workgroups of one XCD walk the tiles
// of a few problems at a time and share those problems' factor chunks in that XCD's L2; a
// workgroup whose range is used up takes tiles from the next ranges.  Called by thread 0 of
// the workgroup; *visited (thread 0's, 0 at the start of the launch) counts the ranges used up.
constexpr int kQueues = 8;

__device__ __forceinline__ int grab_tile(const SampleArgs &a, int *visited) {
    const int ntiles = (int)a.ntiles;
    while (*visited < kQueues) {
        const int x = ((int)blockIdx.x + *visited) % kQueues;
        const int lo = (int)((int64_t)x * ntiles / kQueues);
        const int hi = (int)((int64_t)(x + 1) * ntiles / kQueues);
        const int i = atomicAdd(a.queue + x, 1);
        if (lo + i < hi) return lo + i;
        ++*visited;
    }
    return ntiles;
}

template <int PF>
struct Prefetch {
    f32x4 w[PF > 0 ? PF : 1];

    // every load is issued (indices past the chunk re-read its last word; store_ skips
    // them), so no load sits in a branch and the compiler's wait counting stays exact
    template <int... K>
    __device__ __forceinline__ void load_(const f32x4 *src, int tid, int nthr, int n, std::integer_sequence<int, K...>) {
        ((w[K] = src[min(tid + K * nthr, n - 1)]), ...);
    }
    template <int... K>
    __device__ __forceinline__ void store_(f32x4 *dst, int tid, int nthr, int n, std::integer_sequence<int, K...>) const {
        ((tid + K * nthr < n ? (void)(dst[tid + K * nthr] = w[K]) : (void)0), ...);
    }
    __device__ __forceinline__ void load(const float4 *src, int tid, int nthr, int n) {
        load_(reinterpret_cast<const f32x4 *>(src), tid, nthr, n, std::make_integer_sequence<int, PF>{});
    }
    __device__ __forceinline__ void store(float4 *dst, int tid, int nthr, int n) const {
        store_(reinterpret_cast<f32x4 *>(dst), tid, nthr, n, std::make_integer_sequence<int, PF>{});
    }
};

// L lanes per chain, EPT components and RPT residual entries per lane; PF > 0: the next
// block's factor stream is loaded into PF registers per thread while the current block is
// sampled (when the plan's largest stream fits), so the block switch only writes LDS.
// Prefetching instances run at most 256 threads per workgroup (one wavefront per SIMD),
// which leaves them the whole register file.  H: the instance for plans with a hierarchy of
// partitions (a level drawn per sweep, blocks staged to their own size, no prefetch); the
// single-partition instances carry none of its code.
template <int L, int EPT, int RPT, int PF, bool H, bool P>
__global__ __launch_bounds__(PF > 0 ? 256 : 512) void k_sample32(SampleArgs a) {
    static_assert(!(H && PF > 0), "hierarchies run the non-prefetching instances");
    static_assert(H || !P, "the gamma prior runs in the extended instances");
    extern __shared__ __align__(16) unsigned char smem32[];
    constexpr int ROW = EPT * L;
    constexpr int MP = RPT * L;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid % L;
    const int slotc = tid / L;
    float2 *sVW = reinterpret_cast<float2 *>(smem32);
    float *sD = reinterpret_cast<float *>(smem32 + a.lds_off_d);
    float *sU = reinterpret_cast<float *>(smem32 + a.lds_off_u);
    float *sUnif = reinterpret_cast<float *>(smem32 + a.lds_off_unif);
    float *sCE = reinterpret_cast<float *>(smem32 + a.lds_off_ce);   // per chain: centres, steps
    __shared__ int s_tile;
    const int64_t s0 = cload(a.sweep);   // constant during a launch (k_bump runs between launches)
    const int64_t nsw = a.nsw;
    // the first sweep of the snapshot rows, for their reduction into the sums of A and A^2
    if (a.snapA && blockIdx.x == 0 && tid == 0) *a.snap_first = s0;
    const bool prefetch = PF > 0 && a.prefetch;
    Prefetch<PF> pf;

    int visited = 0;   // thread 0's: tile ranges used up
    for (;;) {
        if (tid == 0) s_tile = grab_tile(a, &visited);
        __syncthreads();
        const int tile = __builtin_amdgcn_readfirstlane(s_tile);   // uniform: descriptors load to SGPRs
        __syncthreads();
        if (tile >= a.ntiles) break;
        const TileDesc td = cload(a.tiles + tile);
        const ProbDesc pd = cload(a.probs + td.problem);
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
        float *urow = sUnif + slotc * ROW;
        // gamma prior: the acceptance uniforms in a second row per chain, after the first rows
        const bool PRI = P && pd.has_prior;
        float *urowA = sUnif + (nthr / L + slotc) * ROW;
        PriorRegs<EPT> pr;
        pr.rej = 0;
        const int nw = (int)a.chunk_words;
        float4 *stage = reinterpret_cast<float4 *>(smem32);
        // the blocks of a sweep: all of the partition, or of the sweep's level of a hierarchy
        // (Fig. 2), drawn for all chains of the problem at once
        const int NL = H ? (int)pd.levels : 1;
        auto level_of = [&](int64_t s, int &lf, int &lc) {
            lf = 0;
            lc = (int)pd.B;
            if (NL > 1) {
                const uint32_t l = sweep_level(a.seed, pd.index, (uint32_t)s, (uint32_t)NL);
                const int2 e = cload(reinterpret_cast<const int2 *>(a.lvl) + pd.off_lvl + l);
                lf = e.x;
                lc = e.y;
            }
        };
        int lf, lc;
        level_of(s0, lf, lc);
        if (prefetch) pf.load(a.F32 + cload(a.blocks + pd.off_blk + lf).off_chunk, tid, nthr, nw);
        // components of the next block to sample, loaded one block ahead (the blocks of a
        // partition are disjoint, so sampling a block leaves the next one's components
        // unchanged; where a hierarchy's next level overlaps, they are loaded again below)
        float An[EPT];
        {
            const BlockDesc b0 = cload(a.blocks + pd.off_blk + lf);
#pragma unroll
            for (int t = 0; t < EPT; ++t) An[t] = Ag[b0.n0 + min(lane + L * t, (int)b0.nb - 1)];
            // wait for them here (once per tile): the block loop then starts with no load of
            // this path outstanding, so the prefetch below is not waited for early
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        }
        // The components of the block sampled last (and its snapshot row) are stored while the
        // next block is sampled: a store issued at the end of a block would still be in flight
        // when the next block waits for its prefetched loads, and the wait would include it.
        const int64_t NR = (N + 3) / 4 * 4;
        float Ap[EPT];
        int64_t p_n0 = 0, p_row = -1;
        int p_nb = 0;
        auto store_prev = [&]() {
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                const int q = lane + L * t;
                if (active && q < p_nb) __builtin_nontemporal_store(Ap[t], Ag + p_n0 + q);
            }
            if (p_row >= 0) {
                // the chain state and the snapshot rows stream past the caches (the state is
                // read a sweep later, the rows after the launch), which keep the block
                // factors the staging reads
                float *sa = a.snapA + pd.off_sa + (p_row * pd.C + chain) * NR + p_n0;
#pragma unroll
                for (int t = 0; t < EPT; ++t) {
                    const int q = lane + L * t;
                    if (active && q < p_nb) __builtin_nontemporal_store(Ap[t], sa + q);
                }
            }
        };

        for (int64_t s = s0; s < s0 + nsw; ++s) {
            int nf, nc;   // the next sweep's level
            level_of(s + 1, nf, nc);
            int64_t g_end = 0, g_chunk0 = 0;   // the staged group of blocks (extended instances)
            int g_uoff = 0;                    // the next block's segment of the uniform rows
            for (int64_t b = 0; b < lc; ++b) {
                const BlockDesc bd = cload(a.blocks + pd.off_blk + lf + b);
                const int nb = (int)bd.nb, kb = (int)bd.kb;
                // modes of the block: one per grid point, or one fewer under a linear
                // constraint (extended instances only)
                const int nm = H ? (int)bd.nm : nb;
                float Ar[EPT];
#pragma unroll
                for (int t = 0; t < EPT; ++t) Ar[t] = (lane + L * t < nb && active) ? An[t] : 0.0f;
                if (PRI) {
#pragma unroll
                    for (int t = 0; t < EPT; ++t) {
                        const int q = lane + L * t;
                        pr.W[t] = q < nb ? a.wm1f[pd.off_n + bd.n0 + q] : 0.0f;
                        pr.Lg[t] = __log2f(Ar[t]);
                    }
                }
                // the block's rows, singular values and U rows in LDS and its uniforms: at the
                // plan's fixed offsets, or, for the extended instances, in the image of its group
                // (consecutive blocks of the level staged by one copy, each packed to its size:
                // nm + 2 rows, round4(kb) values, kb U rows) and a segment of the uniform rows
                const float *sDb = sD, *sUb = sU;
                const float2 *sVWb = sVW;
                float *urowb = urow, *urowAb = urowA;
                if constexpr (H) {
                    if (b >= g_end) {
                        const int gn = bd.grp_n > 0 ? bd.grp_n : 1;
                        const int gw = bd.grp_n > 0 ? bd.grp_words
                                                    : (nm + 2) * ROW / 2 + (kb + 3) / 4 + (a.u_lds ? kb * MP / 4 : 0);
                        __syncthreads();   // the previous group's readers of the LDS rows are done
                        stage_sync(stage, a.F32 + bd.off_chunk, gw, tid, nthr);
                        // the group's uniforms, one Philox call per four modes of each block; the
                        // calls of the group are dealt to the chain's lanes in turn
                        int pcall = 0, uo = 0;
                        for (int j = 0; j < gn; ++j) {
                            const int nmj = j == 0 ? nm : (int)cload(a.blocks + pd.off_blk + lf + b + j).nm;
                            const int cj = (nmj + 3) / 4;
                            for (int g = ((lane - pcall) % L + L) % L; g < cj; g += L) {
                                const U4 w = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s,
                                                          (uint32_t)(b + j), (uint32_t)g);
                                float *d = urow + uo + 4 * g;
                                d[0] = word_u32(w.x);
                                d[1] = word_u32(w.y);
                                d[2] = word_u32(w.z);
                                d[3] = word_u32(w.w);
                                if (PRI) {
                                    const U4 x = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s,
                                                              (uint32_t)(b + j), (uint32_t)g, 4u);
                                    float *e = urowA + uo + 4 * g;
                                    e[0] = word_u32(x.x);
                                    e[1] = word_u32(x.y);
                                    e[2] = word_u32(x.z);
                                    e[3] = word_u32(x.w);
                                }
                            }
                            pcall += cj;
                            uo += 4 * cj;
                        }
                        __syncthreads();
                        g_end = b + gn;
                        g_chunk0 = bd.off_chunk;
                        g_uoff = 0;
                    }
                    const int64_t base = bd.off_chunk - g_chunk0;   // 16-byte words into the group image
                    const int n1 = (nm + 2) * ROW / 2, n2 = (kb + 3) / 4;
                    sVWb = reinterpret_cast<const float2 *>(stage + base);
                    sDb = reinterpret_cast<const float *>(stage + base + n1);
                    sUb = sDb + 4 * n2;
                    urowb = urow + g_uoff;
                    urowAb = urowA + g_uoff;
                    g_uoff += 4 * ((nm + 3) / 4);
                } else {
                    __syncthreads();   // the previous block's readers of the LDS rows are done
                    if (prefetch)
                        pf.store(stage, tid, nthr, nw);
                    else
                        stage_sync(stage, a.F32 + bd.off_chunk, nw, tid, nthr);
                    // this block's uniforms: one Philox call per four modes
                    for (int g = lane; 4 * g < nm; g += L) {
                        const U4 w = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s,
                                                  (uint32_t)b, (uint32_t)g);
                        float *d = urow + 4 * g;
                        d[0] = word_u32(w.x);
                        d[1] = word_u32(w.y);
                        d[2] = word_u32(w.z);
                        d[3] = word_u32(w.w);
                    }
                    __syncthreads();
                }
                store_prev();
                const float *Ug = a.U32 + bd.off_U32;
                float2 vw[EPT];
                load_row<EPT>(vw, sVWb, lane, L);
                // data modes (U rows from LDS, or from global memory when they do not fit;
                // two copies of the loop, so the LDS one waits on no global loads)
                float *sc = sCE + slotc * 2 * a.kce;
                if (PRI) {
                    if (a.u_lds)
                        data_moves<L, EPT, RPT, true>(kb, sVWb, sDb, sUb, urowb, sc, a.kce, lane, vw, Ar, rr, &pr, urowAb);
                    else
                        data_moves<L, EPT, RPT, true>(kb, sVWb, sDb, Ug, urowb, sc, a.kce, lane, vw, Ar, rr, &pr, urowAb);
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
                } else if (a.u_lds)
                    data_moves<L, EPT, RPT>(kb, sVWb, sDb, sUb, urowb, sc, a.kce, lane, vw, Ar, rr);
                else {
                    data_moves<L, EPT, RPT>(kb, sVWb, sDb, Ug, urowb, sc, a.kce, lane, vw, Ar, rr);
                    // the U row loaded ahead past the last data mode is never read: wait for
                    // it here, or the compiler waits for every load in flight (the prefetch
                    // below included) where its register is reused
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
                }
                BlockDesc bn;
                {
                    // the next block (of this sweep, or the first of the next): its components,
                    // which were stored when this sweep sampled it, and its factor chunk, loaded
                    // during the zero modes.  The component loads are unconditional and clamped
                    // into the block (the padding lanes are zeroed when the block starts; with
                    // one block the values are replaced below), so that no branch leaves the
                    // compiler's wait counting inexact and nothing waits for them early.
                    bn = cload(a.blocks + pd.off_blk + (b + 1 < lc ? lf + b + 1 : nf));
#pragma unroll
                    for (int t = 0; t < EPT; ++t)
                        An[t] = __builtin_nontemporal_load(Ag + bn.n0 + min(lane + L * t, (int)bn.nb - 1));
                    if (prefetch && (b + 1 < lc || s + 1 < s0 + nsw)) pf.load(a.F32 + bn.off_chunk, tid, nthr, nw);
                }
                // this visit's slot entries of the sums, read during the zero modes
                AccAhead<L, EPT> acch;
                int64_t acc_sl = -1;
                if constexpr (!H) {
                    acc_sl = acc_slot(a, pd, td, tid / 64, s);
                    const int64_t o = pd.off_slot + (acc_sl >= 0 ? acc_sl : 0) * N;
                    acc_read_ahead<L, EPT>(acch, a.accA + o, a.accA2 + o, bd.n0, nb, tid % 64);
                }
                // zero modes, three per iteration, each row loaded two moves ahead (the
                // rows past the block's last are spare LDS rows, loaded and never used)
                if (PRI) {
                    zero_moves<L, EPT, true>(kb, nm, sVWb, urowb, urowAb, lane, vw, Ar, &pr);
                } else {
                    int i = kb;
                    float2 vb[EPT], vc[EPT];
                    load_row<EPT>(vb, sVWb + (i + 1) * ROW, lane, L);
                    for (; i + 3 <= nm; i += 3) {
                        load_row<EPT>(vc, sVWb + (i + 2) * ROW, lane, L);
                        const float u0 = urowb[i], u1 = urowb[i + 1], u2 = urowb[i + 2];
                        zero_move<L, EPT>(vw, Ar, u0);
                        load_row<EPT>(vw, sVWb + (i + 3) * ROW, lane, L);
                        zero_move<L, EPT>(vb, Ar, u1);
                        load_row<EPT>(vb, sVWb + (i + 4) * ROW, lane, L);
                        zero_move<L, EPT>(vc, Ar, u2);
                    }
                    if (i < nm) zero_move<L, EPT>(vw, Ar, urowb[i]);
                    if (i + 1 < nm) zero_move<L, EPT>(vb, Ar, urowb[i + 1]);
                }
                if constexpr (H) {
                    // a hierarchy's next block may overlap this block (whose components are
                    // stored only while the next one is sampled) or the previous one: store
                    // this block now and load the next one's components once the stores are
                    // done
                    const bool ov = (bn.n0 < bd.n0 + nb && bd.n0 < bn.n0 + bn.nb) ||
                                    (p_nb > 0 && bn.n0 < p_n0 + p_nb && p_n0 < bn.n0 + bn.nb);
                    if (ov) {
#pragma unroll
                        for (int t = 0; t < EPT; ++t) {
                            const int q = lane + L * t;
                            if (active && q < nb) Ag[bd.n0 + q] = Ar[t];
                        }
                        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the stores are done
#pragma unroll
                        for (int t = 0; t < EPT; ++t) An[t] = Ag[bn.n0 + min(lane + L * t, (int)bn.nb - 1)];
                    }
                }
                if constexpr (!H) {
                    if (acc_sl >= 0)
                        acc_block<L, EPT>(a.accA + pd.off_slot + acc_sl * N, a.accA2 + pd.off_slot + acc_sl * N,
                                                bd.n0, nb, tid % 64, active, Ar, acch);
                }
#pragma unroll
                for (int t = 0; t < EPT; ++t) Ap[t] = Ar[t];
                if (pd.B == 1) {   // the next block is this one
#pragma unroll
                    for (int t = 0; t < EPT; ++t) An[t] = Ar[t];
                }
                p_n0 = bd.n0;
                p_nb = nb;
                p_row = (a.snapA && s >= a.burnin) ? s - s0 : -1;
            }
            if constexpr (H) {
                // the extended instances add the sweep's state to the sums once per sweep (a
                // level of many small blocks would otherwise wait for one read-modify-write of
                // the sums per block): the last block is stored, the stores are waited for,
                // and the state is read back
                const int64_t sl = acc_slot(a, pd, td, tid / 64, s);
                if (sl >= 0) {
                    store_prev();
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the state is in memory
                    acc_state<L>(a.accA + pd.off_slot + sl * N, a.accA2 + pd.off_slot + sl * N, Ag, N, tid % 64,
                                 active);
                }
            }
            lf = nf;
            lc = nc;
        }
        store_prev();
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int m = lane + L * t;
            if (active && m < M) rg[m] = rr[t];
        }
        if (PRI && active && pr.rej) atomicAdd(&a.counters[2], (unsigned long long)pr.rej);
    }
}

// three compiled forms per shape: the plain one, the extended one (hierarchies, constraints)
// and the extended one with the gamma prior's test, so that each carries only its own code
template <int L, int EPT, int RPT, int PF>
hipError_t launch_sample32_t(const SampleArgs &a, int threads, int grid, size_t lds, hipStream_t s) {
    if (a.hier) {
        if constexpr (PF > 0) {
            return hipErrorInvalidValue;   // the extended forms are non-prefetching
        } else {
            if (a.prior)
                hipLaunchKernelGGL((k_sample32<L, EPT, RPT, 0, true, true>), dim3(grid), dim3(threads), lds, s, a);
            else
                hipLaunchKernelGGL((k_sample32<L, EPT, RPT, 0, true, false>), dim3(grid), dim3(threads), lds, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_sample32<L, EPT, RPT, PF, false, false>), dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <int L, int EPT, int RPT, int PF>
hipError_t allow_lds_sample32_t(int bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)k_sample32<L, EPT, RPT, PF, false, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if constexpr (PF == 0) {
        hipError_t e1 = hipFuncSetAttribute((const void *)k_sample32<L, EPT, RPT, 0, true, false>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess) e = e1;
        e1 = hipFuncSetAttribute((const void *)k_sample32<L, EPT, RPT, 0, true, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess) e = e1;
    }
    return e;
}

}  // namespace asmk
