// Float32 sampler for many chains: eight lanes per chain, sixty-four chains per workgroup
// (Sec. IV.B-C, the moves of sample32.h).
//
// With fewer lanes per chain each move costs fewer instructions per chain: a wavefront holds
// eight chains, so one pass of the truncated-normal draw serves eight chains instead of four,
// and the two interval reductions take three lane exchanges instead of four.  The price is
// registers and LDS: a lane holds 16 components and 52 residual entries, and the block's
// factors (V and w rows, singular values, U rows) fill almost all of the LDS, so the per-chain
// uniform rows of sample32.h do not fit.  This sampler therefore
//   * holds the uniforms in registers: a Philox call yields the four uniforms of four
//     consecutive modes; the lanes of a chain make one call each and a move takes its uniform
//     from the lane that holds it by a lane shuffle (no LDS storage);
//   * blocks the residual per lane (lane j holds r_m for m in [52 j, 52 j + 52)), so that the
//     block's centres c = U_b^T r and its residual update read the U rows as 16-byte words;
//   * gives a lane pairs of neighbouring components, so that it reads its (V, w) entries of a
//     row as 16-byte words too;
//   * keeps one LDS slot per data mode and chain: the centre c_i, overwritten by the step
//     e_i = delta_i d_i once mode i has moved.
// The uniforms of modes 0 .. 31 come from one Philox call per lane at the block's start (they
// serve the data modes and the first zero modes), those of every later 32 modes from one call
// per lane when the zero modes reach them; a move takes its uniform from the lane holding it,
// the words rotated once per run so that a move reads a fixed register.  The (V, w) rows
// alternate between two register sets, each loaded a move ahead.
#pragma once

#include "sample32.h"

namespace asmk {

// The uniform of data mode i (i < 4 L): lane i / 4 of the chain holds it as word i mod 4.
template <int L>
__device__ __forceinline__ float data_uniform(const float (&ud)[4], int i) {
    const int k = i & 3;
    const float v = k == 0 ? ud[0] : k == 1 ? ud[1] : k == 2 ? ud[2] : ud[3];
    return __shfl(v, i >> 2, L);
}

// The components a lane holds: pairs of neighbours, q(t) = 2 lane + 2 L (t / 2) + t mod 2, so
// that a lane reads its (V, w) entries of a row as 16-byte words (two neighbouring pairs of
// the row per load; LDS serves 16-byte reads at about 1.4 times the rate of 8-byte ones)
template <int L>
__device__ __forceinline__ int comp_of(int lane, int t) {
    return 2 * lane + 2 * L * (t >> 1) + (t & 1);
}

template <int L, int EPT>
__device__ __forceinline__ void load_row_pairs(float2 (&vw)[EPT], const float2 *row, int lane) {
    const float4 *r4 = reinterpret_cast<const float4 *>(row) + lane;
#pragma unroll
    for (int j = 0; j < EPT / 2; ++j) {
        const float4 x = r4[L * j];
        vw[2 * j] = make_float2(x.x, x.y);
        vw[2 * j + 1] = make_float2(x.z, x.w);
    }
}

// A lane's components stored past the caches as pairs (8-byte stores, 64 contiguous bytes per
// chain and store; a block may start at an odd component, so the pairs are only 4-byte
// aligned, which global stores allow), the last pair split when the block ends inside it
typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

template <int L, int EPT>
__device__ __forceinline__ void store_pairs(float *row, const float (&Ap)[EPT], int lane, int nb, bool active) {
#pragma unroll
    for (int j = 0; j < EPT / 2; ++j) {
        const int q = comp_of<L>(lane, 2 * j);
        if (active && q + 1 < nb) {
            f32x2_a4 v;
            v.x = Ap[2 * j];
            v.y = Ap[2 * j + 1];
            __builtin_nontemporal_store(v, reinterpret_cast<f32x2_a4 *>(row + q));
        } else if (active && q < nb) {
            __builtin_nontemporal_store(Ap[2 * j], row + q);
        }
    }
}

// acc_read_ahead (sample32.h) for the paired components
template <int L, int EPT>
__device__ __forceinline__ void acc_read_ahead_pairs(AccAhead<L, EPT> &h, const double *accA, const double *accA2,
                                                     int64_t n0, int nb, int wlane) {
    constexpr int GW = 64 / L;
    const int lane = wlane % L, grp = wlane / L;
#pragma unroll
    for (int j = 0; j < AccAhead<L, EPT>::KA; ++j) {
        const int t = min(grp + GW * j, EPT - 1);
        const int64_t q = n0 + min(comp_of<L>(lane, t), nb - 1);
        h.a[j] = accA[q];
        h.a2[j] = accA2[q];
    }
}

// c_i = U_i . r for the block's data modes, written to sc[i] by the chain's first lane; U rows
// of MP = RPT L floats in LDS, the lane's residual entries RPT consecutive ones
template <int L, int RPT>
__device__ __forceinline__ void centres_blocked(int kb, const float *sU, const float (&rr)[RPT], int lane, float *sc) {
    constexpr int MP = RPT * L;
    static_assert(RPT % 4 == 0, "whole 16-byte words per lane");
    for (int i = 0; i < kb; ++i) {
        const float4 *row = reinterpret_cast<const float4 *>(sU + i * MP + RPT * lane);
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
#pragma unroll
        for (int j = 0; j < RPT / 4; ++j) {
            const float4 u = row[j];
            c0 = fmaf(u.x, rr[4 * j], c0);
            c1 = fmaf(u.y, rr[4 * j + 1], c1);
            c2 = fmaf(u.z, rr[4 * j + 2], c2);
            c3 = fmaf(u.w, rr[4 * j + 3], c3);
        }
        const float c = seg_sum<L>((c0 + c1) + (c2 + c3));
        if (lane == 0) sc[i] = c;
    }
}

// r -= sum_i e_i U_i over the block's data modes, the steps e_i from sc
template <int L, int RPT>
__device__ __forceinline__ void residual_blocked(int kb, const float *sU, const float *sc, int lane, float (&rr)[RPT]) {
    constexpr int MP = RPT * L;
    for (int i = 0; i < kb; ++i) {
        const float e = sc[i];
        const float4 *row = reinterpret_cast<const float4 *>(sU + i * MP + RPT * lane);
#pragma unroll
        for (int j = 0; j < RPT / 4; ++j) {
            const float4 u = row[j];
            rr[4 * j] = fmaf(-e, u.x, rr[4 * j]);
            rr[4 * j + 1] = fmaf(-e, u.y, rr[4 * j + 1]);
            rr[4 * j + 2] = fmaf(-e, u.z, rr[4 * j + 2]);
            rr[4 * j + 3] = fmaf(-e, u.w, rr[4 * j + 3]);
        }
    }
}

// Zero modes i0 .. i0 + n - 1 with their uniforms in registers: mode i0 + j is word q[j mod 4]
// of lane lb + (C + j) / 4 of the chain (q holds a lane's four words rotated by C = i0 mod 4;
// C < 0: the rotation c is given at run time).  Move j reads row set j mod 2, where row i0 + j
// was loaded a move ahead; on entry R[0] holds row i0, on return R[n mod 2] holds row i0 + n.
// lbase is the byte address of the chain's first lane for ds_bpermute.
template <int L, int EPT, int C>
__device__ __forceinline__ void zero_run(const float2 *sVW, int i0, int n, const float (&q)[4], int lb, int lbase,
                                         int lane, float2 (&R)[2][EPT], float (&Ar)[EPT], int c = C) {
    constexpr int ROW = EPT * L;
    // bodies of 4 moves (4 is a multiple of the 2 row sets and the 4 words); the body's
    // uniforms are fetched first, so that waiting for one of them leaves the rows loaded after
    // it (a move ahead) in flight; within a body the source lanes are lb + h / 4 + (C + k) / 4,
    // so one address per body serves the four shuffles (the rest is their immediate offsets)
#pragma unroll 1
    for (int h = 0; h < n; h += 4) {
        const int addr = lbase + ((lb + (h >> 2)) << 2);
        float u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            u[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(addr + 4 * (((C < 0 ? c : C) + k) >> 2),
                                                               __float_as_int(q[k])));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = h + k;
            if (j < n) {
                // row i0 + j + 1 into the set row i0 + j - 1 left (the row past the block's
                // last mode is a spare row of the staging area)
                load_row_pairs<L, EPT>(R[(k + 1) % 2], sVW + (i0 + j + 1) * ROW, lane);
                zero_move<L, EPT>(R[k % 2], Ar, u[k]);
            }
        }
    }
}

// The zero modes z0 .. nb - 1 of a block (z0 even): those below 4 L with the data modes'
// uniforms (lane j holds modes 4 j .. 4 j + 3; q1 holds them rotated by z0 mod 4), then windows
// of 4 L modes, one Philox call per lane each.  On entry R[0] holds row z0; 4 L - z0 is even,
// so every run after the first starts on row set 0.
template <int L, int EPT>
__device__ __forceinline__ void zero_modes_w(const float2 *sVW, int z0, int nb, const float (&q1)[4],
                                             const SampleArgs &a, uint32_t problem, uint32_t chain, uint32_t s,
                                             uint32_t b, int lane, float2 (&R)[2][EPT], float (&Ar)[EPT]) {
    constexpr int W = 4 * L;
    const int lbase = (int)((__lane_id() & ~(L - 1)) << 2);
    const int n1 = min(nb, W) - z0;
    if (n1 > 0) zero_run<L, EPT, -1>(sVW, z0, n1, q1, z0 >> 2, lbase, lane, R, Ar, z0 & 3);
    for (int w0 = W; w0 < nb; w0 += W) {
        const U4 x = move_words32(a.seed, problem, chain, s, b, (uint32_t)(w0 / 4 + lane));
        const float q[4] = {word_u32(x.x), word_u32(x.y), word_u32(x.z), word_u32(x.w)};
        zero_run<L, EPT, 0>(sVW, w0, min(W, nb - w0), q, 0, lbase, lane, R, Ar);
    }
}

// Copy words [w0, w1) of a block's chunk to the same words of the staging area by LDS-direct
// loads (global_load_lds_dwordx4: no registers; done when vmcnt reaches zero).  The LDS
// address of such a load is that of the wavefront's first lane, the others' words follow it.
__device__ __forceinline__ void stage_direct(float4 *dst, const float4 *src, int w0, int w1, int tid, int nthr) {
    typedef __attribute__((address_space(3))) void lds_void;
    const int wbase = tid & ~63;
    for (int i0 = w0; i0 < w1; i0 += nthr) {
        const int i = i0 + tid;
        if (i < w1) __builtin_amdgcn_global_load_lds((const void *)(src + i), (lds_void *)(dst + i0 + wbase), 16, 0, 0);
    }
}

// acc_block (sample32.h) four components at a time: the float64 sums and their butterflies
// over the wavefront's chains hold 16 registers instead of 4 EPT, which the sampler's rows,
// components and residual entries leave free
template <int L, int EPT>
__device__ __forceinline__ void acc_block_chunked(double *accA, double *accA2, int64_t n0, int nb, int wlane,
                                                  bool active, const float (&Ar)[EPT], const AccAhead<L, EPT> &h) {
    constexpr int GW = 64 / L;
    constexpr int STEPS = (L == 64) ? 0 : (L == 32) ? 1 : (L == 16) ? 2 : (L == 8) ? 3 : (L == 4) ? 4 : 5;
    const int lane = wlane % L, grp = wlane / L;
#pragma unroll
    for (int t0 = 0; t0 < EPT; t0 += 4) {
        double s1[4], s2[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double x = active ? (double)Ar[t0 + k] : 0.0;
            s1[k] = x;
            s2[k] = x * x;
        }
#pragma unroll
        for (int st = 0; st < STEPS; ++st) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s1[k] += __shfl_xor(s1[k], L << st);
                s2[k] += __shfl_xor(s2[k], L << st);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = t0 + k;
            const int q = comp_of<L>(lane, t);
            if (t % GW == grp && q < nb) {
                accA[n0 + q] = h.a[t / GW] + s1[k];
                accA2[n0 + q] = h.a2[t / GW] + s2[k];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int L, int EPT, int RPT>
__global__ __launch_bounds__(512) void k_sample32w(SampleArgs a) {
    static_assert(L == 8, "the uniform windows of 4 L modes hold one Philox call per lane of a chain");
    extern __shared__ __align__(16) unsigned char smem32[];
    constexpr int ROW = EPT * L;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid % L;
    const int slotc = tid / L;
    float2 *sVW = reinterpret_cast<float2 *>(smem32);
    const float *sD = reinterpret_cast<const float *>(smem32 + a.lds_off_d);
    const float *sU = reinterpret_cast<const float *>(smem32 + a.lds_off_u);
    float *sCE = reinterpret_cast<float *>(smem32 + a.lds_off_ce);   // per chain: centres, then steps
    __shared__ int s_tile;
    const int64_t s0 = cload(a.sweep);   // constant during a launch (k_bump runs between launches)
    const int64_t nsw = a.nsw;
    if (a.snapA && blockIdx.x == 0 && tid == 0) *a.snap_first = s0;
    const int nw = (int)a.chunk_words;
    const int wrows = (int)(a.lds_off_d / 16);   // 16-byte words of the (V, w) rows
    float4 *stage = reinterpret_cast<float4 *>(smem32);

    int visited = 0;   // thread 0's: tile ranges used up
    for (;;) {
        if (tid == 0) s_tile = grab_tile(a, &visited);
        __syncthreads();
        const int tile = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (tile >= a.ntiles) break;
        const TileDesc td = cload(a.tiles + tile);
        const ProbDesc pd = cload(a.probs + td.problem);
        const int M = (int)pd.M;
        const int64_t N = pd.N;
        const int B = (int)pd.B;
        const bool active = slotc < td.nchains;
        const int64_t chain = td.chain0 + (active ? slotc : 0);
        float *Ag = a.A32 + pd.off_A + chain * N;
        float *rg = a.r32 + pd.off_r + chain * (int64_t)M;
        float rr[RPT];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int m = RPT * lane + t;
            rr[t] = (m < M && active) ? rg[m] : 0.0f;
        }
        float *sc = sCE + slotc * a.kce;
        float An[EPT];
        {
            const BlockDesc b0 = cload(a.blocks + pd.off_blk);
#pragma unroll
            for (int t = 0; t < EPT; ++t) An[t] = Ag[b0.n0 + min(comp_of<L>(lane, t), (int)b0.nb - 1)];
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), once per tile
        }
        // the components of the block sampled last (and its snapshot row), stored during the
        // next block's zero modes, past the caches (the state is read a sweep later, the rows
        // after the launch)
        const int64_t NR = (N + 3) / 4 * 4;
        float Ap[EPT];
        int64_t p_n0 = 0, p_row = -1;
        int p_nb = 0;
        auto store_prev = [&]() {
            store_pairs<L, EPT>(Ag + p_n0, Ap, lane, p_nb, active);
            if (p_row >= 0)
                store_pairs<L, EPT>(a.snapA + pd.off_sa + (p_row * pd.C + chain) * NR + p_n0, Ap, lane, p_nb, active);
        };

        for (int64_t s = s0; s < s0 + nsw; ++s) {
            for (int b = 0; b < B; ++b) {
                const BlockDesc bd = cload(a.blocks + pd.off_blk + b);
                const int nb = (int)bd.nb, kb = (int)bd.kb;
                float Ar[EPT];
#pragma unroll
                for (int t = 0; t < EPT; ++t) Ar[t] = (comp_of<L>(lane, t) < nb && active) ? An[t] : 0.0f;
                __syncthreads();   // the previous block's readers of the LDS rows are done
                // the staging area by LDS-direct loads: the block's nb + 2 rows, its singular
                // values and U rows (waiting here for all of it, with one barrier, measured
                // faster than letting the zero modes' rows arrive during the data modes behind
                // a second barrier, at which the wavefronts wait for the slowest data modes)
                const float4 *chunk = a.F32 + bd.off_chunk;
                stage_direct(stage, chunk, 0, min((nb + 2) * (ROW / 2), wrows), tid, nthr);
                stage_direct(stage, chunk, wrows, nw, tid, nthr);
                // the data modes' uniforms (modes 0 .. 4 L - 1, one Philox call per lane)
                float ud[4];
                {
                    const U4 x = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s, (uint32_t)b,
                                              (uint32_t)lane);
                    ud[0] = word_u32(x.x);
                    ud[1] = word_u32(x.y);
                    ud[2] = word_u32(x.z);
                    ud[3] = word_u32(x.w);
                }
                __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the chunk is in LDS
                __syncthreads();
                float2 R[2][EPT];
                load_row_pairs<L, EPT>(R[0], sVW, lane);
                if (kb > 0) {
                    centres_blocked<L, RPT>(kb, sU, rr, lane, sc);
                    int i = 0;
                    for (; i + 2 <= kb; i += 2) {
                        load_row_pairs<L, EPT>(R[1], sVW + (i + 1) * ROW, lane);
                        const float u0 = data_uniform<L>(ud, i), u1 = data_uniform<L>(ud, i + 1);
                        const float d0 = sD[i], d1 = sD[i + 1], c0 = sc[i], c1 = sc[i + 1];
                        data_move<L, EPT>(R[0], c0, u0, d0, Ar, sc + i, lane);
                        load_row_pairs<L, EPT>(R[0], sVW + (i + 2) * ROW, lane);
                        data_move<L, EPT>(R[1], c1, u1, d1, Ar, sc + i + 1, lane);
                    }
                    if (i < kb) {
                        data_move<L, EPT>(R[0], sc[i], data_uniform<L>(ud, i), sD[i], Ar, sc + i, lane);
                        load_row_pairs<L, EPT>(R[0], sVW + (i + 1) * ROW, lane);
                    }
                    residual_blocked<L, RPT>(kb, sU, sc, lane, rr);
                }
                // the first zero mode z0: kb, or kb + 1 when kb is odd (mode kb then moves on its
                // own below), so that the zero modes below 4 L are an even number; the data
                // modes' words for them, rotated by z0 mod 4
                const int z0 = min(kb + (kb & 1), nb);
                float q1[4];
                {
                    const int c = z0 & 3;
                    q1[0] = c == 0 ? ud[0] : c == 1 ? ud[1] : c == 2 ? ud[2] : ud[3];
                    q1[1] = c == 0 ? ud[1] : c == 1 ? ud[2] : c == 2 ? ud[3] : ud[0];
                    q1[2] = c == 0 ? ud[2] : c == 1 ? ud[3] : c == 2 ? ud[0] : ud[1];
                    q1[3] = c == 0 ? ud[3] : c == 1 ? ud[0] : c == 2 ? ud[1] : ud[2];
                }
                // the previous block's components (and snapshot row), stored after the data
                // modes, whose waits would otherwise include them (vmcnt counts stores too), and
                // before the next block's components are loaded (with two blocks that is the
                // block stored here); the first wait after them is at the end of the zero modes
                store_prev();
                // the next block (of this sweep, or the first of the next): its components,
                // loaded during the zero modes
                {
                    // whole rows from one base address (immediate offsets, no per-entry
                    // clamping: entries past the block belong to the next block, or to the
                    // spare floats past the last chain, and are never used)
                    const BlockDesc bn = cload(a.blocks + pd.off_blk + (b + 1 < B ? b + 1 : 0));
                    const float *src = Ag + bn.n0;
#pragma unroll
                    for (int j = 0; j < EPT / 2; ++j) {
                        const f32x2_a4 v =
                            __builtin_nontemporal_load(reinterpret_cast<const f32x2_a4 *>(src + comp_of<L>(lane, 2 * j)));
                        An[2 * j] = v.x;
                        An[2 * j + 1] = v.y;
                    }
                }
                // this visit's slot entries of the sums, read during the zero modes
                AccAhead<L, EPT> acch;
                const int64_t acc_sl = acc_slot(a, pd, td, tid / 64, s);
                {
                    const int64_t o = pd.off_slot + (acc_sl >= 0 ? acc_sl : 0) * N;
                    acc_read_ahead_pairs<L, EPT>(acch, a.accA + o, a.accA2 + o, bd.n0, nb, tid % 64);
                }
                // zero modes kb .. nb - 1
                if (z0 > kb) {
                    // the odd zero mode kb, with its row loaded after it (once per block)
                    zero_move<L, EPT>(R[0], Ar, data_uniform<L>(ud, kb));
                    load_row_pairs<L, EPT>(R[0], sVW + (kb + 1) * ROW, lane);
                }
                zero_modes_w<L, EPT>(sVW, z0, nb, q1, a, pd.index, (uint32_t)chain, (uint32_t)s, (uint32_t)b, lane,
                                     R, Ar);
                if (acc_sl >= 0)
                    acc_block_chunked<L, EPT>(a.accA + pd.off_slot + acc_sl * N, a.accA2 + pd.off_slot + acc_sl * N,
                                              bd.n0, nb, tid % 64, active, Ar, acch);
#pragma unroll
                for (int t = 0; t < EPT; ++t) Ap[t] = Ar[t];
                if (B == 1) {   // the next block is this one
#pragma unroll
                    for (int t = 0; t < EPT; ++t) An[t] = Ar[t];
                }
                p_n0 = bd.n0;
                p_nb = nb;
                p_row = (a.snapA && s >= a.burnin) ? s - s0 : -1;
            }
        }
        store_prev();
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int m = RPT * lane + t;
            if (active && m < M) rg[m] = rr[t];
        }
    }
}

template <int L, int EPT, int RPT>
hipError_t launch_sample32w_t(const SampleArgs &a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_sample32w<L, EPT, RPT>), dim3(grid), dim3(512), lds, s, a);
    return hipGetLastError();
}

template <int L, int EPT, int RPT>
hipError_t allow_lds_sample32w_t(int bytes) {
    return hipFuncSetAttribute((const void *)k_sample32w<L, EPT, RPT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               bytes);
}

}  // namespace asmk
