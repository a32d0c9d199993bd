// Two-role float32 sampler: the data modes of block b + 1 run beside the zero modes of
// block b (Sec. IV.B-C).
//
// A zero-mode move changes only the components of its own block (V_i lies in the null space
// of the block's kernel, so r is untouched), and a data-mode move of block b + 1 reads only r
// and the components of block b + 1.  The zero modes of block b and the data modes of block
// b + 1 therefore act on disjoint state, and running them at the same time gives every move
// exactly the inputs of the one-role order (data modes, then zero modes, block after block):
// the results are bit-identical to k_sample32 with the same instance.
//
// A workgroup of 16 chains runs 512 threads in two roles of four wavefronts each, one of each
// role per SIMD, so that each SIMD interleaves two independent instruction streams:
//   data role (threads 0..255):   block steps j = 0, 1, ...: loads A of step j, runs its data
//                                 modes, hands A to the zero role through LDS (written between
//                                 the next stage's two barriers, so one buffer suffices);
//                                 carries r for the whole launch;
//   zero role (threads 256..511): step j - 1: takes A from the hand-off buffer, runs the zero
//                                 modes, adds the block's final components to the sums of A,
//                                 stores A (and its snapshot row).
// Stage t runs data step t and zero step t - 1; the two barriers of a stage separate the
// staging writes from the moves.  A block's components are stored by the zero role at stage
// j + 1 and loaded again by the data role at stage j + B, so problems need B >= 2.
// The data role also runs the first z zero modes of its block (z = p_zs, chosen to balance
// the two roles), the zero role the rest.  Each role stages its own part of the block's
// packed chunk, prefetched into registers one stage ahead: the data part (rows 0..max k + z
// + 1 of (V, w), the singular values and, with ULDS, the U rows; without, the data role reads
// its U rows from global memory) and the zero part (rows k_b + z..n_b + 1).
#pragma once

#include "sample32.h"

namespace asmk {

// LDS areas of the two-role sampler
struct AreasP {
    float2 *vwd;   // data rows 0..max k + 1
    float *d;      // singular values, then the U rows (one staged range)
    float *u;
    float2 *vwz;   // zero rows k_b..n_b + 1 of the block of the zero role
    float *und;    // data-role uniforms, p_kd per chain
    float *unz;    // zero-role uniforms, ROW per chain (indexed by mode)
    float *h;      // hand-off of A: cpw rows of ROW
    float *ce;     // data-role centres and steps: 2 kce per chain
};

// Zero modes i0..i1-1, three per iteration, each row loaded two moves ahead; row i is at
// rows + (i - i0) ROW, and the two rows past i1 - 1 are staged, loaded and never used.
template <int L, int EPT>
__device__ __forceinline__ void zero_moves_p(const float2 *rows, int i0, int i1, const float *urow, int lane,
                                             float (&Ar)[EPT]) {
    constexpr int ROW = EPT * L;
    float2 vw[EPT], vb[EPT], vc[EPT];
    load_row<EPT>(vw, rows, lane, L);
    load_row<EPT>(vb, rows + ROW, lane, L);
    int i = i0;
    for (; i + 3 <= i1; i += 3) {
        const float2 *rw = rows + (i - i0) * ROW;
        load_row<EPT>(vc, rw + 2 * ROW, lane, L);
        const float u0 = urow[i], u1 = urow[i + 1], u2 = urow[i + 2];
        zero_move<L, EPT>(vw, Ar, u0);
        load_row<EPT>(vw, rw + 3 * ROW, lane, L);
        zero_move<L, EPT>(vb, Ar, u1);
        load_row<EPT>(vb, rw + 4 * ROW, lane, L);
        zero_move<L, EPT>(vc, Ar, u2);
    }
    if (i < i1) zero_move<L, EPT>(vw, Ar, urow[i]);
    if (i + 1 < i1) zero_move<L, EPT>(vb, Ar, urow[i + 1]);
}

// Barrier with LDS ordering only: the stage's first barrier separates LDS readers from the
// staging writes and needs no wait for global stores still in flight (the second barrier of
// each stage is a full one, which orders the component stores before later loads).
__device__ __forceinline__ void barrier_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The tile queue, walked by both roles with the same barriers: 0 and above is a tile,
// -1 ends the launch.  *visited is the data role's thread 0's count of used-up tile ranges.
__device__ __forceinline__ int next_tile_p(const SampleArgs &a, int *s_tile, int tid, int *visited) {
    if (tid == 0) *s_tile = grab_tile(a, visited);
    __syncthreads();
    const int tile = __builtin_amdgcn_readfirstlane(*s_tile);
    __syncthreads();
    return tile < a.ntiles ? tile : -1;
}

// Data role: data modes of block step t at stage t; r for the whole launch.
template <int L, int EPT, int RPT, int PFR, int PFU, bool ULDS>
__device__ __forceinline__ void data_role_p(const SampleArgs &a, const AreasP &ar, int *s_tile, int tid) {
    constexpr int ROW = EPT * L;
    const int lane = tid % L;
    const int slotc = tid / L;
    const int64_t s0 = cload(a.sweep);   // constant during a launch (k_bump runs between launches)
    const int64_t nsw = a.nsw;
    Prefetch<PFR> pfr;
    Prefetch<PFU> pfu;
    int visited = 0;
    for (;;) {
        const int tile = next_tile_p(a, s_tile, tid, &visited);
        if (tile < 0) break;
        const TileDesc td = cload(a.tiles + tile);
        const ProbDesc pd = cload(a.probs + td.problem);
        const int M = (int)pd.M;
        const int64_t N = pd.N;
        const int B = (int)pd.B;
        const bool active = slotc < td.nchains;
        const int64_t chain = td.chain0 + (active ? slotc : 0);
        float *Ag = a.A32 + pd.off_A + chain * N;
        float *rg = a.r32 + pd.off_r + chain * (int64_t)M;
        const int64_t total = nsw * B;
        float rr[RPT];
#pragma unroll
        for (int t2 = 0; t2 < RPT; ++t2) {
            const int m = lane + L * t2;
            rr[t2] = (m < M && active) ? rg[m] : 0.0f;
        }
        float *urow = ar.und + slotc * a.p_kd;
        // the data parts and the components of step 0; components are loaded one stage ahead
        // when B >= 3 (the zero role stored them at least two stages before), else at the
        // start of their stage (stored at the end of the stage before)
        float An[EPT];
        {
            const BlockDesc b0 = cload(a.blocks + pd.off_blk);
#pragma unroll
            for (int t2 = 0; t2 < EPT; ++t2) An[t2] = Ag[b0.n0 + min(lane + L * t2, (int)b0.nb - 1)];
            pfr.load(a.F32 + b0.off_chunk, tid, 256, a.p_wd);
            pfu.load(a.F32 + b0.off_chunk + a.p_du_word, tid, 256, a.p_wu);
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), once per tile
        }
        float hA[EPT];   // the components of the previous step, handed over at this stage
        float *h = ar.h + slotc * ROW;
        for (int64_t t = 0; t <= total; ++t) {
            const bool step = t < total;
            const int64_t s = s0 + t / B;
            const int b = (int)(t % B);
            const BlockDesc bd = cload(a.blocks + pd.off_blk + b);
            const int nb = (int)bd.nb, kb = (int)bd.kb;
            const int ke = min(kb + a.p_zs, nb);   // this role runs modes 0..ke-1
            barrier_lds();   // the previous stage's readers of the staging areas are done
            if (t > 0) {
                // the hand-off of step t - 1: the zero role reads it after this stage's second
                // barrier and is done with it before the next stage's first one
#pragma unroll
                for (int t2 = 0; t2 < EPT; ++t2) h[lane + L * t2] = hA[t2];
            }
            if (step) {
                pfr.store(reinterpret_cast<float4 *>(ar.vwd), tid, 256, a.p_wd);
                pfu.store(reinterpret_cast<float4 *>(ar.d), tid, 256, a.p_wu);
                for (int g = lane; 4 * g < ke; g += L) {
                    const U4 w = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s, (uint32_t)b,
                                              (uint32_t)g);
                    float *d = urow + 4 * g;
                    d[0] = word_u32(w.x);
                    d[1] = word_u32(w.y);
                    d[2] = word_u32(w.z);
                    d[3] = word_u32(w.w);
                }
            }
            __syncthreads();
            if (!step) continue;
            if (B < 3 && t > 0) {
#pragma unroll
                for (int t2 = 0; t2 < EPT; ++t2)
                    An[t2] = __builtin_nontemporal_load(Ag + bd.n0 + min(lane + L * t2, nb - 1));
            }
            float Ar[EPT];
#pragma unroll
            for (int t2 = 0; t2 < EPT; ++t2) Ar[t2] = (lane + L * t2 < nb && active) ? An[t2] : 0.0f;
            if (t + 1 < total) {
                // the data parts (and with B >= 3 the components) of the next step
                const BlockDesc bn = cload(a.blocks + pd.off_blk + (b + 1 < B ? b + 1 : 0));
                if (B >= 3) {
#pragma unroll
                    for (int t2 = 0; t2 < EPT; ++t2)
                        An[t2] = __builtin_nontemporal_load(Ag + bn.n0 + min(lane + L * t2, (int)bn.nb - 1));
                }
                pfr.load(a.F32 + bn.off_chunk, tid, 256, a.p_wd);
                pfu.load(a.F32 + bn.off_chunk + a.p_du_word, tid, 256, a.p_wu);
            }
            float2 vw[EPT];
            load_row<EPT>(vw, ar.vwd, lane, L);
            float *sc = ar.ce + slotc * 2 * a.kce;
            if constexpr (ULDS) {
                data_moves<L, EPT, RPT>(kb, ar.vwd, ar.d, ar.u, urow, sc, a.kce, lane, vw, Ar, rr);
            } else {
                data_moves<L, EPT, RPT>(kb, ar.vwd, ar.d, a.U32 + bd.off_U32, urow, sc, a.kce, lane, vw, Ar, rr);
                // the U row loaded ahead past the last data mode is never read: wait for it here,
                // or the compiler waits for every load in flight where its register is reused
                __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            }
            if (ke > kb) zero_moves_p<L, EPT>(ar.vwd + kb * ROW, kb, ke, urow, lane, Ar);
#pragma unroll
            for (int t2 = 0; t2 < EPT; ++t2) hA[t2] = Ar[t2];
        }
#pragma unroll
        for (int t2 = 0; t2 < RPT; ++t2) {
            const int m = lane + L * t2;
            if (active && m < M) rg[m] = rr[t2];
        }
    }
}

// The zero role's stages of one tile.  With DELAY (four blocks or more) the components of a
// finished block are stored at the next stage, after its second barrier: a store issued at the
// end of a stage would still be in flight at the next stage's waits for the prefetched rows,
// which count it.  The data role reads a block again B stages after the zero role took it
// (B - 1 with its one-stage-ahead load), so the delayed store still precedes that load by a
// barrier when B >= 4; with two or three blocks the stores stay at the end of the stage.
template <int L, int EPT, int PFZ, bool DELAY>
__device__ __forceinline__ void zero_stages_p(const SampleArgs &a, const AreasP &ar, const ProbDesc &pd,
                                              const TileDesc &td, int64_t chain, bool active, int tid,
                                              int64_t s0) {
    constexpr int ROW = EPT * L;
    constexpr int RW = ROW / 2;   // 16-byte words per (V, w) row
    constexpr int CPW = 256 / L;
    const int lane = tid % L;
    const int slotc = tid / L;
    const int64_t N = pd.N;
    const int64_t NR = (N + 3) / 4 * 4;
    const int B = (int)pd.B;
    float *Ag = a.A32 + pd.off_A + chain * N;
    const int64_t total = a.nsw * B;
    float *urow = ar.unz + slotc * ROW;
    Prefetch<PFZ> pfz;
    float Ap[EPT];                      // a finished block's components, stored at the next stage
    int64_t p_n0 = 0, p_row = -1;
    int p_nb = 0;
    auto store_prev = [&]() {
#pragma unroll
        for (int t2 = 0; t2 < EPT; ++t2) {
            const int q = lane + L * t2;
            if (active && q < p_nb) __builtin_nontemporal_store(Ap[t2], Ag + p_n0 + q);
        }
        if (p_row >= 0) {
            float *sa = a.snapA + pd.off_sa + (p_row * pd.C + chain) * NR + p_n0;
#pragma unroll
            for (int t2 = 0; t2 < EPT; ++t2) {
                const int q = lane + L * t2;
                if (active && q < p_nb) __builtin_nontemporal_store(Ap[t2], sa + q);
            }
        }
        p_nb = 0;
        p_row = -1;
    };
    for (int64_t t = 0; t <= total; ++t) {
        const bool step = t >= 1;
        const int64_t j = step ? t - 1 : 0;
        const int64_t s = s0 + j / B;
        const int b = (int)(j % B);
        const BlockDesc bd = cload(a.blocks + pd.off_blk + b);
        const int nb = (int)bd.nb;
        const int kz = min((int)bd.kb + a.p_zs, nb);   // this role runs modes kz..nb-1
        barrier_lds();
        if (step) {
            pfz.store(reinterpret_cast<float4 *>(ar.vwz), tid, 256, (nb + 2 - kz) * RW);
            for (int g = kz / 4 + lane; 4 * g < nb; g += L) {
                const U4 w = move_words32(a.seed, pd.index, (uint32_t)chain, (uint32_t)s, (uint32_t)b,
                                          (uint32_t)g);
                float *d = urow + 4 * g;
                d[0] = word_u32(w.x);
                d[1] = word_u32(w.y);
                d[2] = word_u32(w.z);
                d[3] = word_u32(w.w);
            }
        }
        __syncthreads();
        if (t < total) {
            // the zero part of step t, sampled at the next stage
            const BlockDesc bn = cload(a.blocks + pd.off_blk + (int)(t % B));
            const int kn = min((int)bn.kb + a.p_zs, (int)bn.nb);
            pfz.load(a.F32 + bn.off_chunk + kn * RW, tid, 256, ((int)bn.nb + 2 - kn) * RW);
        }
        // after the loads: their address arithmetic may wait for earlier memory operations
        if (DELAY) store_prev();
        if (!step) continue;
        float Ar[EPT];
        const float *h = ar.h + slotc * ROW;
#pragma unroll
        for (int t2 = 0; t2 < EPT; ++t2) Ar[t2] = h[lane + L * t2];
        // this visit's slot entries of the sums, read during the zero modes
        AccAhead<L, EPT> acch;
        const int64_t sl = acc_slot(a, pd, td, tid / 64, s);
        {
            const int64_t o = pd.off_slot + (sl >= 0 ? sl : 0) * N;
            acc_read_ahead<L, EPT>(acch, a.accA + o, a.accA2 + o, bd.n0, nb, tid % 64);
        }
        zero_moves_p<L, EPT>(ar.vwz, kz, nb, urow, lane, Ar);
        if (sl >= 0)
            acc_block<L, EPT>(a.accA + pd.off_slot + sl * N, a.accA2 + pd.off_slot + sl * N, bd.n0, nb,
                                    tid % 64, active, Ar, acch);
#pragma unroll
        for (int t2 = 0; t2 < EPT; ++t2) Ap[t2] = Ar[t2];
        p_n0 = bd.n0;
        p_nb = nb;
        p_row = (a.snapA && s >= a.burnin) ? s - s0 : -1;
        if (!DELAY) store_prev();
    }
    if (DELAY) store_prev();
}

// Zero role: zero modes of block step t - 1 at stage t.
template <int L, int EPT, int PFZ>
__device__ __forceinline__ void zero_role_p(const SampleArgs &a, const AreasP &ar, int *s_tile, int tid) {
    const int slotc = tid / L;
    const int64_t s0 = cload(a.sweep);   // constant during a launch (k_bump runs between launches)
    int visited = 0;   // unused: thread 0 is in the data role
    for (;;) {
        const int tile = next_tile_p(a, s_tile, tid + 256, &visited);
        if (tile < 0) break;
        const TileDesc td = cload(a.tiles + tile);
        const ProbDesc pd = cload(a.probs + td.problem);
        const bool active = slotc < td.nchains;
        const int64_t chain = td.chain0 + (active ? slotc : 0);
        if (pd.B >= 4)
            zero_stages_p<L, EPT, PFZ, true>(a, ar, pd, td, chain, active, tid, s0);
        else
            zero_stages_p<L, EPT, PFZ, false>(a, ar, pd, td, chain, active, tid, s0);
    }
}

template <int L, int EPT, int RPT, int PFR, int PFU, int PFZ, bool ULDS>
__global__ __launch_bounds__(512) void k_sample32p(SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem32[];
    __shared__ int s_tile;
    AreasP ar;
    ar.vwd = reinterpret_cast<float2 *>(smem32 + a.p_off_vwd);
    ar.d = reinterpret_cast<float *>(smem32 + a.p_off_d);
    ar.u = reinterpret_cast<float *>(smem32 + a.p_off_u);
    ar.vwz = reinterpret_cast<float2 *>(smem32 + a.p_off_vwz);
    ar.und = reinterpret_cast<float *>(smem32 + a.p_off_und);
    ar.unz = reinterpret_cast<float *>(smem32 + a.p_off_unz);
    ar.h = reinterpret_cast<float *>(smem32 + a.p_off_h);
    ar.ce = reinterpret_cast<float *>(smem32 + a.p_off_ce);
    if (a.snapA && blockIdx.x == 0 && threadIdx.x == 0) *a.snap_first = cload(a.sweep);
    // the role is uniform per wavefront; the two branches hold disjoint live registers
    if (threadIdx.x < 256)
        data_role_p<L, EPT, RPT, PFR, PFU, ULDS>(a, ar, &s_tile, (int)threadIdx.x);
    else
        zero_role_p<L, EPT, PFZ>(a, ar, &s_tile, (int)threadIdx.x - 256);
}

template <int L, int EPT, int RPT, int PFR, int PFU, int PFZ, bool ULDS>
hipError_t launch_sample32p_t(const SampleArgs &a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_sample32p<L, EPT, RPT, PFR, PFU, PFZ, ULDS>), dim3(grid), dim3(512), lds, s, a);
    return hipGetLastError();
}

template <int L, int EPT, int RPT, int PFR, int PFU, int PFZ, bool ULDS>
hipError_t allow_lds_sample32p_t(int bytes) {
    return hipFuncSetAttribute((const void *)k_sample32p<L, EPT, RPT, PFR, PFU, PFZ, ULDS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace asmk
