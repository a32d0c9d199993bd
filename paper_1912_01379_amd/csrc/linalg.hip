// Float64 kernels over the chain states of all problems:
//   refresh  -- r = g~ - K~ A for every chain (the residual of Eq. (CompChi)), a dense
//               (chains x N) x (N x M) contraction on the float64 matrix cores;
//   cross    -- sum over chains of r A^T (M x N), the cross moment whose centred version
//               Cov(r~, A) gives the sensitivity of the average to the data;
//   finalize -- the average of Eq. (MCint), its standard error over independent chain
//               groups, and the posterior standard deviation;
//   vjp      -- J^T v with J = d<A>/dG = -Cov(A, r~) T.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace asmk {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double load_state(const float *A32, const double *A64, int64_t i, int fp32) {
    return fp32 ? (double)A32[i] : A64[i];
}

// MFMA f64 16x16x4 layouts (checked on the device): operand a: lane l holds row l%16, k = l/16;
// operand b: lane l holds column l%16, k = l/16; result: lane l, element j holds row l/16 + 4j,
// column l%16.
//
// Refresh: r_c = g~ - K~ A_c for every chain c, the (chains x N) x (N x M) contraction on the
// float64 matrix cores.  A workgroup of 4 wavefronts owns 64 chains and up to 128 data points
// (column group blockIdx.y); the grid points pass through LDS in chunks of kRefKC, the chains'
// components (64 x kRefKC, rows padded to kRefLDA words) and K~ (128 x kRefKC doubles, rows
// padded to kRefLDK doubles, as stored: data point by data point), the next chunk loaded into
// registers while the current one is multiplied.  Wavefront w forms chains 16 w .. 16 w + 15, one
// accumulator per 16 data points.
constexpr int kRefKC = 32, kRefLDA = 36, kRefLDK = 34, kRefCols = 128;

template <typename T>
__global__ __launch_bounds__(256) void k_refresh(const ProbDesc *probs, const double *Kt, const double *gt,
                                                 const T *Ast, T *rst) {
    __shared__ __align__(16) T sA[64 * kRefLDA];
    __shared__ __align__(16) double sK[kRefCols * kRefLDK];
    const ProbDesc pd = probs[blockIdx.z];
    const int64_t M = pd.M, N = pd.N, C = pd.C;
    const int64_t c0 = (int64_t)blockIdx.x * 64, m0 = (int64_t)blockIdx.y * kRefCols;
    if (c0 >= C || m0 >= M) return;
    const int ncol = (int)min<int64_t>(kRefCols, M - m0);
    const int ncb = (ncol + 15) / 16;
    const T *Ab = Ast + pd.off_A;
    const double *K = Kt + pd.off_K;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int i = lane % 16, kk = lane / 16;
    // staging: the components, 64 chains x kRefKC values (8 per thread), and K~, ncol rows of
    // kRefKC doubles as double2 words (8 per thread)
    T pa[8];
    double2 pk[8];
    auto load = [&](int64_t n0) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int e = tid + 256 * h, row = e / kRefKC, k = e % kRefKC;
            const int64_t c = c0 + row, n = n0 + k;
            pa[h] = (c < C && n < N) ? Ab[c * N + n] : T(0);
        }
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int e = tid + 256 * h, col = e / (kRefKC / 2), k2 = e % (kRefKC / 2);
            const int64_t m = m0 + col, n = n0 + 2 * k2;
            double2 v = make_double2(0.0, 0.0);
            if (col < ncol) {
                if (n < N) v.x = K[m * N + n];
                if (n + 1 < N) v.y = K[m * N + n + 1];
            }
            pk[h] = v;
        }
    };
    d4 acc[kRefCols / 16];
#pragma unroll
    for (int c = 0; c < kRefCols / 16; ++c) acc[c] = d4{0, 0, 0, 0};
    load(0);
    for (int64_t n0 = 0; n0 < N; n0 += kRefKC) {
        __syncthreads();   // the previous chunk is consumed
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int e = tid + 256 * h, row = e / kRefKC, k = e % kRefKC;
            sA[row * kRefLDA + k] = pa[h];
        }
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int e = tid + 256 * h, col = e / (kRefKC / 2), k2 = e % (kRefKC / 2);
            *reinterpret_cast<double2 *>(sK + col * kRefLDK + 2 * k2) = pk[h];
        }
        __syncthreads();
        if (n0 + kRefKC < N) load(n0 + kRefKC);
#pragma unroll
        for (int k4 = 0; k4 < kRefKC; k4 += 4) {
            const double av = (double)sA[(16 * wave + i) * kRefLDA + k4 + kk];
#pragma unroll
            for (int c = 0; c < kRefCols / 16; ++c)
                if (c < ncb)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sK[(16 * c + i) * kRefLDK + k4 + kk], acc[c], 0,
                                                                  0, 0);
        }
    }
    const double *g = gt + pd.off_m;
#pragma unroll
    for (int c = 0; c < kRefCols / 16; ++c) {
        if (c >= ncb) continue;
        const int64_t m = m0 + 16 * c + lane % 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t ch = c0 + 16 * wave + lane / 16 + 4 * j;
            if (ch < C && m < M) rst[pd.off_r + ch * M + m] = (T)(g[m] - acc[c][j]);
        }
    }
}

// chi2[c] = |r_c|^2 (float64 accumulation); if `drift` is given, the relative change of
// |r|^2 against prev[c] is folded into drift[c] by a running maximum.
__global__ __launch_bounds__(64) void k_rownorm(const ProbDesc *probs, const int32_t *chain_problem,
                                                const int32_t *chain_local, const float *r32,
                                                const double *r64, int fp32, double *out,
                                                const double *prev, double *drift) {
    const ProbDesc pd = probs[chain_problem[blockIdx.x]];
    const int64_t c = chain_local[blockIdx.x];
    const int64_t M = pd.M;
    double s = 0.0;
    for (int64_t m = threadIdx.x; m < M; m += 64) {
        const double x = load_state(r32, r64, pd.off_r + c * M + m, fp32);
        s += x * x;
    }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x == 0) {
        if (drift) {
            const double p = prev[pd.off_c + c];
            const double dr = fabs(p - s) / (s > 0.0 ? s : 1.0);
            drift[pd.off_c + c] = fmax(drift[pd.off_c + c], dr);
        }
        out[pd.off_c + c] = s;
    }
}

hipError_t launch_refresh_all(const ProbDesc *probs_dev, int64_t P, int64_t max_c, int64_t max_m,
                              const double *Kt, const double *gt, const float *A32, float *r32,
                              const double *A64, double *r64, int fp32, hipStream_t s) {
    const dim3 grid((unsigned)((max_c + 63) / 64), (unsigned)((max_m + kRefCols - 1) / kRefCols), (unsigned)P);
    if (fp32)
        hipLaunchKernelGGL(k_refresh<float>, grid, dim3(256), 0, s, probs_dev, Kt, gt, A32, r32);
    else
        hipLaunchKernelGGL(k_refresh<double>, grid, dim3(256), 0, s, probs_dev, Kt, gt, A64, r64);
    return hipGetLastError();
}

hipError_t launch_rownorm(const ProbDesc *probs_dev, const int32_t *chain_problem,
                          const int32_t *chain_local, int64_t total_chains, const float *r32,
                          const double *r64, int fp32, double *out, const double *prev,
                          double *drift, hipStream_t s) {
    hipLaunchKernelGGL(k_rownorm, dim3((unsigned)total_chains), dim3(64), 0, s, probs_dev,
                       chain_problem, chain_local, r32, r64, fp32, out, prev, drift);
    return hipGetLastError();
}

// Cross moment of one sweep of the float64 sampler, added to per-split float64 partial sums:
//   X_split[m][n] += sum_{c in split} r[c][m] A[c][n]  for n < N,  X_split[m][N] += sum r[c][m]
// (the last column treats A as having an extra component equal to one).  The splits are
// (group, part): the chains of chain group g in `parts` ranges, or, with batch means
// (bgroup >= 0), all chains of the sweep in `parts` ranges of batch bgroup.  One wavefront
// owns a 32 x 32 tile of one split (2 x 2 MFMA f64 16x16x4 blocks), so the partial sums are
// updated without atomics and the order of every addition is fixed.
__device__ __forceinline__ double cross_b(const float *A32, const double *A64, int fp32, int64_t base,
                                          int64_t n, int64_t N, bool ok) {
    if (!ok) return 0.0;
    if (n == N) return 1.0;
    return load_state(A32, A64, base + n, fp32);
}

__global__ __launch_bounds__(64) void k_cross(const ProbDesc *probs, int parts, int bgroup, const float *A32,
                                              const float *r32, const double *A64, const double *r64,
                                              int fp32, double *cross) {
    const ProbDesc pd = probs[blockIdx.z];
    const int64_t M = pd.M, N = pd.N, C = pd.C, N1 = N + 1;
    const int64_t ntm = (M + 31) / 32, ntn = (N1 + 31) / 32;
    const int64_t tile = blockIdx.x;
    if (tile >= ntm * ntn) return;
    const int g = bgroup >= 0 ? bgroup : (int)blockIdx.y / parts, part = (int)blockIdx.y % parts;
    const int split = g * parts + part;
    const int64_t G = pd.groups;
    const int64_t cg0 = bgroup >= 0 ? 0 : C * g / G, cg1 = bgroup >= 0 ? C : C * (g + 1) / G;
    const int64_t c_lo = cg0 + (cg1 - cg0) * part / parts, c_hi = cg0 + (cg1 - cg0) * (part + 1) / parts;
    const int64_t m0 = (tile / ntn) * 32, n0 = (tile % ntn) * 32;
    const int lane = threadIdx.x;
    const int i = lane % 16, k = lane / 16;
    const int64_t ma0 = m0 + i, ma1 = m0 + 16 + i;
    const int64_t nb0 = n0 + i, nb1 = n0 + 16 + i;
    const bool okm0 = ma0 < M, okm1 = ma1 < M, okn0 = nb0 < N1, okn1 = nb1 < N1;
    d4 a00 = {0, 0, 0, 0}, a01 = {0, 0, 0, 0}, a10 = {0, 0, 0, 0}, a11 = {0, 0, 0, 0};
    for (int64_t c0 = c_lo; c0 < c_hi; c0 += 4) {
        const int64_t c = c0 + k;
        const bool okc = c < c_hi;
        const int64_t rb = pd.off_r + c * M, ab = pd.off_A + c * N;
        const double r0 = (okc && okm0) ? load_state(r32, r64, rb + ma0, fp32) : 0.0;
        const double r1 = (okc && okm1) ? load_state(r32, r64, rb + ma1, fp32) : 0.0;
        const double b0 = cross_b(A32, A64, fp32, ab, nb0, N, okc && okn0);
        const double b1 = cross_b(A32, A64, fp32, ab, nb1, N, okc && okn1);
        a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(r0, b0, a00, 0, 0, 0);
        a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(r0, b1, a01, 0, 0, 0);
        a10 = __builtin_amdgcn_mfma_f64_16x16x4f64(r1, b0, a10, 0, 0, 0);
        a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(r1, b1, a11, 0, 0, 0);
    }
    double *X = cross + pd.off_cross + (int64_t)split * M * N1;
    const int64_t col0 = n0 + lane % 16, col1 = col0 + 16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t row0 = m0 + lane / 16 + 4 * j, row1 = row0 + 16;
        if (row0 < M && col0 < N1) X[row0 * N1 + col0] += a00[j];
        if (row0 < M && col1 < N1) X[row0 * N1 + col1] += a01[j];
        if (row1 < M && col0 < N1) X[row1 * N1 + col0] += a10[j];
        if (row1 < M && col1 < N1) X[row1 * N1 + col1] += a11[j];
    }
}

hipError_t launch_cross_all(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles, int groups, int parts,
                            int bgroup, const float *A32, const float *r32, const double *A64,
                            const double *r64, int fp32, double *cross, hipStream_t s) {
    const unsigned gy = (unsigned)(bgroup >= 0 ? parts : groups * parts);
    hipLaunchKernelGGL(k_cross, dim3((unsigned)max_tiles, gy, (unsigned)P), dim3(64), 0, s, probs_dev, parts,
                       bgroup, A32, r32, A64, r64, fp32, cross);
    return hipGetLastError();
}

// Cross moments from the per-sweep snapshots of one launch of the float32 sampler.  The
// residual rows, written by k_project from the A snapshots, hold the residual of each sampled
// state, g~ - K~ A (M entries), or, for problems with a range basis Q (rank_r > 0), its
// coordinates Q^T (g~ - K~ A) (rank_r entries); with x the row entries and the snapshot rows
// k = (sweep, chain) of a split,
//   X_split[i][n] += sum_{k in split} x_k[i] A_k[n] (n < N),  X_split[i][N] += sum x_k[i].
// Splits are (group, part): the rows of chain group g (or, with batch means, of the sweeps of
// batch g), in `parts` ranges, so the partial sums are per-group moments (the error bar of
// the VJP).  A workgroup of 4 wavefronts owns a 64 x 128 output tile and one split; each
// wavefront owns 64 x 32 of it (4 x 2 MFMA f64 16x16x4 blocks).  The rows pass through LDS in
// chunks of kSnapKC, so every snapshot value is read from memory once per workgroup tile that
// needs it; the float32 values are widened to float64 as they enter the MFMAs.  The kernel is
// sized (14 KB of LDS, about 100 VGPRs, 256 threads) to share CUs with other work.  Snapshot
// rows are padded to multiples of four floats.
constexpr int kSnapTM = 64, kSnapTN = 128, kSnapKC = 16;
// LDS row strides (floats) of the chunk's x and A rows: 16 words past the tile width, so that
// the four k-rows an MFMA operand reads fall into different LDS banks
constexpr int kSnapLDR = kSnapTM + 16, kSnapLDA = kSnapTN + 16;

__host__ __device__ int64_t cross_snap_tiles(int64_t Mx, int64_t N) {
    return ((Mx + kSnapTM - 1) / kSnapTM) * ((N + 1 + kSnapTN - 1) / kSnapTN);
}

// The snapshot rows of group g in a launch of nsnap sweeps from sweep s0: sweeps j in
// [j0, j1) of the launch and chains [c0, c1) (chain groups), or every chain of the sweeps of
// batch g (batch means: sweep s - burnin in batch floor((s - burnin) G / sweeps)).
struct GroupRows {
    int64_t j0, j1, c0, c1;
};

__device__ __forceinline__ GroupRows group_rows(const ProbDesc &pd, int g, int64_t nsnap, int64_t s0,
                                                int64_t burnin, int64_t sweeps) {
    GroupRows r;
    const int64_t G = pd.groups;
    if (pd.batches > 1) {
        const int64_t lo = burnin + (g * sweeps + G - 1) / G, hi = burnin + ((g + 1) * sweeps + G - 1) / G;
        r.j0 = min(max(lo - s0, (int64_t)0), nsnap);
        r.j1 = min(max(hi - s0, (int64_t)0), nsnap);
        r.c0 = 0;
        r.c1 = pd.C;
    } else {
        r.j0 = 0;
        r.j1 = nsnap;
        r.c0 = pd.C * g / G;
        r.c1 = pd.C * (g + 1) / G;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_cross_snap(const ProbDesc *probs, int parts, int64_t nsnap,
                                                    const float *snapA, const float *snapR,
                                                    const int64_t *snap_first, int64_t burnin, int64_t sweeps,
                                                    double *cross) {
    __shared__ __align__(16) float sr[kSnapKC * kSnapLDR];
    __shared__ __align__(16) float sa[kSnapKC * kSnapLDA];
    const ProbDesc pd = probs[blockIdx.z];
    const int ksplit = pd.groups * parts;
    const int64_t M = pd.M, N = pd.N, N1 = N + 1;
    const int64_t Mx = pd.rank_r > 0 ? pd.rank_r : M;   // rows of the cross moment
    const int64_t ldr = (M + 3) / 4 * 4, lda = (N + 3) / 4 * 4;
    const int64_t ntn = (N1 + kSnapTN - 1) / kSnapTN;
    // XCD-aware order when the splits come in multiples of 8: workgroups are dealt to the 8
    // XCDs in turn, so workgroup x runs on XCD x % 8; all tiles of one split then run on one
    // XCD and read the split's snapshot rows through that XCD's L2
    const int64_t maxt = gridDim.x / ksplit;
    int split;
    int64_t tile;
    if (ksplit % 8 == 0) {
        const int64_t xcd = blockIdx.x % 8, j = blockIdx.x / 8;
        split = (int)(xcd + 8 * (j / maxt));
        tile = j % maxt;
    } else {
        split = (int)(blockIdx.x / maxt);
        tile = blockIdx.x % maxt;
    }
    if (tile >= cross_snap_tiles(Mx, N)) return;
    const int g = split / parts, part = split % parts;
    const GroupRows gr = group_rows(pd, g, nsnap, *snap_first, burnin, sweeps);
    const int64_t nc = gr.c1 - gr.c0;
    const int64_t K = (gr.j1 - gr.j0) * nc;
    const int64_t k_lo = K * part / parts, k_hi = K * (part + 1) / parts;
    // the snapshot row of chunk row r (< kSnapKC) for the chunk starting at split row
    // js nc + cs: rows run over the group's chains, then its sweeps (no division per row)
    int64_t js = nc > 0 ? k_lo / nc : 0, cs = nc > 0 ? k_lo % nc : 0;
    auto row_of = [&](int r) {
        int64_t jj = js, cc = cs + r;
        while (cc >= nc) {
            cc -= nc;
            ++jj;
        }
        return (gr.j0 + jj) * pd.C + gr.c0 + cc;
    };
    auto next_chunk = [&]() {
        cs += kSnapKC;
        while (cs >= nc) {
            cs -= nc;
            ++js;
        }
    };
    const int64_t m0 = (tile / ntn) * kSnapTM, n0 = (tile % ntn) * kSnapTN;
    const float *Rb = snapR + pd.off_sr;
    const float *Ab = snapA + pd.off_sa;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    // the wavefront's 64 x 32 sub-tile: all rows of the tile, columns 32 wave .. 32 wave + 31,
    // so that rows past Mx (the range basis' rank is rarely a multiple of 64) leave every
    // wavefront the same number of MFMAs (a wavefront's SIMD is fixed by its index)
    const int i = lane % 16, kk = lane / 16;
    d4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
    // 16 x 16 sub-tiles entirely past Mx or N + 1 are skipped (wavefront-uniform)
    const int64_t nw = n0 + 32 * wave;
    // one 16-byte word of x and two of A per thread and chunk, loaded a chunk ahead
    const int rrow = tid / (kSnapTM / 4), rc4 = tid % (kSnapTM / 4);
    const int64_t rm = m0 + 4 * rc4;
    auto load_r = [&](int64_t kc) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (rrow < kc && rm < ldr) v = *reinterpret_cast<const float4 *>(Rb + row_of(rrow) * ldr + rm);
        if (rm + 0 >= Mx) v.x = 0.f;
        if (rm + 1 >= Mx) v.y = 0.f;
        if (rm + 2 >= Mx) v.z = 0.f;
        if (rm + 3 >= Mx) v.w = 0.f;
        return v;
    };
    auto load_a = [&](int64_t kc, int h) {
        const int e = tid + h * 256;
        const int row = e / (kSnapTN / 4), c4 = e % (kSnapTN / 4);
        const int64_t n = n0 + 4 * c4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < kc) {
            if (n < lda) v = *reinterpret_cast<const float4 *>(Ab + row_of(row) * lda + n);
            if (n + 0 >= N) v.x = (n + 0 == N) ? 1.f : 0.f;
            if (n + 1 >= N) v.y = (n + 1 == N) ? 1.f : 0.f;
            if (n + 2 >= N) v.z = (n + 2 == N) ? 1.f : 0.f;
            if (n + 3 >= N) v.w = (n + 3 == N) ? 1.f : 0.f;
        }
        return v;
    };
    float4 pr = make_float4(0.f, 0.f, 0.f, 0.f), pa0 = pr, pa1 = pr;
    if (k_lo < k_hi) {
        const int64_t kc = (k_hi - k_lo) < kSnapKC ? (k_hi - k_lo) : kSnapKC;
        pr = load_r(kc);
        pa0 = load_a(kc, 0);
        pa1 = load_a(kc, 1);
    }
    for (int64_t c0 = k_lo; c0 < k_hi; c0 += kSnapKC) {
        __syncthreads();   // the previous chunk is consumed
        // x rows: kc x 64 (columns past Mx, rows past kc: 0); A rows with the column of ones
        // at n = N: kc x 128
        *reinterpret_cast<float4 *>(sr + rrow * kSnapLDR + 4 * rc4) = pr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + h * 256;
            const int row = e / (kSnapTN / 4), c4 = e % (kSnapTN / 4);
            *reinterpret_cast<float4 *>(sa + row * kSnapLDA + 4 * c4) = h == 0 ? pa0 : pa1;
        }
        __syncthreads();
        if (c0 + kSnapKC < k_hi) {
            const int64_t c1 = c0 + kSnapKC;
            const int64_t kc = (k_hi - c1) < kSnapKC ? (k_hi - c1) : kSnapKC;
            next_chunk();
            pr = load_r(kc);
            pa0 = load_a(kc, 0);
            pa1 = load_a(kc, 1);
        }
#pragma unroll
        for (int k4 = 0; k4 < kSnapKC; k4 += 4) {
            const int row = k4 + kk;
            double ra[4], bb[2];
#pragma unroll
            for (int a = 0; a < 4; ++a) ra[a] = (double)sr[row * kSnapLDR + 16 * a + i];
#pragma unroll
            for (int b = 0; b < 2; ++b) bb[b] = (double)sa[row * kSnapLDA + 32 * wave + 16 * b + i];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    if (m0 + 16 * a < Mx && nw + 16 * b < N1)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[a], bb[b], acc[a][b], 0, 0, 0);
        }
    }
    double *X = cross + pd.off_cross + (int64_t)split * Mx * N1;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = m0 + 16 * a + lane / 16 + 4 * j;
                const int64_t col = nw + 16 * b + lane % 16;
                if (row < Mx && col < N1) X[row * N1 + col] += acc[a][b][j];
            }
}

hipError_t launch_cross_snap(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles, int groups, int parts,
                             int64_t nsnap, const float *snapA, const float *snapR, const int64_t *snap_first,
                             int64_t burnin, int64_t sweeps, double *cross, hipStream_t s) {
    const int64_t ksplit = (int64_t)groups * parts;
    hipLaunchKernelGGL(k_cross_snap, dim3((unsigned)(max_tiles * ksplit), 1, (unsigned)P), dim3(256), 0, s,
                       probs_dev, parts, nsnap, snapA, snapR, snap_first, burnin, sweeps, cross);
    return hipGetLastError();
}

// The residual coordinates of every snapshot row of a launch, from the sampled state itself:
// y_k = y0 - W A_k with W = Q^T K~ and y0 = Q^T g~ (range basis Q, rank_r > 0), or W = K~ and
// y0 = g~ (rank_r = 0: y_k = g~ - K~ A_k).  The float32 sampler's carried residual drifts
// between refreshes (its zero modes are float32 roundings of exact null vectors, and K~ is
// ill-conditioned), so the VJP's moments take the residual of the state, in float64.
// A (rows x N, float32) times W^T (N x Mx): a workgroup of 4 wavefronts owns kProjRows rows
// and up to kProjCols columns (column group blockIdx.y); the grid points pass through LDS in
// chunks of kProjKC, the A rows (kProjRows x kProjKC floats, rows padded to kProjLDA words) and
// the map (kProjKC x kProjCols doubles, n-major as stored, rows padded to kProjLDW doubles), the
// next chunk loaded into registers while the current one is multiplied.  The paddings put the
// four k-rows an MFMA operand reads into different LDS banks.  Wavefront w forms rows
// 32 w .. 32 w + 31 by MFMA f64 16x16x4, one accumulator per 16 x 16 block.
constexpr int kProjKC = 32, kProjLDA = 36, kProjRows = 128, kProjCols = 64, kProjLDW = 80;

__global__ __launch_bounds__(256) void k_project(const ProbDesc *probs, int64_t nsnap, const double *WY,
                                                 const float *snapA, float *yrow) {
    __shared__ __align__(16) float sA[kProjRows * kProjLDA];
    __shared__ __align__(16) double sW[kProjKC * kProjLDW];
    const ProbDesc pd = probs[blockIdx.z];
    const int64_t N = pd.N, Mx = pd.rank_r > 0 ? pd.rank_r : pd.M, rows = nsnap * pd.C;
    const int64_t ldr = (pd.M + 3) / 4 * 4, lda = (N + 3) / 4 * 4;
    const int64_t r0 = (int64_t)blockIdx.x * kProjRows, j0 = (int64_t)blockIdx.y * kProjCols;
    if (r0 >= rows || j0 >= Mx) return;
    const int ncol = (int)min<int64_t>(kProjCols, Mx - j0);   // columns of this group
    const int ncb = (ncol + 15) / 16;                          // 16-column MFMA blocks
    const float *Ab = snapA + pd.off_sa;
    float *Yb = yrow + pd.off_sr;
    const double *WT = WY + pd.off_w, *y0 = WY + pd.off_w + Mx * N;   // WT[n Mx + j]
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int i = lane % 16, kk = lane / 16;
    // staging: A, kProjRows rows x 8 float4 (four per thread); the map, kProjKC x ncol doubles
    // as double2 words (four per thread)
    constexpr int HA = kProjRows * (kProjKC / 4) / 256, HW = kProjKC * (kProjCols / 2) / 256;
    float4 pa[HA];
    double2 pw[HW];
    auto load = [&](int64_t n0) {
#pragma unroll
        for (int h = 0; h < HA; ++h) {
            const int e = tid + 256 * h, row = e / (kProjKC / 4), c4 = e % (kProjKC / 4);
            const int64_t r = r0 + row, n = n0 + 4 * c4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < rows && n < lda) v = *reinterpret_cast<const float4 *>(Ab + r * lda + n);
            if (n + 0 >= N) v.x = 0.f;
            if (n + 1 >= N) v.y = 0.f;
            if (n + 2 >= N) v.z = 0.f;
            if (n + 3 >= N) v.w = 0.f;
            pa[h] = v;
        }
        const int half = (ncol + 1) / 2;   // double2 words per grid point
#pragma unroll
        for (int h = 0; h < HW; ++h) {
            const int e = tid + 256 * h, k = e / (kProjCols / 2), c2 = e % (kProjCols / 2);
            double2 v = make_double2(0.0, 0.0);
            const int64_t n = n0 + k;
            if (c2 < half && n < N) {
                const int64_t j = j0 + 2 * c2;
                v.x = WT[n * Mx + j];
                v.y = (2 * c2 + 1 < ncol) ? WT[n * Mx + j + 1] : 0.0;
            }
            pw[h] = v;
        }
    };
    d4 acc[2][kProjCols / 16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < kProjCols / 16; ++c) acc[a][c] = d4{0, 0, 0, 0};
    load(0);
    for (int64_t n0 = 0; n0 < N; n0 += kProjKC) {
        __syncthreads();   // the previous chunk is consumed
#pragma unroll
        for (int h = 0; h < HA; ++h) {
            const int e = tid + 256 * h, row = e / (kProjKC / 4), c4 = e % (kProjKC / 4);
            *reinterpret_cast<float4 *>(sA + row * kProjLDA + 4 * c4) = pa[h];
        }
#pragma unroll
        for (int h = 0; h < HW; ++h) {
            const int e = tid + 256 * h, k = e / (kProjCols / 2), c2 = e % (kProjCols / 2);
            *reinterpret_cast<double2 *>(sW + k * kProjLDW + 2 * c2) = pw[h];
        }
        __syncthreads();
        if (n0 + kProjKC < N) load(n0 + kProjKC);
#pragma unroll
        for (int k4 = 0; k4 < kProjKC; k4 += 4) {
            double av[2], wv[kProjCols / 16];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = (double)sA[(32 * wave + 16 * a + i) * kProjLDA + k4 + kk];
#pragma unroll
            for (int c = 0; c < kProjCols / 16; ++c) wv[c] = sW[(k4 + kk) * kProjLDW + 16 * c + i];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < kProjCols / 16; ++c)
                    if (c < ncb) acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], wv[c], acc[a][c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < kProjCols / 16; ++c) {
            if (c >= ncb) continue;
            const int64_t col = j0 + 16 * c + lane % 16;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = r0 + 32 * wave + 16 * a + lane / 16 + 4 * j;
                if (row < rows && col < Mx) Yb[row * ldr + col] = (float)(y0[col] - acc[a][c][j]);
            }
        }
}

hipError_t launch_project(const ProbDesc *probs_dev, int64_t P, int64_t max_rows, int64_t max_mx, int64_t nsnap,
                          const double *WY, const float *snapA, float *yrow, hipStream_t s) {
    if (max_rows <= 0 || max_mx <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_project, dim3((unsigned)((max_rows + kProjRows - 1) / kProjRows),
                                       (unsigned)((max_mx + kProjCols - 1) / kProjCols),
                                       (unsigned)P),
                       dim3(256), 0, s, probs_dev, nsnap, WY, snapA, yrow);
    return hipGetLastError();
}

// [W^T | y0] of every problem for k_project: W = Q^T K~ (Mx x N), stored n-major (entry
// (j, n) at off_w + n Mx + j), and y0 = Q^T g~ (at off_w + N Mx), or K~ and g~ themselves
// without a range basis; one thread per entry.
__global__ void k_resid_map(const ProbDesc *probs, const double *Kt, const double *gt, const double *Q, double *WY) {
    const ProbDesc pd = probs[blockIdx.y];
    const int64_t M = pd.M, N = pd.N, Mx = pd.rank_r > 0 ? pd.rank_r : M;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Mx * (N + 1)) return;
    const int64_t n = e / Mx, j = e % Mx;   // n = N: the entry of y0
    const double *K = Kt + pd.off_K, *g = gt + pd.off_m;
    double x;
    if (pd.rank_r > 0) {
        const double *q = Q + pd.off_q + j * M;
        x = 0.0;
        for (int64_t m = 0; m < M; ++m) x = fma(q[m], n < N ? K[m * N + n] : g[m], x);
    } else {
        x = n < N ? K[j * N + n] : g[j];
    }
    WY[pd.off_w + n * Mx + j] = x;
}

hipError_t launch_resid_map(const ProbDesc *probs_dev, int64_t P, int64_t max_entries, const double *Kt,
                            const double *gt, const double *Q, double *WY, hipStream_t s) {
    if (max_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_resid_map, dim3((unsigned)((max_entries + 255) / 256), (unsigned)P), dim3(256), 0, s,
                       probs_dev, Kt, gt, Q, WY);
    return hipGetLastError();
}

// Orthonormal basis Q of the range of K~ to a relative 1e-10, for the compressed cross moments
// of the VJP: Cov(r~, A) = -K~ Cov(A, A) lies in range(K~) = the span of the blocks' columns
// d_i U_i (their data modes, Sec. IV.B-C; what a block's rank cut drops is below the rounding
// of K~).  Pivoted modified Gram-Schmidt: the column with the largest remaining norm becomes
// the next direction, reorthogonalised once against the directions found, and is projected
// out of every column; it stops when the largest remaining norm falls below 1e-10 of the
// first, or at max_r directions (then rank 0: the problem keeps its uncompressed moments).
// One workgroup per problem; the columns live in `work`.
__global__ __launch_bounds__(1024) void k_range_basis(const ProbDesc *probs, const int64_t *col_first,
                                                      const int64_t *colU, const int64_t *colD, const double *U64,
                                                      const double *d64, const int64_t *work_off, double *work,
                                                      double *Q, int32_t *rank_out, int max_r) {
    extern __shared__ double rb_sm[];   // q (M), then reduction scratch
    const int p = blockIdx.x;
    const ProbDesc pd = probs[p];
    const int64_t M = pd.M;
    const int64_t cf = col_first[p], K = col_first[p + 1] - cf;
    double *W = work + work_off[p];
    double *Qp = Q + pd.off_q;
    double *q = rb_sm;
    double *red = rb_sm + M;            // blockDim.x values
    int *redi = reinterpret_cast<int *>(red + blockDim.x);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int64_t e = tid; e < K * M; e += nt) {
        const int64_t c = e / M, m = e % M;
        W[e] = d64[colD[cf + c]] * U64[colU[cf + c] + m];
    }
    __syncthreads();
    double first = -1.0;
    int R = 0;
    for (;;) {
        // the column of largest remaining norm
        double best = -1.0;
        int bi = -1;
        for (int64_t c = tid; c < K; c += nt) {
            double s2 = 0.0;
            for (int64_t m = 0; m < M; ++m) s2 = fma(W[c * M + m], W[c * M + m], s2);
            if (s2 > best) {
                best = s2;
                bi = (int)c;
            }
        }
        red[tid] = best;
        redi[tid] = bi;
        __syncthreads();
        for (int o = nt / 2; o > 0; o >>= 1) {
            if (tid < o && (red[tid + o] > red[tid] || (red[tid + o] == red[tid] && redi[tid + o] >= 0 &&
                                                       (redi[tid] < 0 || redi[tid + o] < redi[tid])))) {
                red[tid] = red[tid + o];
                redi[tid] = redi[tid + o];
            }
            __syncthreads();
        }
        const double bn2 = red[0];
        const int jb = redi[0];
        __syncthreads();
        if (first < 0.0) first = bn2;
        if (jb < 0 || !(bn2 > 1e-20 * first) || R >= (int)M) break;
        if (R >= max_r) {
            R = 0;   // too many directions for the compressed form
            break;
        }
        const double inv = 1.0 / sqrt(bn2);
        for (int64_t m = tid; m < M; m += nt) q[m] = W[(int64_t)jb * M + m] * inv;
        __syncthreads();
        // reorthogonalise against the directions found: q -= Q (Q^T q), then normalise
        for (int k = tid; k < R; k += nt) {
            double dq = 0.0;
            for (int64_t m = 0; m < M; ++m) dq = fma(Qp[(int64_t)k * M + m], q[m], dq);
            red[k] = dq;
        }
        __syncthreads();
        for (int64_t m = tid; m < M; m += nt) {
            double x = q[m];
            for (int k = 0; k < R; ++k) x = fma(-red[k], Qp[(int64_t)k * M + m], x);
            q[m] = x;
        }
        __syncthreads();
        double part = 0.0;
        for (int64_t m = tid; m < M; m += nt) part = fma(q[m], q[m], part);
        red[tid] = part;
        __syncthreads();
        for (int o = nt / 2; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        const double qn = 1.0 / sqrt(red[0]);
        __syncthreads();
        for (int64_t m = tid; m < M; m += nt) {
            q[m] *= qn;
            Qp[(int64_t)R * M + m] = q[m];
        }
        __syncthreads();
        // remove the direction from every column
        for (int64_t c = tid; c < K; c += nt) {
            double dq = 0.0;
            for (int64_t m = 0; m < M; ++m) dq = fma(q[m], W[c * M + m], dq);
            for (int64_t m = 0; m < M; ++m) W[c * M + m] = fma(-dq, q[m], W[c * M + m]);
        }
        __syncthreads();
        ++R;
    }
    if (tid == 0) rank_out[p] = R;
}

hipError_t launch_range_basis(const ProbDesc *probs_dev, int64_t P, int64_t max_m, const int64_t *col_first,
                              const int64_t *colU, const int64_t *colD, const double *U64, const double *d64,
                              const int64_t *work_off, double *work, double *Q, int32_t *rank_out, int max_r,
                              hipStream_t s) {
    const size_t lds = (size_t)max_m * sizeof(double) + 1024 * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(k_range_basis, dim3((unsigned)P), dim3(1024), lds, s, probs_dev, col_first, colU, colD, U64,
                       d64, work_off, work, Q, rank_out, max_r);
    return hipGetLastError();
}

// One thread per (problem, n): group sums in a fixed order, then mean, standard error over
// the groups and posterior standard deviation.
__global__ void k_finalize(const ProbDesc *probs, int64_t P, const int64_t *n_prefix,
                           const double *accA, const double *accA2, const int32_t *slot_group,
                           const double *slot_count, double *mean, double *stderr_,
                           double *post_sd, double *gmean) {
    const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gi >= n_prefix[P]) return;
    int64_t lo = 0, hi = P - 1;   // problem p with n_prefix[p] <= gi < n_prefix[p+1]
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (n_prefix[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const ProbDesc pd = probs[lo];
    const int64_t n = gi - n_prefix[lo];
    const int64_t N = pd.N;
    double gs[64], gc[64];
    const int G = pd.groups;
    for (int g = 0; g < G; ++g) gs[g] = gc[g] = 0.0;
    double s1 = 0.0, s2 = 0.0, tot = 0.0;
    for (int64_t sl = 0; sl < pd.nslot; ++sl) {
        const double x1 = accA[pd.off_slot + sl * N + n];
        const double x2 = accA2[pd.off_slot + sl * N + n];
        const int g = slot_group[pd.off_tab + sl];
        const double cnt = slot_count[pd.off_tab + sl];
        gs[g] += x1;
        gc[g] += cnt;
        s1 += x1;
        s2 += x2;
        tot += cnt;
    }
    const double mu = tot > 0.0 ? s1 / tot : 0.0;
    double gm_sum = 0.0;
    int ng = 0;
    for (int g = 0; g < G; ++g)
        if (gc[g] > 0.0) {
            gm_sum += gs[g] / gc[g];
            ++ng;
        }
    const double gbar = ng > 0 ? gm_sum / ng : 0.0;
    double v = 0.0;
    for (int g = 0; g < G; ++g)
        if (gc[g] > 0.0) {
            const double d = gs[g] / gc[g] - gbar;
            v += d * d;
        }
    const double se = ng > 1 ? sqrt(v / (double)(ng - 1) / (double)ng) : NAN;
    if (gmean) {   // the group means, groups x (sum N), NaN for a group without samples
        const int64_t tn = n_prefix[P];
        for (int g = 0; g < G; ++g) gmean[g * tn + pd.off_n + n] = gc[g] > 0.0 ? gs[g] / gc[g] : NAN;
    }
    const double var = tot > 0.0 ? s2 / tot - mu * mu : 0.0;
    mean[pd.off_n + n] = mu;
    stderr_[pd.off_n + n] = se;
    if (post_sd) post_sd[pd.off_n + n] = sqrt(var > 0.0 ? var : 0.0);
}

hipError_t launch_finalize(const ProbDesc *probs_dev, int64_t P, const int64_t *n_prefix_dev,
                           int64_t total_n, const double *accA, const double *accA2,
                           const int32_t *slot_group, const double *slot_count, double *mean,
                           double *stderr_, double *post_sd, double *gmean, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((total_n + 127) / 128)), dim3(128), 0, s,
                       probs_dev, P, n_prefix_dev, accA, accA2, slot_group, slot_count, mean,
                       stderr_, post_sd, gmean);
    return hipGetLastError();
}

// The VJP J^T v = -T^T Cov(r~, A) v (Sec. II: Eq. (PI) differentiated in the data; T the
// whitening), per chain group from the group's own moments and pooled over all samples; its
// error bar is the standard deviation of the group values over sqrt(G).  With a range basis
// (rank_r > 0) the moments are of y = Q^T r and Cov(r~, A) = Q Cov(y, A).
// Scratch per plan (total_m = sum of M over the problems, index g * total_m + off_m + i):
//   XV[g][i] = sum_parts sum_n X[i][n] v_n,  XS[g][i] = sum_parts X[i][N]   (G groups)
//   Z[g][i] (G + 1 rows: the groups, then the pooled value), GR[g][m] the same after -T^T Q
//   AV[p G + g] = (sum of A over group g) . v,  NG[p G + g] = samples of group g

// one workgroup per (row i of the moments, group g, problem)
__global__ __launch_bounds__(256) void k_vjp_rows(const ProbDesc *probs, int64_t total_m, int parts,
                                                  const double *cross, const double *v, double *XV, double *XS) {
    const ProbDesc pd = probs[blockIdx.z];
    const int64_t Mx = pd.rank_r > 0 ? pd.rank_r : pd.M;
    const int64_t i = blockIdx.x;
    if (i >= Mx) return;
    const int g = blockIdx.y;
    if (g >= pd.groups) return;
    const int64_t N = pd.N, N1 = N + 1;
    const double *vv = v + pd.off_n;
    double xv = 0.0, xs = 0.0;
    for (int part = 0; part < parts; ++part) {
        const double *X = cross + pd.off_cross + ((int64_t)(g * parts + part) * Mx + i) * N1;
        for (int64_t n = threadIdx.x; n < N; n += blockDim.x) xv = fma(X[n], vv[n], xv);
        if (threadIdx.x == 0) xs += X[N];
    }
    __shared__ double red[256];
    red[threadIdx.x] = xv;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        XV[g * total_m + pd.off_m + i] = red[0];
        XS[g * total_m + pd.off_m + i] = xs;
    }
}

// one workgroup per (group, problem): the group's sum of A dotted with v, and its samples
__global__ __launch_bounds__(256) void k_vjp_group_av(const ProbDesc *probs, const double *accA,
                                                      const int32_t *slot_group, const double *slot_count,
                                                      const double *v, double *AV, double *NG) {
    const ProbDesc pd = probs[blockIdx.y];
    const int g = blockIdx.x;
    if (g >= pd.groups) return;
    const int64_t N = pd.N;
    const double *vv = v + pd.off_n;
    double av = 0.0, ng = 0.0;
    for (int64_t sl = 0; sl < pd.nslot; ++sl) {
        if (slot_group[pd.off_tab + sl] != g) continue;
        ng += slot_count[pd.off_tab + sl];
        const double *a = accA + pd.off_slot + sl * N;
        for (int64_t n = threadIdx.x; n < N; n += blockDim.x) av = fma(a[n], vv[n], av);
    }
    __shared__ double red[256];
    red[threadIdx.x] = av;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        AV[blockIdx.y * (int64_t)pd.groups + g] = red[0];
        NG[blockIdx.y * (int64_t)pd.groups + g] = ng;
    }
}

// one thread per moment row over all problems: the centred moments z_g = XV_g / n_g -
// (XS_g / n_g)(AV_g / n_g) of each group and the pooled one (row G)
__global__ void k_vjp_z(const ProbDesc *probs, int64_t P, const int64_t *m_prefix, int64_t total_m,
                        const double *XV, const double *XS, const double *AV, const double *NG, double *Z) {
    const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gi >= m_prefix[P]) return;
    int64_t lo = 0, hi = P - 1;   // problem p with m_prefix[p] <= gi < m_prefix[p+1]
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (m_prefix[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const ProbDesc pd = probs[lo];
    const int64_t i = gi - m_prefix[lo];
    const int64_t Mx = pd.rank_r > 0 ? pd.rank_r : pd.M;
    const int G = pd.groups;
    if (i >= Mx) {
        for (int g = 0; g <= G; ++g) Z[g * total_m + gi] = 0.0;
        return;
    }
    double sxv = 0.0, sxs = 0.0, sav = 0.0, sn = 0.0;
    for (int g = 0; g < G; ++g) {
        const double n = NG[lo * (int64_t)G + g];
        const double xv = XV[g * total_m + gi], xs = XS[g * total_m + gi], av = AV[lo * (int64_t)G + g];
        Z[g * total_m + gi] = n > 0.0 ? xv / n - (xs / n) * (av / n) : 0.0;
        sxv += xv;
        sxs += xs;
        sav += av;
        sn += n;
    }
    Z[G * total_m + gi] = sn > 0.0 ? sxv / sn - (sxs / sn) * (sav / sn) : 0.0;
}

// one workgroup per (row g of Z, problem): y = Q z (or z), then GR = -T^T y: -y / sigma for
// iid noise, or -L^-T y (back substitution) for a covariance C = L L^T
__global__ __launch_bounds__(256) void k_vjp_map(const ProbDesc *probs, int64_t total_m, const double *Q,
                                                 const double *sigma, const double *Lchol, const double *Z,
                                                 double *GR) {
    const ProbDesc pd = probs[blockIdx.y];
    const int g = blockIdx.x;
    if (g > pd.groups) return;
    const int64_t M = pd.M, R = pd.rank_r;
    const double *z = Z + g * total_m + pd.off_m;
    double *y = GR + g * total_m + pd.off_m;
    for (int64_t m = threadIdx.x; m < M; m += blockDim.x) {
        double x = 0.0;
        if (R > 0) {
            for (int64_t k = 0; k < R; ++k) x = fma(Q[pd.off_q + k * M + m], z[k], x);
        } else {
            x = z[m];
        }
        y[m] = x;
    }
    __syncthreads();
    if (!pd.has_cov) {
        for (int64_t m = threadIdx.x; m < M; m += blockDim.x) y[m] = -y[m] / sigma[pd.off_m + m];
        return;
    }
    // L^T x = y, in place from the last row up
    const double *L = Lchol + pd.off_L;
    __shared__ double red[256];
    for (int64_t i = M - 1; i >= 0; --i) {
        double part = 0.0;
        for (int64_t k = i + 1 + threadIdx.x; k < M; k += blockDim.x) part += L[k * M + i] * y[k];
        red[threadIdx.x] = part;
        __syncthreads();
        for (int o = blockDim.x / 2; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) y[i] = (y[i] - red[0]) / L[i * M + i];
        __syncthreads();
    }
    for (int64_t m = threadIdx.x; m < M; m += blockDim.x) y[m] = -y[m];
}

// one thread per data point: the pooled J^T v and the standard deviation of the group values
// over sqrt(G) (groups with samples only)
__global__ void k_vjp_out(const ProbDesc *probs, int64_t P, const int64_t *m_prefix, int64_t total_m,
                          const double *GR, const double *NG, double *grad, double *grad_se) {
    const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gi >= m_prefix[P]) return;
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (m_prefix[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const ProbDesc pd = probs[lo];
    const int G = pd.groups;
    grad[gi] = GR[G * total_m + gi];
    if (!grad_se) return;
    double s = 0.0;
    int ng = 0;
    for (int g = 0; g < G; ++g)
        if (NG[lo * (int64_t)G + g] > 0.0) {
            s += GR[g * total_m + gi];
            ++ng;
        }
    const double mu = ng > 0 ? s / ng : 0.0;
    double v = 0.0;
    for (int g = 0; g < G; ++g)
        if (NG[lo * (int64_t)G + g] > 0.0) {
            const double d = GR[g * total_m + gi] - mu;
            v += d * d;
        }
    grad_se[gi] = ng > 1 ? sqrt(v / (double)(ng - 1) / (double)ng) : NAN;
}

hipError_t launch_vjp(const ProbDesc *probs_dev, int64_t P, const int64_t *m_prefix_dev, int64_t total_m,
                      int64_t max_m, int groups, int parts, const double *cross, const double *accA,
                      const int32_t *slot_group, const double *slot_count, const double *Q, const double *sigma,
                      const double *Lchol, const double *v, double *scratch, double *grad, double *grad_se,
                      hipStream_t s) {
    const int64_t G = groups;
    double *XV = scratch, *XS = XV + G * total_m, *Z = XS + G * total_m, *GR = Z + (G + 1) * total_m;
    double *AV = GR + (G + 1) * total_m, *NG = AV + P * G;
    hipLaunchKernelGGL(k_vjp_rows, dim3((unsigned)max_m, (unsigned)G, (unsigned)P), dim3(256), 0, s, probs_dev,
                       total_m, parts, cross, v, XV, XS);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vjp_group_av, dim3((unsigned)G, (unsigned)P), dim3(256), 0, s, probs_dev, accA, slot_group,
                       slot_count, v, AV, NG);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_vjp_z, dim3((unsigned)((total_m + 127) / 128)), dim3(128), 0, s, probs_dev, P, m_prefix_dev,
                       total_m, XV, XS, AV, NG, Z);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_vjp_map, dim3((unsigned)(G + 1), (unsigned)P), dim3(256), 0, s, probs_dev, total_m, Q,
                       sigma, Lchol, Z, GR);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_vjp_out, dim3((unsigned)((total_m + 127) / 128)), dim3(128), 0, s, probs_dev, P,
                       m_prefix_dev, total_m, GR, NG, grad, grad_se);
    return hipGetLastError();
}

int64_t vjp_scratch_doubles(int64_t P, int64_t total_m, int groups) {
    return (2 * (int64_t)groups + 2 * ((int64_t)groups + 1)) * total_m + 2 * P * groups;
}

// float64 copy of one problem's chain state
__global__ void k_state64(const ProbDesc *probs, int64_t p, const float *A32, const float *r32,
                          const double *A64, const double *r64, const double *chi2, int fp32,
                          double *A, double *r, double *chi2_out) {
    const ProbDesc pd = probs[p];
    const int64_t tA = pd.C * pd.N, tR = pd.C * pd.M;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tA;
         i += (int64_t)gridDim.x * blockDim.x)
        if (A) A[i] = load_state(A32, A64, pd.off_A + i, fp32);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tR;
         i += (int64_t)gridDim.x * blockDim.x)
        if (r) r[i] = load_state(r32, r64, pd.off_r + i, fp32);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < pd.C;
         i += (int64_t)gridDim.x * blockDim.x)
        if (chi2_out) chi2_out[i] = chi2[pd.off_c + i];
}

hipError_t launch_state64(const ProbDesc *probs_dev, int64_t p, const ProbDesc &ph, const float *A32,
                          const float *r32, const double *A64, const double *r64,
                          const double *chi2, int fp32, double *A, double *r, double *chi2_out,
                          hipStream_t s) {
    int64_t total = ph.C * (ph.N > ph.M ? ph.N : ph.M);
    int grid = (int)((total + 255) / 256);
    if (grid > 2048) grid = 2048;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_state64, dim3(grid), dim3(256), 0, s, probs_dev, p, A32, r32, A64, r64,
                       chi2, fp32, A, r, chi2_out);
    return hipGetLastError();
}

}  // namespace asmk
