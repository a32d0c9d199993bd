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

// D(16 chains x 16 rows) = A(16 x 4 grid points) * K~^T(4 x 16); MFMA f64 16x16x4 layouts:
// operand a: lane l holds row l%16, k = l/16; operand b: lane l holds column l%16, k = l/16;
// result: lane l, element j holds row l/16 + 4j, column l%16 (checked on the device).
__global__ __launch_bounds__(256) void k_refresh(const ProbDesc *probs, const double *Kt,
                                                 const double *gt, const float *A32, float *r32,
                                                 const double *A64, double *r64, int fp32) {
    const ProbDesc pd = probs[blockIdx.y];
    const int64_t M = pd.M, N = pd.N, C = pd.C;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t ntm = (M + 15) / 16, ntc = (C + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= ntm * ntc) return;
    const int64_t c0 = (tile / ntm) * 16, m0 = (tile % ntm) * 16;
    const int i = lane % 16, k = lane / 16;
    const int64_t ca = c0 + i, mb = m0 + i;
    const double *K = Kt + pd.off_K;
    const int64_t abase = pd.off_A + ca * N;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const bool ca_ok = ca < C, mb_ok = mb < M;
    int64_t n0 = 0;
    for (; n0 + 16 <= N; n0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t n = n0 + 4 * u + k;
            const double a = ca_ok ? load_state(A32, A64, abase + n, fp32) : 0.0;
            const double b = mb_ok ? K[mb * N + n] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
    }
    for (; n0 < N; n0 += 4) {
        const int64_t n = n0 + k;
        const double a = (ca_ok && n < N) ? load_state(A32, A64, abase + n, fp32) : 0.0;
        const double b = (mb_ok && n < N) ? K[mb * N + n] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    const int64_t m = m0 + lane % 16;
    const double *g = gt + pd.off_m;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t c = c0 + lane / 16 + 4 * j;
        if (c < C && m < M) {
            const double rv = g[m] - acc[j];
            const int64_t idx = pd.off_r + c * M + m;
            if (fp32)
                r32[idx] = (float)rv;
            else
                r64[idx] = rv;
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

hipError_t launch_refresh_all(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles,
                              const double *Kt, const double *gt, const float *A32, float *r32,
                              const double *A64, double *r64, int fp32, hipStream_t s) {
    const unsigned gx = (unsigned)((max_tiles + 3) / 4);
    hipLaunchKernelGGL(k_refresh, dim3(gx, (unsigned)P), dim3(256), 0, s, probs_dev, Kt, gt, A32,
                       r32, A64, r64, fp32);
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

// Cross moment of one sweep, added to per-split float64 partial sums:
//   X_k[m][n] += sum_{c in split k} r[c][m] A[c][n]  for n < N, and X_k[m][N] += sum r[c][m]
// (the last column treats A as having an extra component equal to one).  One wavefront owns
// a 32 x 32 tile of one split (2 x 2 MFMA f64 16x16x4 blocks), so the partial sums are
// updated without atomics and the order of every addition is fixed.
__device__ __forceinline__ double cross_b(const float *A32, const double *A64, int fp32, int64_t base,
                                          int64_t n, int64_t N, bool ok) {
    if (!ok) return 0.0;
    if (n == N) return 1.0;
    return load_state(A32, A64, base + n, fp32);
}

__global__ __launch_bounds__(64) void k_cross(const ProbDesc *probs, int ksplit, const float *A32,
                                              const float *r32, const double *A64, const double *r64,
                                              int fp32, double *cross) {
    const ProbDesc pd = probs[blockIdx.z];
    const int64_t M = pd.M, N = pd.N, C = pd.C, N1 = N + 1;
    const int64_t ntm = (M + 31) / 32, ntn = (N1 + 31) / 32;
    const int64_t tile = blockIdx.x;
    if (tile >= ntm * ntn) return;
    const int split = blockIdx.y;
    const int64_t m0 = (tile / ntn) * 32, n0 = (tile % ntn) * 32;
    const int64_t c_lo = C * split / ksplit, c_hi = C * (split + 1) / ksplit;
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

hipError_t launch_cross_all(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles, int ksplit,
                            const float *A32, const float *r32, const double *A64,
                            const double *r64, int fp32, double *cross, hipStream_t s) {
    hipLaunchKernelGGL(k_cross, dim3((unsigned)max_tiles, (unsigned)ksplit, (unsigned)P), dim3(64), 0, s,
                       probs_dev, ksplit, A32, r32, A64, r64, fp32, cross);
    return hipGetLastError();
}

// Cross moments from the per-sweep snapshots of one launch of the float32 sampler: with the
// rows k = (sweep, chain) of the snapshots,
//   X_split[m][n] += sum_{k in split} r_k[m] A_k[n] (n < N),  X_split[m][N] += sum r_k[m].
// A workgroup of 4 wavefronts owns a 64 x 128 output tile and a range of rows; each
// wavefront owns 32 x 64 of it (2 x 4 MFMA f64 16x16x4 blocks).  The rows pass through LDS
// in chunks of kSnapKC, so every snapshot value is read from memory once per workgroup tile
// that needs it; the float32 values are widened to float64 as they enter the MFMAs.  The
// kernel is sized (12 KB of LDS, about 100 VGPRs, 256 threads) to share CUs with the
// sampler, which it runs beside on a second stream.  Snapshot rows are padded to multiples
// of four floats.
constexpr int kSnapTM = 64, kSnapTN = 128, kSnapKC = 16;

__host__ __device__ int64_t cross_snap_tiles(int64_t M, int64_t N) {
    return ((M + kSnapTM - 1) / kSnapTM) * ((N + 1 + kSnapTN - 1) / kSnapTN);
}

__global__ __launch_bounds__(256) void k_cross_snap(const ProbDesc *probs, int ksplit, int64_t nsnap,
                                                    const float *snapA, const float *snapR, double *cross) {
    __shared__ __align__(16) float sr[kSnapKC * kSnapTM];
    __shared__ __align__(16) float sa[kSnapKC * kSnapTN];
    const ProbDesc pd = probs[blockIdx.z];
    const int64_t M = pd.M, N = pd.N, N1 = N + 1;
    const int64_t ldr = (M + 3) / 4 * 4, lda = (N + 3) / 4 * 4;
    const int64_t ntn = (N1 + kSnapTN - 1) / kSnapTN;
    // XCD-aware order: workgroups are dealt to the 8 XCDs in turn, so workgroup x runs on XCD
    // x % 8; all tiles of one chain split then run on one XCD and read the split's snapshot
    // rows through that XCD's L2 (ksplit is a multiple of 8)
    const int64_t maxt = gridDim.x / ksplit;
    const int64_t xcd = blockIdx.x % 8, j = blockIdx.x / 8;
    const int split = (int)(xcd + 8 * (j / maxt));
    const int64_t tile = j % maxt;
    if (tile >= cross_snap_tiles(M, N)) return;
    const int64_t m0 = (tile / ntn) * kSnapTM, n0 = (tile % ntn) * kSnapTN;
    const int64_t K = nsnap * pd.C;
    const int64_t k_lo = K * split / ksplit, k_hi = K * (split + 1) / ksplit;
    const float *Rb = snapR + pd.off_sr;
    const float *Ab = snapA + pd.off_sa;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    const int wm = wave / 2, wn = wave % 2;   // the wavefront's 32 x 64 sub-tile
    const int i = lane % 16, kk = lane / 16;
    d4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
    // 16 x 16 sub-tiles entirely past M or N + 1 are skipped (wavefront-uniform)
    const int64_t mw = m0 + 32 * wm, nw = n0 + 64 * wn;
    // one 16-byte word of r and two of A per thread and chunk, loaded a chunk ahead
    const int rrow = tid / (kSnapTM / 4), rc4 = tid % (kSnapTM / 4);
    const int64_t rm = m0 + 4 * rc4;
    auto load_r = [&](int64_t c0, int64_t kc) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (rrow < kc && rm < ldr) v = *reinterpret_cast<const float4 *>(Rb + (c0 + rrow) * ldr + rm);
        if (rm + 0 >= M) v.x = 0.f;
        if (rm + 1 >= M) v.y = 0.f;
        if (rm + 2 >= M) v.z = 0.f;
        if (rm + 3 >= M) v.w = 0.f;
        return v;
    };
    auto load_a = [&](int64_t c0, int64_t kc, int h) {
        const int e = tid + h * 256;
        const int row = e / (kSnapTN / 4), c4 = e % (kSnapTN / 4);
        const int64_t n = n0 + 4 * c4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < kc) {
            if (n < lda) v = *reinterpret_cast<const float4 *>(Ab + (c0 + row) * lda + n);
            if (n + 0 >= N) v.x = (n + 0 == N) ? 1.f : 0.f;
            if (n + 1 >= N) v.y = (n + 1 == N) ? 1.f : 0.f;
            if (n + 2 >= N) v.z = (n + 2 == N) ? 1.f : 0.f;
            if (n + 3 >= N) v.w = (n + 3 == N) ? 1.f : 0.f;
        }
        return v;
    };
    float4 pr, pa0, pa1;
    {
        const int64_t kc = (k_hi - k_lo) < kSnapKC ? (k_hi - k_lo) : kSnapKC;
        pr = load_r(k_lo, kc);
        pa0 = load_a(k_lo, kc, 0);
        pa1 = load_a(k_lo, kc, 1);
    }
    for (int64_t c0 = k_lo; c0 < k_hi; c0 += kSnapKC) {
        __syncthreads();   // the previous chunk is consumed
        // r rows: kc x 64 (columns past M, rows past kc: 0); A rows with the column of ones
        // at n = N: kc x 128
        *reinterpret_cast<float4 *>(sr + rrow * kSnapTM + 4 * rc4) = pr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + h * 256;
            const int row = e / (kSnapTN / 4), c4 = e % (kSnapTN / 4);
            *reinterpret_cast<float4 *>(sa + row * kSnapTN + 4 * c4) = h == 0 ? pa0 : pa1;
        }
        __syncthreads();
        if (c0 + kSnapKC < k_hi) {
            const int64_t c1 = c0 + kSnapKC;
            const int64_t kc = (k_hi - c1) < kSnapKC ? (k_hi - c1) : kSnapKC;
            pr = load_r(c1, kc);
            pa0 = load_a(c1, kc, 0);
            pa1 = load_a(c1, kc, 1);
        }
#pragma unroll
        for (int k4 = 0; k4 < kSnapKC; k4 += 4) {
            const int row = k4 + kk;
            double ra[2], bb[4];
#pragma unroll
            for (int a = 0; a < 2; ++a) ra[a] = (double)sr[row * kSnapTM + 32 * wm + 16 * a + i];
#pragma unroll
            for (int b = 0; b < 4; ++b) bb[b] = (double)sa[row * kSnapTN + 64 * wn + 16 * b + i];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (mw + 16 * a < M && nw + 16 * b < N1)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[a], bb[b], acc[a][b], 0, 0, 0);
        }
    }
    double *X = cross + pd.off_cross + (int64_t)split * M * N1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = m0 + 32 * wm + 16 * a + lane / 16 + 4 * j;
                const int64_t col = n0 + 64 * wn + 16 * b + lane % 16;
                if (row < M && col < N1) X[row * N1 + col] += acc[a][b][j];
            }
}

hipError_t launch_cross_snap(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles, int ksplit, int64_t nsnap,
                             const float *snapA, const float *snapR, double *cross, hipStream_t s) {
    if (ksplit % 8 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cross_snap, dim3((unsigned)(max_tiles * ksplit), 1, (unsigned)P), dim3(256), 0, s,
                       probs_dev, ksplit, nsnap, snapA, snapR, cross);
    return hipGetLastError();
}

// One thread per (problem, n): group sums in a fixed order, then mean, standard error over
// the groups and posterior standard deviation.
__global__ void k_finalize(const ProbDesc *probs, int64_t P, const int64_t *n_prefix,
                           const double *accA, const double *accA2, const int32_t *slot_group,
                           const double *slot_count, double *mean, double *stderr_,
                           double *post_sd) {
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
    const double var = tot > 0.0 ? s2 / tot - mu * mu : 0.0;
    mean[pd.off_n + n] = mu;
    stderr_[pd.off_n + n] = se;
    if (post_sd) post_sd[pd.off_n + n] = sqrt(var > 0.0 ? var : 0.0);
}

hipError_t launch_finalize(const ProbDesc *probs_dev, int64_t P, const int64_t *n_prefix_dev,
                           int64_t total_n, const double *accA, const double *accA2,
                           const int32_t *slot_group, const double *slot_count, double *mean,
                           double *stderr_, double *post_sd, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((total_n + 127) / 128)), dim3(128), 0, s,
                       probs_dev, P, n_prefix_dev, accA, accA2, slot_group, slot_count, mean,
                       stderr_, post_sd);
    return hipGetLastError();
}

// y_m = (1/S) sum_n X[m][n] v_n - rbar_m (Abar . v) with X summed over the splits and
// rbar_m = X[m][N] / S; then grad = -T^T y: -y/sigma for iid noise, or -L^-T y for a
// covariance C = L L^T.
__global__ __launch_bounds__(256) void k_vjp_y(const ProbDesc *probs, int64_t P, const int64_t *m_prefix,
                                               int ksplit, const double *cross, const double *mean,
                                               const double *nsamples, const double *sigma, const double *v,
                                               double *y, double *grad) {
    // one workgroup per data point m (over all problems); threads over n
    const int64_t gi = blockIdx.x;
    if (gi >= m_prefix[P]) return;
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (m_prefix[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const ProbDesc pd = probs[lo];
    const int64_t m = gi - m_prefix[lo];
    const int64_t N = pd.N, N1 = N + 1, M = pd.M;
    const double S = nsamples[lo];
    const double *vv = v + pd.off_n;
    const double *mu = mean + pd.off_n;
    double xv = 0.0, av = 0.0, rs = 0.0;
    for (int64_t n = threadIdx.x; n <= N; n += blockDim.x) {
        double x = 0.0;
        for (int k = 0; k < ksplit; ++k) x += cross[pd.off_cross + (int64_t)k * M * N1 + m * N1 + n];
        if (n < N) {
            xv += x * vv[n];
            av += mu[n] * vv[n];
        } else {
            rs = x;
        }
    }
    __shared__ double red[3][256];
    red[0][threadIdx.x] = xv;
    red[1][threadIdx.x] = av;
    red[2][threadIdx.x] = rs;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w /= 2) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ym = red[0][0] / S - (red[2][0] / S) * red[1][0];
        y[pd.off_m + m] = ym;
        if (!pd.has_cov) grad[pd.off_m + m] = -ym / sigma[pd.off_m + m];
    }
}

// x = L^-T y (back substitution), grad = -x; one workgroup per problem with a covariance.
__global__ __launch_bounds__(256) void k_vjp_cov(const ProbDesc *probs, const double *Lchol,
                                                 const double *y, double *grad) {
    const ProbDesc pd = probs[blockIdx.x];
    if (!pd.has_cov) return;
    const int64_t M = pd.M;
    const double *L = Lchol + pd.off_L;
    double *x = grad + pd.off_m;   // holds x during the solve, negated at the end
    __shared__ double red[256];
    for (int64_t i = M - 1; i >= 0; --i) {
        double part = 0.0;
        for (int64_t k = i + 1 + threadIdx.x; k < M; k += blockDim.x) part += L[k * M + i] * x[k];
        red[threadIdx.x] = part;
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) x[i] = (y[pd.off_m + i] - red[0]) / L[i * M + i];
        __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < M; i += blockDim.x) x[i] = -x[i];
}

hipError_t launch_vjp(const ProbDesc *probs_dev, int64_t P, const int64_t *m_prefix_dev,
                      int64_t total_m, int ksplit, const double *cross, const double *mean,
                      const double *nsamples, const double *sigma, const double *Lchol,
                      const double *v, double *y, double *grad, int any_cov, hipStream_t s) {
    hipLaunchKernelGGL(k_vjp_y, dim3((unsigned)total_m), dim3(256), 0, s, probs_dev,
                       P, m_prefix_dev, ksplit, cross, mean, nsamples, sigma, v, y, grad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !any_cov) return e;
    hipLaunchKernelGGL(k_vjp_cov, dim3((unsigned)P), dim3(256), 0, s, probs_dev, Lchol, y, grad);
    return hipGetLastError();
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
