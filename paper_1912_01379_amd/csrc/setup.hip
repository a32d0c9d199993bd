// One-time float64 setup of a plan: input checks, whitening (Sec. IV, after Eq. (chi2):
// C^-1 = T^T T, g~ = T g, K~ = T K with T = diag(1/sigma) or T = L^-1 for C = L L^T),
// per-block singular value decompositions K~_b = U_b D_b V_b^T (Sec. IV.B-C), the zero
// modes of each block, float32 packing for the batched sampler, and the start state.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "rng_tn.h"

namespace asmk {

// ------------------------------------------------------------------------------------
// checks
// ------------------------------------------------------------------------------------
__global__ void k_check_finite(const double *x, int64_t n, int *flag, int bit) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1 << bit);
}

__global__ void k_check_positive(const double *x, int64_t n, int *flag, int bit) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !(x[i] > 0.0 && isfinite(x[i]));
    if (bad) atomicOr(flag, 1 << bit);
}

hipError_t launch_check_finite(const double *x, int64_t n, int *flag, int bit, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int grid = (int)((n + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_check_finite, dim3(grid), dim3(256), 0, s, x, n, flag, bit);
    return hipGetLastError();
}

hipError_t launch_check_positive(const double *x, int64_t n, int *flag, int bit, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int grid = (int)((n + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_check_positive, dim3(grid), dim3(256), 0, s, x, n, flag, bit);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// whitening
// ------------------------------------------------------------------------------------
__global__ void k_whiten_diag(const double *K, const double *G, const double *sigma, int64_t M,
                              int64_t N, double *Kt, double *gt) {
    const int64_t total = M * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / N;
        Kt[i] = K[i] / sigma[m];
    }
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M;
         m += (int64_t)gridDim.x * blockDim.x)
        gt[m] = G[m] / sigma[m];
}

hipError_t launch_whiten_diag(const double *K, const double *G, const double *sigma, int64_t M,
                              int64_t N, double *Kt, double *gt, hipStream_t s) {
    int64_t total = M * N;
    int grid = (int)((total + 255) / 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_whiten_diag, dim3(grid), dim3(256), 0, s, K, G, sigma, M, N, Kt, gt);
    return hipGetLastError();
}

// Cholesky C = L L^T, column by column (left-looking), one workgroup.  L is row-major and
// receives the lower triangle (upper part zeroed).  Sets `bit` in *flag if C is not SPD.
__global__ __launch_bounds__(1024) void k_cholesky(const double *C, int64_t M, double *L, int *flag,
                                                   int bit) {
    __shared__ double s_diag;
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    for (int64_t i = threadIdx.x; i < M * M; i += blockDim.x) {
        const int64_t r = i / M, c = i % M;
        L[i] = (c <= r) ? C[i] : 0.0;
    }
    __syncthreads();
    for (int64_t j = 0; j < M; ++j) {
        // s_i = C_ij - sum_{k<j} L_ik L_jk for i >= j
        for (int64_t i = j + threadIdx.x; i < M; i += blockDim.x) {
            double acc = L[i * M + j];
            const double *li = L + i * M;
            const double *lj = L + j * M;
            for (int64_t k = 0; k < j; ++k) acc -= li[k] * lj[k];
            L[i * M + j] = acc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const double dj = L[j * M + j];
            if (!(dj > 0.0) || !isfinite(dj)) {
                s_bad = 1;
                s_diag = 1.0;
            } else {
                s_diag = sqrt(dj);
            }
        }
        __syncthreads();
        if (s_bad) break;
        const double dj = s_diag;
        for (int64_t i = j + threadIdx.x; i < M; i += blockDim.x)
            L[i * M + j] = (i == j) ? dj : L[i * M + j] / dj;
        __syncthreads();
    }
    if (threadIdx.x == 0 && s_bad) atomicOr(flag, 1 << bit);
}

hipError_t launch_cholesky(const double *C, int64_t M, double *L, int *flag, int bit, hipStream_t s) {
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, C, M, L, flag, bit);
    return hipGetLastError();
}

// X = L^-1 B by forward substitution; one thread per column of B (row-major, ldb).
__global__ void k_trsm_lower(const double *L, int64_t M, const double *B, int64_t ncols,
                             int64_t ldb, double *X) {
    const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    for (int64_t i = 0; i < M; ++i) {
        double acc = B[i * ldb + col];
        const double *li = L + i * M;
        for (int64_t k = 0; k < i; ++k) acc -= li[k] * X[k * ldb + col];
        X[i * ldb + col] = acc / li[i];
    }
}

hipError_t launch_trsm_lower(const double *L, int64_t M, const double *B, int64_t ncols,
                             int64_t ldb, double *X, hipStream_t s) {
    int grid = (int)((ncols + 127) / 128);
    hipLaunchKernelGGL(k_trsm_lower, dim3(grid), dim3(128), 0, s, L, M, B, ncols, ldb, X);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// per-block SVD: one-sided (Hestenes) Jacobi in float64, one workgroup per block.
//
// The min(M, N_b) columns of X (the block itself when M >= N_b, else its transpose) are
// made mutually orthogonal by plane rotations applied in round-robin order; the product
// of the rotations (Acc) gives the right singular vectors (or the left ones for the
// transposed case) and the column norms the singular values.  The data modes are the
// first k = min(k_req, numerical rank) by descending singular value, each signed so that
// sum_q (q+1) V_qi > 0.  The zero modes are the last N_b - k columns of the Householder
// product that triangularises the data-mode columns of V.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(512) void k_block_svd(const SvdTask *tasks, const double *Kt,
                                                   double *work, double *V64, double *U64,
                                                   double *d64, int32_t *kb_out) {
    const SvdTask tk = tasks[blockIdx.x];
    const int64_t M = tk.M, N = tk.N, nb = tk.nb, n0 = tk.n0;
    const bool tr = M < nb;
    const int64_t ncol = tr ? M : nb;
    const int64_t len = tr ? nb : M;
    double *X = work + tk.off_work;                 // len x ncol, column-major
    double *Acc = X + len * ncol;                   // ncol x ncol, column-major
    double *nrm = Acc + ncol * ncol;                // ncol
    double *ordd = nrm + ncol;                      // ncol (indices as doubles)
    double *refl = ordd + ncol;                     // nb x nb reflectors
    double *vvs = refl + nb * nb;                   // nb
    const double *Kb = Kt + tk.off_K;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid / 64, lane = tid % 64, nwaves = nthr / 64;
    __shared__ int s_rot;

    for (int64_t i = tid; i < len * ncol; i += nthr) {
        const int64_t j = i / len, e = i % len;
        X[i] = tr ? Kb[j * N + n0 + e] : Kb[e * N + n0 + j];
    }
    for (int64_t i = tid; i < ncol * ncol; i += nthr) Acc[i] = (i / ncol == i % ncol) ? 1.0 : 0.0;
    __syncthreads();

    const int64_t nc2 = ncol + (ncol & 1);
    const int64_t npairs = nc2 / 2;
    // A pair counts as orthogonal once |x_p . x_q| <= sqrt(len) eps |x_p| |x_q|, the size of
    // the rounding error of the computed inner product.  A pair of columns both below
    // skip |x|_max is not rotated: in a rank-deficient block such columns hold only the
    // rounding noise of the rotations of the larger columns, which each of those renews, so
    // their mutual test is never passed and the sweeps would run on for them alone.  Every
    // pair with a larger column is still rotated until it passes, so the larger columns (the
    // data modes) come out as without the skip; the small ones only shrink in rotations with
    // larger ones and stay below skip |x|_max <= max(M, N_b) eps d_1 / 4, the rank threshold
    // applied below, so they end as zero modes (built from the data-mode columns).
    constexpr double kEps = 2.220446049250313e-16;
    const double tol = sqrt((double)len) * kEps;
    const double skip = fmin(4.0 * sqrt((double)len), 0.25 * (double)(M > nb ? M : nb)) * kEps;
    __shared__ double s_cmax[8], s_thr2;
    for (int sweep = 0; sweep < 60; ++sweep) {
        // the largest squared column norm of the sweep's start
        double cm = 0.0;
        for (int64_t j = wave; j < ncol; j += nwaves) {
            const double *xj = X + j * len;
            double a = 0.0;
            for (int64_t e = lane; e < len; e += 64) a += xj[e] * xj[e];
            cm = fmax(cm, wave_sum(a));
        }
        if (lane == 0) s_cmax[wave] = cm;
        if (tid == 0) s_rot = 0;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int w = 0; w < nwaves; ++w) m = fmax(m, s_cmax[w]);
            s_thr2 = skip * skip * m;
        }
        __syncthreads();
        const double thr2 = s_thr2;
        int rotated = 0;
        for (int64_t r = 0; r < nc2 - 1; ++r) {
            for (int64_t k = wave; k < npairs; k += nwaves) {
                // circle method: position 0 fixed, the others rotate by r
                auto pos = [&](int64_t i) -> int64_t {
                    return i == 0 ? 0 : 1 + (i - 1 + r) % (nc2 - 1);
                };
                int64_t p = pos(k), q = pos(nc2 - 1 - k);
                if (p >= ncol || q >= ncol) continue;
                if (p > q) { int64_t t = p; p = q; q = t; }
                double *xp = X + p * len, *xq = X + q * len;
                double al = 0, be = 0, ga = 0;
                for (int64_t e = lane; e < len; e += 64) {
                    const double a = xp[e], b = xq[e];
                    al += a * a;
                    be += b * b;
                    ga += a * b;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (al < thr2 && be < thr2) continue;
                if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = c * t;
                for (int64_t e = lane; e < len; e += 64) {
                    const double a = xp[e], b = xq[e];
                    xp[e] = c * a - s * b;
                    xq[e] = s * a + c * b;
                }
                double *ap = Acc + p * ncol, *aq = Acc + q * ncol;
                for (int64_t e = lane; e < ncol; e += 64) {
                    const double a = ap[e], b = aq[e];
                    ap[e] = c * a - s * b;
                    aq[e] = s * a + c * b;
                }
                rotated = 1;
            }
            __syncthreads();
        }
        if (rotated && lane == 0) atomicOr(&s_rot, 1);
        __syncthreads();
        if (!s_rot) break;
        __syncthreads();
    }

    // singular values and their descending order
    for (int64_t j = tid; j < ncol; j += nthr) {
        double a = 0;
        const double *xj = X + j * len;
        for (int64_t e = 0; e < len; ++e) a += xj[e] * xj[e];
        nrm[j] = sqrt(a);
    }
    __syncthreads();
    for (int64_t j = tid; j < ncol; j += nthr) {
        int64_t rank = 0;
        const double sj = nrm[j];
        for (int64_t i = 0; i < ncol; ++i) {
            const double si = nrm[i];
            rank += (si > sj) || (si == sj && i < j);
        }
        ordd[rank] = (double)j;
    }
    __syncthreads();
    __shared__ int64_t s_k;
    if (tid == 0) {
        const double s1 = nrm[(int64_t)ordd[0]];
        const double thr = (double)(M > nb ? M : nb) * 2.220446049250313e-16 * s1;
        int64_t r = 0;
        if (s1 > 0.0)
            for (int64_t i = 0; i < ncol; ++i) r += nrm[(int64_t)ordd[i]] > thr;
        int64_t k = r;
        if (tk.kreq >= 0 && tk.kreq < k) k = tk.kreq;
        s_k = k;
        kb_out[tk.block] = (int32_t)k;
    }
    __syncthreads();
    const int64_t k = s_k;
    double *Vb = V64 + tk.off_V;   // mode-major: Vb[i*nb + q]
    double *Ub = U64 + tk.off_U;   // mode-major: Ub[i*M + m]
    for (int64_t i = wave; i < k; i += nwaves) {
        const int64_t j = (int64_t)ordd[i];
        const double sv = nrm[j];
        const double *xj = X + j * len;
        const double *aj = Acc + j * ncol;
        // sign rule: sum_q (q+1) V_qi > 0
        double sgn = 0;
        for (int64_t q = lane; q < nb; q += 64) sgn += (double)(q + 1) * (tr ? xj[q] / sv : aj[q]);
        sgn = wave_sum(sgn);
        const double f = sgn < 0 ? -1.0 : 1.0;
        for (int64_t q = lane; q < nb; q += 64) Vb[i * nb + q] = f * (tr ? xj[q] / sv : aj[q]);
        for (int64_t m = lane; m < M; m += 64) Ub[i * M + m] = f * (tr ? aj[m] : xj[m] / sv);
        if (lane == 0) d64[tk.off_d + i] = sv;
    }
    __syncthreads();

    // Householder completion of the data-mode columns; Y (nb x k, column-major) is a
    // working copy of V_data that the reflectors triangularise.
    double *Y = X;   // reuse (nb * k <= len * ncol)
    for (int64_t i = tid; i < nb * k; i += nthr) {
        const int64_t j = i / nb, q = i % nb;
        Y[i] = Vb[j * nb + q];
    }
    __syncthreads();
    __shared__ double s_beta, s_vv;
    for (int64_t j = 0; j < k; ++j) {
        double *yj = Y + j * nb;
        double *vj = refl + j * nb;   // reflector v_j stored at rows j..nb-1
        if (wave == 0) {
            double s2 = 0;
            for (int64_t q = j + lane; q < nb; q += 64) s2 += yj[q] * yj[q];
            s2 = wave_sum(s2);
            const double alpha = yj[j];
            const double norm = sqrt(s2);
            const double beta = alpha >= 0.0 ? -norm : norm;
            for (int64_t q = j + lane; q < nb; q += 64) vj[q] = (q == j) ? alpha - beta : yj[q];
            double vv = 0;
            for (int64_t q = j + lane; q < nb; q += 64) {
                const double vq = (q == j) ? alpha - beta : yj[q];
                vv += vq * vq;
            }
            vv = wave_sum(vv);
            if (lane == 0) {
                s_beta = beta;
                s_vv = vv;
                vvs[j] = vv;
            }
        }
        __syncthreads();
        const double vv = s_vv;
        if (vv > 0.0) {
            for (int64_t c = j + 1 + wave; c < k; c += nwaves) {
                double *yc = Y + c * nb;
                double dot = 0;
                for (int64_t q = j + lane; q < nb; q += 64) dot += vj[q] * yc[q];
                dot = wave_sum(dot);
                const double f = 2.0 * dot / vv;
                for (int64_t q = j + lane; q < nb; q += 64) yc[q] -= f * vj[q];
            }
        }
        __syncthreads();
    }
    // columns k..nb-1: Q e_col with Q = H_0 H_1 ... H_{k-1}
    for (int64_t col = k + wave; col < nb; col += nwaves) {
        // each lane owns the components q = lane + 64 t throughout
        double *e = Vb + col * nb;
        for (int64_t q = lane; q < nb; q += 64) e[q] = (q == col) ? 1.0 : 0.0;
        for (int64_t j = k - 1; j >= 0; --j) {
            const double vv = vvs[j];
            if (!(vv > 0.0)) continue;
            const double *vj = refl + j * nb;
            double dot = 0;
            for (int64_t q = lane; q < nb; q += 64)
                if (q >= j) dot += vj[q] * e[q];
            dot = wave_sum(dot);
            const double f = 2.0 * dot / vv;
            for (int64_t q = lane; q < nb; q += 64)
                if (q >= j) e[q] -= f * vj[q];
        }
    }
}

int64_t svd_work_doubles(int64_t M, int64_t nb) {
    const int64_t ncol = M < nb ? M : nb;
    const int64_t len = M < nb ? nb : M;
    return len * ncol + ncol * ncol + 2 * ncol + nb * nb + nb + 64;
}

hipError_t launch_block_svd_tasks(const SvdTask *tasks_dev, int64_t ntasks, const double *Kt,
                                  double *work, double *V64, double *U64, double *d64,
                                  int32_t *kb_out, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_svd, dim3((unsigned)ntasks), dim3(512), 0, s, tasks_dev, Kt, work,
                       V64, U64, d64, kb_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// float32 packing.  Each block gets a chunk that is the exact image of its LDS staging area:
//   cl.rows rows of cl.row (V, w) pairs, w = -(1/V)(1 - 2^-21), rows past the block's modes
//     and entries past its grid points (0, NaN);
//   cl.d_len singular values (0 past k_b);
//   cl.u_rows rows of cl.mp U values (0 past k_b rows and past M).
// The shrink of w keeps the sampler's computed interval inside the exact one after its
// roundings.  A NaN w is neutral in the interval search, so a component with V = 0 (which no
// step along the mode can make negative; entries below 2^-100 in magnitude are taken as 0)
// and the padding constrain nothing, and a zero V leaves the component unchanged.  U is also
// written to U32 (k_b rows of mp) for plans that read it from global memory.  A zero mode
// whose V has entries of one sign only has an unbounded interval (Sec. IV.B, d_i = 0: the
// posterior is improper): bit 0 of *flags is set.
// ------------------------------------------------------------------------------------
__global__ void k_pack32(const BlockDesc *blocks, const int64_t *blockM, const double *V64,
                         const double *U64, const double *d64, ChunkLayout cl, float4 *F32,
                         float *U32, int *flags) {
    const BlockDesc bd = blocks[blockIdx.x];
    const int64_t M = blockM[blockIdx.x];
    const int64_t nb = bd.nb, kb = bd.kb, mp = bd.mp;
    constexpr double kTiny = 0x1.0p-100;
    const int64_t nm = bd.nm;   // modes (V is nb x nm, mode-major)
    const int64_t rows = cl.compact ? nm + 2 : cl.rows;
    const int64_t d_len = cl.compact ? (kb + 3) / 4 * 4 : cl.d_len;
    const int64_t u_rows = cl.compact ? (cl.u_rows > 0 ? kb : 0) : cl.u_rows;
    float2 *vwc = reinterpret_cast<float2 *>(F32 + bd.off_chunk);
    float *dc = reinterpret_cast<float *>(vwc + rows * cl.row);
    float *uc = dc + d_len;
    for (int64_t i = threadIdx.x; i < rows * cl.row; i += blockDim.x) {
        const int64_t mode = i / cl.row, q = i % cl.row;
        float2 vw;
        const double v = (mode < nm && q < nb) ? V64[bd.off_V + mode * nb + q] : 0.0;
        if (fabs(v) >= kTiny) {
            vw.x = (float)v;
            vw.y = (float)(-(1.0 / v) * (1.0 - 0x1.0p-21));
        } else {
            vw.x = 0.0f;
            vw.y = __builtin_nanf("");
        }
        vwc[i] = vw;
    }
    for (int64_t i = threadIdx.x; i < d_len; i += blockDim.x) dc[i] = i < kb ? (float)d64[bd.off_d + i] : 0.0f;
    for (int64_t i = threadIdx.x; i < u_rows * cl.mp; i += blockDim.x) {
        const int64_t mode = i / cl.mp, m = i % cl.mp;
        uc[i] = (mode < kb && m < M) ? (float)U64[bd.off_U + mode * M + m] : 0.0f;
    }
    for (int64_t i = threadIdx.x; i < kb * mp; i += blockDim.x) {
        const int64_t mode = i / mp, m = i % mp;
        U32[bd.off_U32 + i] = (m < M) ? (float)U64[bd.off_U + mode * M + m] : 0.0f;
    }
    for (int64_t i = kb + threadIdx.x; i < nm; i += blockDim.x) {
        bool pos = false, neg = false;
        for (int64_t q = 0; q < nb; ++q) {
            const double v = V64[bd.off_V + i * nb + q];
            pos |= v >= kTiny;
            neg |= v <= -kTiny;
        }
        if (!(pos && neg)) atomicOr(flags, 1);
    }
}

hipError_t launch_pack32_blocks(const BlockDesc *blocks_dev, const int64_t *blockM_dev,
                                int64_t nblocks, const double *V64, const double *U64,
                                const double *d64, const ChunkLayout &cl, float4 *F32, float *U32,
                                int *flags, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack32, dim3((unsigned)nblocks), dim3(256), 0, s, blocks_dev, blockM_dev, V64,
                       U64, d64, cl, F32, U32, flags);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// noised data for the NNLS start (Sec. IV.D): g~ + xi, xi_m = sqrt(-2 ln u1) cos(2 pi u2) with
// u1, u2 the float64 uniforms of words (w0, w1) and (w2, w3) of Philox on counter
// (2^32 - 2, m, 0, 5), key (seed_lo, seed_hi ^ problem); one workgroup per problem
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_noise_data(const ProbDesc *probs, const double *gt, double *gn,
                                                    uint64_t seed) {
    const ProbDesc pd = probs[blockIdx.x];
    auto u01 = [](uint32_t a, uint32_t b) {
        const uint64_t j = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
        return ((double)j + 0.5) * 0x1.0p-52;
    };
    for (int64_t m = threadIdx.x; m < pd.M; m += blockDim.x) {
        const U4 w = philox10(U4{0xFFFFFFFEu, (uint32_t)m, 0u, 5u}, (uint32_t)seed,
                              (uint32_t)(seed >> 32) ^ pd.index);
        const double xi = sqrt(-2.0 * log(u01(w.x, w.y))) * cos(2.0 * M_PI * u01(w.z, w.w));
        gn[pd.off_m + m] = gt[pd.off_m + m] + xi;
    }
}

hipError_t launch_noise_data(const ProbDesc *probs_dev, int64_t P, const double *gt, double *gn, uint64_t seed,
                             hipStream_t s) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_noise_data, dim3((unsigned)P), dim3(256), 0, s, probs_dev, gt, gn, seed);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// a linear constraint c . A = F (Sec. IV.E): the modes of a block span the complement of its
// share c_b of c.  The Householder reflector H = I - 2 v v^T / v.v maps c_b to beta e_1
// (v = c_b - beta e_1, beta = -sign(c_b[0]) |c_b|, sign(0) = +1), so H e_1 is parallel to c_b
// and Q_b = [H e_2 ... H e_nb] spans the complement: Q_b[q][p] = d_{q,p+1} - 2 v_q v_{p+1} / v.v.
// The block is decomposed as K~_b Q_b = U D V'^T and its modes are V = Q_b V'.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_con_prep(const ConTask *tasks, const double *Kt, const double *con,
                                                  double *KQ, double *hv) {
    const ConTask t = tasks[blockIdx.x];
    const int64_t M = t.M, N = t.N, nb = t.nb, nm = nb - 1;
    const double *c = con + t.off_c;
    double *v = hv + t.off_v;   // nb entries of v, then v.v
    __shared__ double s_norm, s_vv;
    __shared__ double s_part[256];
    double a = 0.0;
    for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) a += c[q] * c[q];
    s_part[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) s_part[threadIdx.x] += s_part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double norm = sqrt(s_part[0]);
        const double alpha = c[0];
        const double beta = alpha >= 0.0 ? -norm : norm;
        const double v0 = alpha - beta;
        s_norm = norm;
        s_vv = v0 * v0 + (s_part[0] - alpha * alpha);
        v[0] = v0;
        v[nb] = s_vv;
    }
    __syncthreads();
    for (int64_t q = 1 + threadIdx.x; q < nb; q += blockDim.x) v[q] = c[q];
    __syncthreads();
    // KQ (M x nm, row-major): K~_b Q_b = K~_b[:, p+1] - (2 v_{p+1} / v.v) (K~_b v)
    const double *K = Kt + t.off_K;
    const double f = 2.0 / s_vv;
    for (int64_t m = threadIdx.x; m < M; m += blockDim.x) {
        const double *row = K + m * N + t.n0;
        double y = 0.0;
        for (int64_t q = 0; q < nb; ++q) y += row[q] * v[q];
        double *out = KQ + t.off_kq + m * nm;
        for (int64_t p = 0; p < nm; ++p) out[p] = row[p + 1] - f * v[p + 1] * y;
    }
}

// V = Q_b V' (V' nm x nm mode-major from the decomposition, V nb x nm mode-major)
__global__ __launch_bounds__(256) void k_con_map(const ConTask *tasks, const double *hv, const double *Vp,
                                                 double *V64) {
    const ConTask t = tasks[blockIdx.x];
    const int64_t nb = t.nb, nm = nb - 1;
    const double *v = hv + t.off_v;
    const double f = 2.0 / v[nb];
    for (int64_t i = 0; i < nm; ++i) {
        const double *vp = Vp + t.off_vp + i * nm;
        __shared__ double s_part[256];
        double a = 0.0;
        for (int64_t p = threadIdx.x; p < nm; p += blockDim.x) a += v[p + 1] * vp[p];
        s_part[threadIdx.x] = a;
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) s_part[threadIdx.x] += s_part[threadIdx.x + o];
            __syncthreads();
        }
        const double w = s_part[0];
        for (int64_t q = threadIdx.x; q < nb; q += blockDim.x)
            V64[t.off_V + i * nb + q] = (q >= 1 ? vp[q - 1] : 0.0) - f * v[q] * w;
        __syncthreads();
    }
}

hipError_t launch_con_prep(const ConTask *tasks_dev, int64_t n, const double *Kt, const double *con, double *KQ,
                           double *hv, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_con_prep, dim3((unsigned)n), dim3(256), 0, s, tasks_dev, Kt, con, KQ, hv);
    return hipGetLastError();
}

hipError_t launch_con_map(const ConTask *tasks_dev, int64_t n, const double *hv, const double *Vp, double *V64,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_con_map, dim3((unsigned)n), dim3(256), 0, s, tasks_dev, hv, Vp, V64);
    return hipGetLastError();
}

// The start moved onto c . A = F: scaled by F / (c . A) when that is positive (keeping it
// non-negative), else projected along c; a negative component sets flag bit `bit`.  The
// start is the same for every chain of a problem; one workgroup per constrained problem.
__global__ __launch_bounds__(256) void k_con_start(const ProbDesc *probs, const int32_t *which,
                                                   const double *con, double *A64, float *A32,
                                                   int fp32, int *flag, int bit) {
    const ProbDesc pd = probs[which[blockIdx.x]];
    const int64_t N = pd.N;
    const double *c = con + pd.off_n;
    __shared__ double s_a[256], s_b[256];
    double a = 0.0, bsum = 0.0;
    for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
        const double x = fp32 ? (double)A32[pd.off_A + n] : A64[pd.off_A + n];
        a += c[n] * x;
        bsum += c[n] * c[n];
    }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = bsum;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_a[threadIdx.x] += s_a[threadIdx.x + o];
            s_b[threadIdx.x] += s_b[threadIdx.x + o];
        }
        __syncthreads();
    }
    const double cs = s_a[0], cc = s_b[0], F = pd.con_value;
    const bool scale = cs != 0.0 && F / cs > 0.0;
    // the other chains first, from chain 0's values, then chain 0 itself
    int bad = 0;
    auto moved = [&](int64_t n) {
        const double x0 = fp32 ? (double)A32[pd.off_A + n] : A64[pd.off_A + n];
        return scale ? x0 * (F / cs) : x0 + c[n] * ((F - cs) / cc);
    };
    for (int64_t i = N + threadIdx.x; i < pd.C * N; i += blockDim.x) {
        const double x = moved(i % N);
        bad |= !(x >= 0.0);
        if (fp32)
            A32[pd.off_A + i] = (float)x;
        else
            A64[pd.off_A + i] = x;
    }
    __syncthreads();
    for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
        const double x = moved(n);
        bad |= !(x >= 0.0);
        if (fp32)
            A32[pd.off_A + n] = (float)x;
        else
            A64[pd.off_A + n] = x;
    }
    if (bad) atomicOr(flag, 1 << bit);
}

// The float32 chains drift off c . A = F by rounding (each move keeps it only to float32
// precision); at every refresh each chain of a constrained problem is scaled back onto it, just
// before its residual is recomputed.  One wavefront per chain.
__global__ __launch_bounds__(64) void k_con_fix(const ProbDesc *probs, const int32_t *chain_problem,
                                                const int32_t *chain_local, const double *con, float *A32) {
    const ProbDesc pd = probs[chain_problem[blockIdx.x]];
    if (!pd.has_con) return;
    const int64_t N = pd.N;
    float *A = A32 + pd.off_A + (int64_t)chain_local[blockIdx.x] * N;
    const double *c = con + pd.off_n;
    double cs = 0.0;
    for (int64_t n = threadIdx.x; n < N; n += 64) cs += c[n] * (double)A[n];
    for (int o = 32; o >= 1; o >>= 1) cs += __shfl_xor(cs, o);
    const double f = pd.con_value / cs;
    if (!(cs != 0.0 && f > 0.0)) return;
    for (int64_t n = threadIdx.x; n < N; n += 64) A[n] = (float)((double)A[n] * f);
}

hipError_t launch_con_fix(const ProbDesc *probs_dev, const int32_t *chain_problem, const int32_t *chain_local,
                          int64_t total_chains, const double *con, float *A32, hipStream_t s) {
    if (total_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_con_fix, dim3((unsigned)total_chains), dim3(64), 0, s, probs_dev, chain_problem,
                       chain_local, con, A32);
    return hipGetLastError();
}

hipError_t launch_con_start(const ProbDesc *probs_dev, const int32_t *which, int64_t n, const double *con,
                            double *A64, float *A32, int fp32, int *flag, int bit, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_con_start, dim3((unsigned)n), dim3(256), 0, s, probs_dev, which, con, A64, A32, fp32,
                       flag, bit);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// start state: A = init, or the best constant fit c* = (K~1).g~/|K~1|^2 (1 if c* <= 0).
// Workgroup (p, y) writes chains [y c_per, (y + 1) c_per) of problem p, each thread the
// components n = tid + 256 t of every such chain (coalesced rows).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_state(const ProbDesc *probs, const double *Kt,
                                                    const double *gt, const double *init,
                                                    const int *has_init, double *A64, float *A32,
                                                    int fp32) {
    const ProbDesc pd = probs[blockIdx.x];
    const int64_t M = pd.M, N = pd.N;
    const int64_t c_per = (pd.C + gridDim.y - 1) / gridDim.y;
    const int64_t c0 = (int64_t)blockIdx.y * c_per, c1 = min(pd.C, c0 + c_per);
    if (c0 >= c1) return;
    const bool use_init = has_init[blockIdx.x] != 0;
    double cstar = 1.0;
    if (!use_init) {
        const double *K = Kt + pd.off_K;
        const double *g = gt + pd.off_m;
        __shared__ double s_num[256], s_den[256];
        double num = 0, den = 0;
        for (int64_t m = threadIdx.x; m < M; m += blockDim.x) {
            double sm = 0;
            for (int64_t n = 0; n < N; ++n) sm += K[m * N + n];
            num += sm * g[m];
            den += sm * sm;
        }
        s_num[threadIdx.x] = num;
        s_den[threadIdx.x] = den;
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) {
                s_num[threadIdx.x] += s_num[threadIdx.x + o];
                s_den[threadIdx.x] += s_den[threadIdx.x + o];
            }
            __syncthreads();
        }
        cstar = s_num[0] / s_den[0];
        if (!(cstar > 0.0) || !isfinite(cstar)) cstar = 1.0;
    }
    for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
        double a = use_init ? init[pd.off_n + n] : cstar;
        a = a + 0.0;   // a -0.0 start would look like a component of the other sign
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t i = c * N + n;
            if (fp32)
                A32[pd.off_A + i] = (float)a;
            else
                A64[pd.off_A + i] = a;
        }
    }
}

hipError_t launch_init_state2(const ProbDesc *probs_dev, int64_t P, int64_t max_c, const double *Kt,
                              const double *gt, const double *init, const int *has_init,
                              double *A64, float *A32, int fp32, hipStream_t s) {
    // about 64 chains per workgroup, at most 256 workgroups per problem
    const int64_t gy = std::min<int64_t>(256, std::max<int64_t>(1, (max_c + 63) / 64));
    hipLaunchKernelGGL(k_init_state, dim3((unsigned)P, (unsigned)gy), dim3(256), 0, s, probs_dev, Kt, gt, init,
                       has_init, A64, A32, fp32);
    return hipGetLastError();
}

}  // namespace asmk

namespace asmk {

// ------------------------------------------------------------------------------------
// Start model from non-negative least squares, as the paper suggests for a short burn-in
// (Sec. IV.D): Lawson-Hanson active-set NNLS of K~ x = g~ in float64, one workgroup per
// problem, each least-squares subproblem by Householder QR of the passive columns.  The
// start is then (1 - blend) x + blend c*, strictly positive.
// ------------------------------------------------------------------------------------
__device__ double blk_sum(double v, double *red) {
    v = wave_sum(v);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    __syncthreads();
    return t;
}

int64_t nnls_work_doubles(int64_t M, int64_t N) {
    const int64_t P = M < N ? M : N;
    return 3 * N + 2 * M + M * P + P + (P + N + 1) / 2 + 64;
}

__global__ __launch_bounds__(1024) void k_nnls(const ProbDesc *probs, const int *use, const double *Kt,
                                              const double *gt, double *work, const int64_t *work_off,
                                              double blend, double *init, int *has_init) {
    const int pidx = blockIdx.x;
    if (!use[pidx]) return;
    const ProbDesc pd = probs[pidx];
    const int64_t M = pd.M, N = pd.N;
    const int64_t PM = M < N ? M : N;
    const double *K = Kt + pd.off_K;
    const double *g = gt + pd.off_m;
    double *x = work + work_off[pidx];
    double *w = x + N;
    double *s = w + N;
    double *r = s + N;
    double *qg = r + M;
    double *Q = qg + M;                     // M x PM, column-major
    double *beta = Q + M * PM;              // PM
    int *P = reinterpret_cast<int *>(beta + PM);   // PM passive indices, then N flags
    int *inP = P + PM;
    __shared__ double red[16];
    __shared__ int s_arg[16];
    __shared__ int s_np, s_t, s_stop;
    __shared__ double s_best, s_alpha, s_tol;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid / 64, lane = tid % 64, nw = nthr / 64;

    for (int64_t n = tid; n < N; n += nthr) {
        x[n] = 0.0;
        inP[n] = 0;
    }
    // tolerance on the gradient: 10 max(M, N) eps |K~|_1
    double cmax = 0.0;
    for (int64_t n = tid; n < N; n += nthr) {
        double cs = 0.0;
        for (int64_t m = 0; m < M; ++m) cs += fabs(K[m * N + n]);
        cmax = fmax(cmax, cs);
    }
    for (int o = 32; o >= 1; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o));
    if (lane == 0) red[wave] = cmax;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < nw; ++i) t = fmax(t, red[i]);
        s_tol = 10.0 * (double)(M > N ? M : N) * 2.220446049250313e-16 * t;
        s_np = 0;
    }
    __syncthreads();

    for (int outer = 0; outer < 3 * N; ++outer) {
        // r = g - K x over the passive set, w = K^T r
        const int np0 = s_np;
        for (int64_t m = tid; m < M; m += nthr) {
            double acc = g[m];
            for (int j = 0; j < np0; ++j) acc -= K[m * N + P[j]] * x[P[j]];
            r[m] = acc;
        }
        __syncthreads();
        for (int64_t n = tid; n < N; n += nthr) {
            double acc = 0.0;
            for (int64_t m = 0; m < M; ++m) acc += K[m * N + n] * r[m];
            w[n] = acc;
        }
        __syncthreads();
        {
            // the largest w_n above the tolerance over the active set, the smallest n among
            // equal values (that of a scan in increasing n): each thread over its n, then the
            // pairs (value, n) combined across the wavefront and the workgroup (thread 0 ends
            // with the result)
            int best = -1;
            double bv = s_tol;
            for (int64_t n = tid; n < N; n += nthr)
                if (!inP[n] && w[n] > bv) {
                    bv = w[n];
                    best = (int)n;
                }
            for (int o = 32; o >= 1; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int ob = __shfl_xor(best, o);
                if (ob >= 0 && (best < 0 || ov > bv || (ov == bv && ob < best))) {
                    bv = ov;
                    best = ob;
                }
            }
            if (lane == 0) {
                red[wave] = bv;
                s_arg[wave] = best;
            }
            __syncthreads();
            if (tid == 0) {
                for (int i = 1; i < nw; ++i)
                    if (s_arg[i] >= 0 && (best < 0 || red[i] > bv || (red[i] == bv && s_arg[i] < best))) {
                        bv = red[i];
                        best = s_arg[i];
                    }
                s_t = best;
                s_stop = (best < 0 || s_np >= PM) ? 1 : 0;
                if (!s_stop) {
                    P[s_np] = best;
                    inP[best] = 1;
                    s_np = s_np + 1;
                }
            }
        }
        __syncthreads();
        if (s_stop) break;

        for (int inner = 0; inner < 3 * (int)N; ++inner) {
            const int np = s_np;
            // least squares on the passive columns: Householder QR of K~[:, P]
            for (int64_t i = tid; i < M * np; i += nthr) {
                const int64_t j = i / M, m = i % M;
                Q[j * M + m] = K[m * N + P[j]];
            }
            for (int64_t m = tid; m < M; m += nthr) qg[m] = g[m];
            __syncthreads();
            for (int k = 0; k < np; ++k) {
                double *qk = Q + (int64_t)k * M;
                double ss = 0.0;
                for (int64_t m = k + tid; m < M; m += nthr) ss += qk[m] * qk[m];
                ss = blk_sum(ss, red);
                const double alpha = qk[k];
                const double nrm = sqrt(ss);
                const double bet = alpha >= 0.0 ? -nrm : nrm;   // R_kk
                const double v0 = alpha - bet;
                const double vv = ss - alpha * alpha + v0 * v0;   // |v|^2
                __syncthreads();
                if (tid == 0) {
                    qk[k] = v0;
                    beta[k] = bet;
                }
                __syncthreads();
                // apply H = I - 2 v v^T / |v|^2 to the remaining columns and to qg
                for (int c = k + 1 + wave; c <= np; c += nw) {
                    double *qc = (c < np) ? Q + (int64_t)c * M : qg;
                    double dot = 0.0;
                    for (int64_t m = k + lane; m < M; m += 64) dot += qk[m] * qc[m];
                    dot = wave_sum(dot);
                    const double f = vv > 0.0 ? 2.0 * dot / vv : 0.0;
                    for (int64_t m = k + lane; m < M; m += 64) qc[m] -= f * qk[m];
                }
                __syncthreads();
            }
            // R s = (Q^T g)[0:np]; R_kk = beta_k, R_ic = Q[c][i] for i < c: by columns, from the
            // last, each solved value taken off the right-hand sides above it by all threads
            for (int k = np - 1; k >= 0; --k) {
                __syncthreads();   // qg[k] has every later column's part taken off
                const double sk = qg[k] / beta[k];
                if (tid == 0) s[P[k]] = sk;
                const double *qk = Q + (int64_t)k * M;
                for (int i = tid; i < k; i += nthr) qg[i] -= qk[i] * sk;
            }
            __syncthreads();
            if (tid == 0) {
                double amin = 2.0;
                int ok = 1;
                for (int k = 0; k < np; ++k) {
                    const int j = P[k];
                    if (!(s[j] > 0.0)) {
                        ok = 0;
                        const double a = x[j] / (x[j] - s[j]);
                        if (a < amin) amin = a;
                    }
                }
                s_stop = ok;
                s_alpha = amin;
                if (ok) {
                    for (int k = 0; k < np; ++k) x[P[k]] = s[P[k]];
                } else {
                    // move towards s until the first passive component reaches zero, then
                    // return every component at (or below) zero to the active set
                    int nn = 0;
                    for (int k = 0; k < np; ++k) {
                        const int j = P[k];
                        double xj = x[j] + amin * (s[j] - x[j]);
                        if (!(xj > 0.0) || (!(s[j] > 0.0) && x[j] / (x[j] - s[j]) <= amin)) {
                            x[j] = 0.0;
                            inP[j] = 0;
                        } else {
                            x[j] = xj;
                            P[nn++] = j;
                        }
                    }
                    s_np = nn;
                }
            }
            __syncthreads();
            if (s_stop || s_np == 0) break;
        }
        __syncthreads();
    }

    // blend with the best constant fit
    double num = 0.0, den = 0.0;
    for (int64_t m = tid; m < M; m += nthr) {
        double sm = 0.0;
        for (int64_t n = 0; n < N; ++n) sm += K[m * N + n];
        num += sm * g[m];
        den += sm * sm;
    }
    num = blk_sum(num, red);
    den = blk_sum(den, red);
    double cstar = num / den;
    if (!(cstar > 0.0) || !isfinite(cstar)) cstar = 1.0;
    for (int64_t n = tid; n < N; n += nthr) init[pd.off_n + n] = (1.0 - blend) * x[n] + blend * cstar;
    if (tid == 0) has_init[pidx] = 1;
}

hipError_t launch_nnls(const ProbDesc *probs_dev, int64_t P, const int *use, const double *Kt,
                       const double *gt, double *work, const int64_t *work_off, double blend,
                       double *init, int *has_init, hipStream_t s) {
    // one workgroup per problem, 16 wavefronts: its products with K~ are bound by memory latency
    hipLaunchKernelGGL(k_nnls, dim3((unsigned)P), dim3(1024), 0, s, probs_dev, use, Kt, gt, work,
                       work_off, blend, init, has_init);
    return hipGetLastError();
}

}  // namespace asmk
