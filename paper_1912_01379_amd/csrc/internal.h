// Internal declarations shared by the translation units of libasm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/asm.h"

namespace asmk {

// ------------------------------------------------------------------------------------
// device-visible tables
// ------------------------------------------------------------------------------------
struct ProbDesc {
    int64_t M, N, B, C;       // data points, grid points, blocks, chains
    int64_t off_K;            // whitened kernel K~ (M x N) in Kt
    int64_t off_m;            // M-vectors (g~, sigma, grad) in concatenated arrays
    int64_t off_n;            // N-vectors (mean, stderr, init) in concatenated arrays
    int64_t off_A;            // chain state A: C x N
    int64_t off_r;            // chain state r: C x M
    int64_t off_c;            // per-chain scalars (chi2, drift): C
    int64_t off_blk;          // first block in the block table
    int64_t off_cross;        // groups x parts splits of Mx x (N+1) partial cross moments
                              // sum x [A, 1]^T, x = r (Mx = M) or Q^T r (Mx = rank_r)
    int64_t off_L;            // Cholesky factor (M x M) when whitened with a covariance
    int64_t off_slot;         // element offset of the problem's accumulator slots (slots x N)
    int64_t off_tab;          // first entry of the problem in the slot tables
    int64_t nslot;            // accumulator slots of the problem
    int64_t batches;          // 1, or G when chains < groups (batch means over sweeps)
    int32_t groups;
    int32_t has_cov;
    uint32_t index;           // problem index (keys the random numbers)
    int32_t has_prior;        // 1: gamma-prior shapes at off_n in the shape array
    int64_t off_sa;           // float32 snapshots of A (sweep, chain) rows of round4(N) floats
    int64_t off_sr;           // float32 residual coordinates of the snapshots, rows of round4(M)
    int64_t levels;           // partitions of the hierarchy (1: one partition of B blocks)
    int64_t has_con;          // 1: a linear constraint c . A = F (c at off_n in the constraint array)
    double con_value;         // F
    int64_t off_lvl;          // first level in the level table (pairs: first block, count)
    int64_t rank_r;           // columns of the range basis Q of K~ (float32 VJP moments in its
                              // coordinates), or 0: the moments are of r itself
    int64_t off_q;            // Q (M x rank_r, column j at off_q + j M) in the basis array
    int64_t off_w;            // [W^T | y0] of the snapshot residuals: W = Q^T K~ (Mx x N) stored
                              // n-major, then y0 = Q^T g~ (Mx); K~ and g~ without a basis (Mx = M)
};

struct BlockDesc {
    int64_t n0, nb, kb;       // first grid point, size, data modes
    int64_t nm;               // modes: nb, or nb - 1 under a linear constraint (V is nb x nm)
    int64_t nbp;              // row length of the float32 (V, -1/V) rows (lanes x components)
    int64_t mp;               // row length of the float32 U rows
    int64_t off_V;            // float64 V, mode-major: V[i*nb + q]
    int64_t off_U;            // float64 U, mode-major: U[i*M + m]
    int64_t off_d;            // float64 singular values (kb)
    int64_t off_chunk;        // float32 factor chunk (16-byte words): the LDS image of the block
    int64_t off_U32;          // float32 U, mode-major, kb x mp (read from global memory when the
                              // U rows are not staged)
    int32_t grp_n;            // extended instances, at the first block of a group: the consecutive
                              // blocks of its level staged together (their chunks are contiguous)
    int32_t grp_words;        //   and the 16-byte words of their chunks
};

struct TileDesc {             // float32 work item: consecutive chains of one problem
    int32_t problem;
    int32_t chain0;
    int32_t nchains;
    int32_t slot;             // first accumulator slot of the tile: one per wavefront of its
                              // chains (times the batches of sweeps for batch means)
};

// ------------------------------------------------------------------------------------
// kernel parameter blocks
// ------------------------------------------------------------------------------------
struct SampleArgs {
    const ProbDesc *probs;
    const BlockDesc *blocks;
    const TileDesc *tiles;
    int64_t ntiles;
    const double *Kt;
    const double *gt;
    const double *V64;
    const double *U64;
    const double *d64;
    const float4 *F32;        // factor chunks, one per block, chunk_words 16-byte words each
    const float *U32;
    int64_t chunk_words;
    float *A32;
    float *r32;
    double *A64;
    double *r64;
    double *chi2;             // per chain (float64 sampler)
    double *drift;            // per chain, running max
    double *accA;             // slots x N (per problem offsets)
    double *accA2;
    unsigned long long *counters;  // [0] clamped, [1] frozen, [2] rejected by the prior test
    int *flags;               // bit 0: unbounded zero mode
    int *queue;               // tile queue: 8 range counters (float32 samplers)
    const int64_t *sweep;     // device sweep counter: first sweep of this launch
    int64_t nsw;              // sweeps in this launch
    int64_t burnin;           // sweeps before accumulation starts
    int64_t sweeps;           // accumulated sweeps (for batch means)
    int64_t refresh_every;    // float64 sampler refreshes inside the kernel
    uint64_t seed;
    int32_t accumulate;       // 1: accumulate the sweeps in [burnin, burnin + sweeps) into the
                              //    slots (float32: each block visit adds its final components)
    int32_t pad;
    int64_t lds_off_d;        // byte offsets in the float32 sampler's LDS: singular values,
    int64_t lds_off_u;        //   U rows,
    int64_t lds_off_unif;     //   per-chain uniform rows,
    int64_t lds_off_ce;       //   per-chain rows of the data modes' centres and steps (2 kce)
    int32_t u_lds;            // 1: U rows are staged in LDS (else read from global memory)
    int32_t prefetch;         // 1: every block's factor stream fits the instance's prefetch
    float *snapA;             // nullable (float32 plans with want_vjp): per-sweep snapshots of A,
    int64_t snap_rows;        //   the input of the cross moments, for the accumulated sweeps of
    int64_t *snap_first;      //   the launch at the problems' off_sa; row = sweep - first sweep,
                              //   which goes to *snap_first
    // two-role float32 sampler (sample32p.h): LDS byte offsets of its areas, the chunk word
    // where the singular values (then the U rows) start, the words of the data rows part and
    // of the d/U part, the data-role uniform row length
    int64_t p_off_vwd, p_off_d, p_off_u, p_off_vwz, p_off_und, p_off_unz, p_off_h, p_off_ce;
    int32_t kce;              // floats per half of a chain's centre/step row (largest k, rounded to 4)
    int32_t pad2;
    int64_t p_du_word;
    int32_t p_wd, p_wu, p_kd, p_zs;   // ... and the zero modes the data role runs per block
    const int32_t *lvl;       // level table: (first block relative to the problem's, count)
    const double *shape;      // gamma-prior shapes w_n (problems with has_prior, at off_n)
    const float *wm1f;        // the same as float32 exponents w_n - 1 (float32 sampler)
    int32_t hier;             // 1: a problem has a hierarchy of partitions or a gamma prior
                              //    (float32: the extended instances, which draw a level per
                              //    sweep, stage each block to its size, and test moves against
                              //    the prior)
    int32_t prior;            // 1: a problem has a gamma prior (the extended form with its test)
};

// ------------------------------------------------------------------------------------
// work items of the per-block decomposition
// ------------------------------------------------------------------------------------
struct SvdTask {
    int64_t M, N;        // problem sizes
    int64_t off_K;       // whitened kernel of the problem
    int64_t n0, nb;      // block columns
    int64_t kreq;        // requested data modes, -1 = numerical rank
    int64_t off_V, off_U, off_d;
    int64_t off_work;    // float64 scratch of the task
    int64_t block;       // global block index (kb output)
};

// ------------------------------------------------------------------------------------
// launchers (defined next to their kernels)
// ------------------------------------------------------------------------------------
// setup.hip
hipError_t launch_check_finite(const double *x, int64_t n, int *flag, int bit, hipStream_t s);
hipError_t launch_check_positive(const double *x, int64_t n, int *flag, int bit, hipStream_t s);
hipError_t launch_whiten_diag(const double *K, const double *G, const double *sigma, int64_t M,
                              int64_t N, double *Kt, double *gt, hipStream_t s);
hipError_t launch_cholesky(const double *C, int64_t M, double *L, int *flag, int bit, hipStream_t s);
hipError_t launch_trsm_lower(const double *L, int64_t M, const double *B, int64_t ncols,
                             int64_t ldb, double *X, hipStream_t s);
int64_t svd_work_doubles(int64_t M, int64_t nb);
struct ConTask {              // a block under a linear constraint (nm = nb - 1 modes)
    int64_t M, N;            // problem sizes
    int64_t off_K;           // whitened kernel of the problem
    int64_t n0, nb;          // block columns
    int64_t off_c;           // constraint share c_b in the constraint array
    int64_t off_v;           // Householder vector (nb) and v.v in the scratch
    int64_t off_kq;          // K~_b Q_b (M x nm) in the kernel array
    int64_t off_vp;          // V' (nm x nm) of its decomposition, in V64
    int64_t off_V;           // the block's modes V = Q_b V' (nb x nm, mode-major), in V64
};
hipError_t launch_con_prep(const ConTask *tasks_dev, int64_t n, const double *Kt, const double *con, double *KQ,
                           double *hv, hipStream_t s);
hipError_t launch_con_map(const ConTask *tasks_dev, int64_t n, const double *hv, const double *Vp, double *V64,
                          hipStream_t s);
hipError_t launch_noise_data(const ProbDesc *probs_dev, int64_t P, const double *gt, double *gn, uint64_t seed,
                             hipStream_t s);
hipError_t launch_con_fix(const ProbDesc *probs_dev, const int32_t *chain_problem, const int32_t *chain_local,
                          int64_t total_chains, const double *con, float *A32, hipStream_t s);
hipError_t launch_con_start(const ProbDesc *probs_dev, const int32_t *which, int64_t n, const double *con,
                            double *A64, float *A32, int fp32, int *flag, int bit, hipStream_t s);
hipError_t launch_block_svd_tasks(const SvdTask *tasks_dev, int64_t ntasks, const double *Kt,
                                  double *work, double *V64, double *U64, double *d64,
                                  int32_t *kb_out, hipStream_t s);
struct ChunkLayout {           // float32 factor chunk of a block, in elements of its kind
    int64_t rows;             // (V, w) rows (the largest block plus two spare rows)
    int64_t row;              // pairs per row
    int64_t d_len;            // singular values (largest k, rounded up to 4)
    int64_t u_rows;           // U rows in the chunk (largest k, or 0)
    int64_t mp;               // floats per U row
    int64_t words;            // 16-byte words of the chunk
    int64_t compact;          // 1: each block's image packed to its own size (nb + 2 rows,
                              //    round4(kb) values, kb U rows when staged), for hierarchies
};
hipError_t launch_pack32_blocks(const BlockDesc *blocks_dev, const int64_t *blockM_dev,
                                int64_t nblocks, const double *V64, const double *U64,
                                const double *d64, const ChunkLayout &cl, float4 *F32, float *U32,
                                int *flags, hipStream_t s);
int64_t nnls_work_doubles(int64_t M, int64_t N);
hipError_t launch_nnls(const ProbDesc *probs_dev, int64_t P, const int *use, const double *Kt,
                       const double *gt, double *work, const int64_t *work_off, double blend,
                       double *init, int *has_init, hipStream_t s);
hipError_t launch_init_state2(const ProbDesc *probs_dev, int64_t P, int64_t max_c, const double *Kt,
                              const double *gt, const double *init, const int *has_init,
                              double *A64, float *A32, int fp32, hipStream_t s);

// sample.hip
hipError_t launch_sample64_grid(const SampleArgs &a, int64_t total_chains, const int32_t *chain_problem,
                                const int32_t *chain_local, size_t lds_bytes, hipStream_t s);
hipError_t set_sample64_lds_limit();

// sample32*.hip: the compiled float32 instances (lanes per chain L, components per lane
// EPT, residual entries per lane RPT)
hipError_t launch_sample32_inst(const SampleArgs &a, int lanes, int ept, int rpt, int chains_per_wg,
                                int grid, size_t lds_bytes, hipStream_t s);
int sample32_pick(int lanes, int64_t max_nb, int64_t max_m, int hier, int *ept, int *rpt, int *pf);
hipError_t set_sample32_lds_limit(int bytes);
hipError_t launch_sample32_l4(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds, hipStream_t s);
hipError_t launch_sample32_l8(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds, hipStream_t s);
hipError_t launch_sample32_l16(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds, hipStream_t s);
hipError_t launch_sample32_l32(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds, hipStream_t s);
hipError_t launch_sample32_l64(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds, hipStream_t s);
hipError_t allow_lds_sample32_l4(int bytes);
hipError_t allow_lds_sample32_l8(int bytes);
hipError_t allow_lds_sample32_l16(int bytes);
hipError_t allow_lds_sample32_l32(int bytes);
hipError_t allow_lds_sample32_l64(int bytes);
// sample32p_l16.hip: the two-role instance (16 lanes per chain, 512 threads)
hipError_t launch_sample32p(const SampleArgs &a, int ept, int rpt, int grid, size_t lds, hipStream_t s);
int sample32p_pick(int64_t max_nb, int64_t max_m, int u_lds, int *ept, int *rpt, int *pfr, int *pfu, int *pfz);
hipError_t allow_lds_sample32p(int bytes);
hipError_t launch_sample32w(const SampleArgs &a, int ept, int rpt, int grid, size_t lds, hipStream_t s);
int sample32w_pick(int64_t max_nb, int64_t max_m, int64_t max_kb, int *ept, int *rpt);
hipError_t allow_lds_sample32w(int bytes);
hipError_t launch_bump(int64_t *sweep, int64_t by, int *queue, hipStream_t s);
hipError_t launch_reset_queue(int *queue, hipStream_t s);
hipError_t launch_tn_draw(const double *c, const double *d, const double *lo, const double *hi,
                          const double *u, double *out, int64_t n, int precision, hipStream_t s);
hipError_t launch_uniforms(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep0,
                           int64_t nsweeps, int64_t nblocks, int64_t nmodes, double *out,
                           hipStream_t s);

// linalg.hip
hipError_t launch_refresh_all(const ProbDesc *probs_dev, int64_t P, int64_t max_c, int64_t max_m,
                              const double *Kt, const double *gt, const float *A32, float *r32,
                              const double *A64, double *r64, int fp32, hipStream_t s);
hipError_t launch_rownorm(const ProbDesc *probs_dev, const int32_t *chain_problem,
                          const int32_t *chain_local, int64_t total_chains, const float *r32,
                          const double *r64, int fp32, double *out, const double *prev,
                          double *drift, hipStream_t s);
hipError_t launch_cross_all(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles, int groups, int parts,
                            int bgroup, const float *A32, const float *r32, const double *A64,
                            const double *r64, int fp32, double *cross, hipStream_t s);
hipError_t launch_cross_snap(const ProbDesc *probs_dev, int64_t P, int64_t max_tiles, int groups, int parts,
                             int64_t nsnap, const float *snapA, const float *snapR, const int64_t *snap_first,
                             int64_t burnin, int64_t sweeps, double *cross, hipStream_t s);
__host__ __device__ int64_t cross_snap_tiles(int64_t Mx, int64_t N);
hipError_t launch_project(const ProbDesc *probs_dev, int64_t P, int64_t max_rows, int64_t max_mx, int64_t nsnap,
                          const double *WY, const float *snapA, float *yrow, hipStream_t s);
hipError_t launch_resid_map(const ProbDesc *probs_dev, int64_t P, int64_t max_entries, const double *Kt,
                            const double *gt, const double *Q, double *WY, hipStream_t s);
hipError_t launch_range_basis(const ProbDesc *probs_dev, int64_t P, int64_t max_m, const int64_t *col_first,
                              const int64_t *colU, const int64_t *colD, const double *U64, const double *d64,
                              const int64_t *work_off, double *work, double *Q, int32_t *rank_out, int max_r,
                              hipStream_t s);
hipError_t launch_finalize(const ProbDesc *probs_dev, int64_t P, const int64_t *n_prefix_dev,
                           int64_t total_n, const double *accA, const double *accA2,
                           const int32_t *slot_group, const double *slot_count, double *mean,
                           double *stderr_, double *post_sd, double *gmean, hipStream_t s);
hipError_t launch_vjp(const ProbDesc *probs_dev, int64_t P, const int64_t *m_prefix_dev, int64_t total_m,
                      int64_t max_m, int groups, int parts, const double *cross, const double *accA,
                      const int32_t *slot_group, const double *slot_count, const double *Q, const double *sigma,
                      const double *Lchol, const double *v, double *scratch, double *grad, double *grad_se,
                      hipStream_t s);
int64_t vjp_scratch_doubles(int64_t P, int64_t total_m, int groups);
hipError_t launch_state64(const ProbDesc *probs_dev, int64_t p, const ProbDesc &ph, const float *A32,
                          const float *r32, const double *A64, const double *r64,
                          const double *chi2, int fp32, double *A, double *r, double *chi2_out,
                          hipStream_t s);

}  // namespace asmk
