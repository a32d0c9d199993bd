/*
 * asm.h -- C ABI of the MI355X blocked-modes sampler for the average spectrum method
 *          (K. Ghanem and E. Koch, "The Average Spectrum Method for Analytic Continuation:
 *          Efficient Blocked Modes Sampling and Dependence on Discretization Grid",
 *          arXiv:1912.01379).
 *
 * The library estimates, for each problem, the average over non-negative models
 *
 *     <A> = int_{A>=0} A exp(-chi^2(A)/2) dA / int_{A>=0} exp(-chi^2(A)/2) dA,
 *     chi^2(A) = (G - K A)^T C^-1 (G - K A)                      (Sec. II, Eq. (PI);
 *                                                                 Sec. IV, Eq. (chi2))
 *
 * by blocked modes sampling (Sec. IV.B-C): the grid is split into blocks, the whitened
 * kernel of each block is decomposed once, K~_b = U_b D_b V_b^T, and a Markov chain moves
 * one block along one of its singular modes at a time, the new mode coordinate being drawn
 * from a Gaussian of width 1/d_i (flat when d_i = 0) truncated to the interval where
 * A stays non-negative (Eq. (modeLimits)).
 *
 * Conventions for every entry point:
 *   - arrays are row-major, float64, and live in device memory unless a comment says host;
 *   - sizes are int64_t; a problem's N columns are the grid points, its M rows the data;
 *   - the caller owns every buffer it passes; the plan owns everything it allocates and
 *     frees it in asm_plan_destroy;
 *   - all GPU work is enqueued on the stream given to asm_plan_create (a hipStream_t, or
 *     NULL for the default stream); calls that return results synchronise that stream;
 *   - every call returns ASM_OK (0) or a negative error code and never aborts;
 *     asm_last_error() gives a message for the last failing call of the calling thread;
 *   - a plan must not be used by two threads at once.
 */
#ifndef ASM_H
#define ASM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------------------- */
#define ASM_OK          0
#define ASM_EINVAL     (-1)  /* bad sizes, NULL required pointer, bad partition or k      */
#define ASM_EDOMAIN    (-2)  /* non-finite input, sigma <= 0, covariance not SPD, init < 0,
                                prior shape not positive and finite                     */
#define ASM_ESTATE     (-3)  /* call out of order (vjp without want_vjp or before run)    */
#define ASM_EUNBOUNDED (-4)  /* a zero mode whose allowed interval is unbounded: the flat
                                prior makes the posterior improper (Sec. IV.B, d_i = 0)   */
#define ASM_EHIP       (-5)  /* a HIP runtime call failed; the message carries its text    */
#define ASM_ENOMEM     (-6)  /* device allocation failed                                  */

/* ---- precision of the chain state and the moves ------------------------------------ */
#define ASM_FP64 0   /* one wavefront per chain, float64 state: the plain sampler        */
#define ASM_FP32 1   /* batched sampler, float32 state and moves; float64 setup, refresh,
                        and accumulation of <A> and of its covariance with the data     */

typedef struct asm_plan asm_plan;

/* One continuation problem (Sec. II, Sec. IV: data g with covariance C, g = K f after discretising
   f on N grid intervals, Eq. (matrixeq)).  The columns of K already contain the
   quadrature weights of the grid (Eq. (Riemann)), so A is the model on the grid. */
typedef struct {
    int64_t M;                   /* data points (rows of K)                                  */
    int64_t N;                   /* grid points (columns of K)                               */
    const double *K;             /* device, M x N                                            */
    const double *G;             /* device, M: the measured data g                           */
    const double *sigma;         /* device, M: iid standard deviations, C = diag(sigma^2);
                                    NULL when cov is given                                   */
    const double *cov;           /* device, M x M symmetric positive definite covariance C,
                                    whitened with its Cholesky factor (Sec. IV after
                                    Eq. (chi2)); NULL when sigma is given                    */
    int64_t B;                   /* number of blocks of the grid partition (Sec. IV.C); with a
                                    hierarchy (levels > 1), of all its partitions together    */
    const int64_t *block_start;  /* host, B+1 offsets 0 = s_0 < s_1 < ... < s_B = N; with a
                                    hierarchy, the partitions one after another, each with its
                                    own B_l+1 offsets from 0 to N (B + levels entries)        */
    const int32_t *k;            /* host, B: largest number of data modes per block, or NULL;
                                    a block uses min(k_b, numerical rank) data modes (singular
                                    values above max(M, N_b) * 2^-52 * d_1); the remaining
                                    modes of the block are its zero modes, d := 0 (Sec. IV.B) */
    const double *init;          /* device, N start model >= 0 shared by all chains, or NULL
                                    for the best constant fit (K~1).g~/|K~1|^2               */
    int64_t levels;              /* partitions of a hierarchy (Fig. 2, Sec. IV.C); 0 or 1: the
                                    single partition block_start.  With L > 1 levels every
                                    sweep samples all blocks of one level, the same for all
                                    chains of the problem: level floor(w_0 L / 2^32) of the
                                    Philox words of counter (2^32 - 1, sweep, 0, 2); the moves
                                    are keyed by the block's index within its level           */
    const int64_t *level_blocks; /* host, levels: B_l per level (sum = B); NULL when levels <= 1 */
    const double *prior_shape;   /* device, N shapes w_n > 0 of the gamma-prior weights, or NULL
                                    for the flat prior: the chains then sample
                                    prod_n A_n^(w_n - 1) exp(-chi^2/2) on A >= 0 (Sec. V.C,
                                    Eq. (gammadist) and Eq. (compat) in the limit of vanishing
                                    scale; w_n = N rho(x_n) / (N~ rho~(x_n)) simulates the flat
                                    prior of grid (N, rho) on this grid (N~, rho~)).  Each
                                    move's draw is then a proposal, accepted when
                                    log u' < sum_q (w_q - 1) log(A'_q / A_q), u' the float64
                                    uniform of counter (chain, sweep, block << 16 | mode, 3);
                                    a rejected move changes nothing                           */
    const double *constraint_c;  /* device, N: a linear constraint c . A = F, or NULL (Sec. IV.E).
                                    Each block moves only in the complement of its share c_b:
                                    H = I - 2 v v^T / v.v with v = c_b - beta e_1,
                                    beta = -sign(c_b[0]) |c_b| (sign(0) = +1), and
                                    Q_b = [H e_2 ... H e_Nb]; the block's N_b - 1 modes are
                                    V = Q_b V' from K~_b Q_b = U D V'^T (sign rule and zero-mode
                                    completion taken in these coordinates).  A block with
                                    c_b = 0 keeps its N_b modes.  The start (any kind) is scaled
                                    by F / (c . A) when that is positive, else moved along c;
                                    ASM_EDOMAIN if it then has a negative component.  With a
                                    fixed partition each block keeps its own c_b . A_b: the
                                    chains reach every state only when some level holds blocks
                                    that span the constraint (one block, or a hierarchy)     */
    double constraint_value;     /* F                                                         */
} asm_problem;

typedef struct {
    int64_t chains;              /* chains per problem (>= 1)                                */
    int64_t burnin;              /* sweeps discarded before averaging                        */
    int64_t sweeps;              /* sweeps averaged; one sweep moves every mode of every block
                                    (of the sweep's level) once, blocks in increasing order  */
    uint64_t seed;               /* Philox4x32-10 key = (seed_lo, seed_hi ^ problem index)    */
    int32_t precision;           /* ASM_FP64 or ASM_FP32                                      */
    int32_t refresh_every;       /* sweeps between float64 recomputations of the residual
                                    g~ - K~ A (0: never; 64 is a good value)                  */
    int32_t want_vjp;            /* 1: accumulate Cov(r~, A) during the run for asm_plan_vjp  */
    int32_t groups;              /* independent chain groups for the error bars (default 32);
                                    with fewer chains than groups, batches of sweeps are used */
    int32_t lanes_per_chain;     /* ASM_FP32 only: 4, 8, 16, 32 or 64 lanes per chain, 0 = tune */
    int32_t use_graph;           /* 1: ASM_FP32 plans replay each refresh cycle from two
                                    hipGraphs (the sampler launch, captured once per run and
                                    kind of cycle; the float64 refresh, once per plan);
                                    results are identical to eager launches                  */
    int32_t start;               /* start model when a problem gives no init: ASM_START_FLAT
                                    ASM_START_NNLS or ASM_START_NNLS_NOISED                   */
    int32_t roles;               /* ASM_FP32 with 16 lanes per chain: 0 = two roles when the
                                    problems allow it (every problem of two blocks or more,
                                    no hierarchy, prior or constraint),
                                    1 = one role, 2 = two roles (ASM_EINVAL if not allowed).
                                    Two roles run the data modes of block b + 1 beside the
                                    zero modes of block b, which act on disjoint state (the
                                    zero modes leave r~ unchanged, Sec. IV.C): the chains
                                    are bit-identical to one role.
                                    3 = the eight-lane sampler: one role, 8 lanes and 64
                                    chains per workgroup, the uniforms in registers and the
                                    residual entries held in consecutive runs per lane
                                    (one partition with no prior or constraint, blocks of
                                    at most 128 points and 32 data modes, at most 416 data
                                    points, U rows in LDS; ASM_EINVAL otherwise).  With
                                    lanes_per_chain 8 and the automatic workgroup, 0 takes
                                    it where allowed.  Its arithmetic order differs from the
                                    other samplers (same distribution, other rounding)     */
    int32_t chains_per_workgroup;/* ASM_FP32 only: chains per workgroup, a power of two with
                                    lanes_per_chain x chains a multiple of 64 and at most 512
                                    (256 for the prefetching instances; the two-role sampler
                                    takes 16); 0 = automatic (tuned with lanes_per_chain = 0).
                                    The chains are the same for any value                    */
    int32_t u_rows;              /* ASM_FP32 only: 0 = the blocks' U rows are staged in LDS
                                    when they fit, 1 = read from global memory; the same
                                    chains either way                                        */
} asm_options;

/* ---- start model ---------------------------------------------------------------------- */
#define ASM_START_FLAT 0   /* the best constant fit c* = (K~1).g~/|K~1|^2 (1 if c* <= 0)    */
#define ASM_START_NNLS 1   /* (1 - 0.01) x + 0.01 c*, x the non-negative least-squares fit of
                              K~ x = g~ (Lawson-Hanson, float64): a start close to the best
                              fit, as Sec. IV.D suggests, kept strictly positive so that no
                              zero mode starts with an empty interval                        */
#define ASM_START_NNLS_NOISED 2   /* the same from noised data, as Sec. IV.D prefers: K~ x = g~ + xi
                              and c* of g~ + xi, xi_m = sqrt(-2 ln u1) cos(2 pi u2) with u1, u2
                              the float64 uniforms ((w0 >> 6) 2^26 + (w1 >> 6) + 1/2) 2^-52 of
                              the words (w0, w1) and (w2, w3) of Philox4x32-10 on counter
                              (2^32 - 2, m, 0, 5), key (seed_lo, seed_hi ^ problem index)    */

typedef struct {
    double setup_ms;             /* whitening + decompositions + packing + start state        */
    double sample_ms;            /* all sweeps, refreshes and accumulation                    */
    double finalize_ms;
    double mode_moves;           /* moves made: sum over problems of chains*(burnin+sweeps)
                                    * modes per sweep (N; fewer under a constraint; the mean
                                    over the levels of a hierarchy)                          */
    double data_moves;           /* of which along modes with d_i > 0                         */
    double chi2_drift_max;       /* largest |chi^2_incremental - chi^2_recomputed| / chi^2
                                    seen at a refresh                                         */
    int64_t clamped;             /* components rounded below zero and set to +0 (ASM_FP64)    */
    int64_t frozen;              /* moves with an empty interval lo = hi (ASM_FP64)           */
    int32_t lanes_per_chain;     /* the value used                                            */
    int32_t chains_per_block;    /* chains per workgroup used                                 */
    double sampler_ms;           /* summed duration of the sampler launches of the run, from
                                    events recorded around each launch on the plan's stream  */
    int64_t sampler_launches;    /* number of those launches                                  */
    int64_t sampler_sweeps;      /* sweeps they covered (each over all chains)                */
    int64_t graph_replays;       /* refresh cycles replayed from captured hipGraphs (use_graph);
                                    their sampler launches are timed like the others          */
    int64_t roles;               /* 1, 2 or 3: the float32 sampler that ran (asm_options.roles) */
    int64_t rejected;            /* moves rejected by the gamma-prior test (prior_shape)      */
} asm_stats;

/* Validate the problems, whiten them, decompose every block (float64 one-sided Jacobi SVD,
   then the zero modes as the Householder completion of the data modes), pack the factors,
   and set every chain to the start model.  problems: host array of n_problems.  On success
   *out receives the plan.  Errors: ASM_EINVAL, ASM_EDOMAIN, ASM_EHIP, ASM_ENOMEM. */
int asm_plan_create(const asm_problem *problems, int64_t n_problems, const asm_options *opts,
                    void *hip_stream, asm_plan **out);

/* Run burnin + sweeps sweeps from the current chain state and write, concatenated over the
   problems (sum N values each, device):
     mean    -- the average model <A> (Eq. (MCint));
     stderr_ -- standard error of each component over the independent chain groups;
     post_sd -- posterior standard deviation of each component (nullable).
   stats (host, nullable) receives timings and counters.  Errors: ASM_EUNBOUNDED (the
   chain state is then unusable), ASM_EHIP. */
int asm_plan_run(asm_plan *plan, double *mean, double *stderr_, double *post_sd,
                 asm_stats *stats);

/* The estimate of the last asm_plan_run again (mean, stderr_: device, sum N each) and the
   average of each chain group (or batch of sweeps when there are fewer chains than groups)
   behind its error bar: group_means, device, groups x sum N, group-major, NaN for a group
   without samples.  The error bar of any statistic of <A> (a linear functional v . <A>, say)
   is the spread of the statistic over the groups divided by sqrt(groups).
   Errors: ASM_EINVAL, ASM_ESTATE (no run yet), ASM_EHIP. */
int asm_plan_group_means(asm_plan *plan, double *mean, double *stderr_, double *group_means);

/* Vector-Jacobian product of the last asm_plan_run: grad_G = J^T v with
   J = d<A>/dG = -Cov(A, r~) T, r~ = T (G - K A), C^-1 = T^T T, obtained by differentiating
   the normalised posterior of Eq. (PI) with respect to the data; Cov is the pooled sample
   covariance of the run's measured sweeps.  grad_se (nullable): the standard error of each
   entry, the standard deviation over the chain groups (over the batches of sweeps when there
   are fewer chains than groups) of the same product formed from each group's own moments,
   divided by sqrt(groups).  Float32 plans take the moments in the coordinates of an
   orthonormal basis of range(K~) (relative cut 1e-10), where Cov(r~, A) lies.
   v: device, sum N; grad_G, grad_se: device, sum M.  Needs want_vjp = 1.
   Errors: ASM_ESTATE, ASM_EINVAL, ASM_EHIP. */
int asm_plan_vjp(asm_plan *plan, const double *v, double *grad_G, double *grad_se);

/* asm_plan_vjp for callers that cannot allocate device memory (code under stream capture,
   serving loops, harnesses that forbid hipMalloc): the same kernels and the same result, bit
   for bit, with their intermediate products in a fixed per-device array of the library
   (64 MiB, 2^23 doubles; the call needs (4 groups + 2) x sum M + 2 x problems x groups of
   them) instead of a plan buffer.  It allocates nothing and does not wait: the work is
   enqueued on the plan's stream, and grad_G / grad_se are ready when that stream reaches it.
   Every call on one device shares the array, so calls that may overlap on a device (other
   streams, other threads, other plans) race and must be ordered by the caller.  The plan's
   device must be current.  Errors: ASM_ESTATE, ASM_EINVAL (a larger problem than the array
   holds, another device current), ASM_EHIP. */
int asm_plan_vjp_noalloc(asm_plan *plan, const double *v, double *grad_G, double *grad_se);

/* Advance every chain by `sweeps` sweeps without accumulating (burn-in style; the sweep
   counter that keys the random numbers advances).  Errors: ASM_EUNBOUNDED, ASM_EHIP. */
int asm_plan_advance(asm_plan *plan, int64_t sweeps);

/* Copy the current chain state of one problem into device buffers (float64):
   A: chains x N, r: chains x M (the whitened residual g~ - K~ A as carried by the
   chains), chi2: chains (nullable; the running chi^2 of the float64 sampler, or |r|^2). */
int asm_plan_state(asm_plan *plan, int64_t problem, double *A, double *r, double *chi2);

/* Block factors of one problem as used by the sampler: kb (host, 1 int32), d (device, kb),
   U (device, M x kb), V (device, N_b x N_b, column i = mode i, data modes first; under a
   constraint the last column is 0, the block having N_b - 1 modes).  Any output pointer may
   be NULL. */
int asm_plan_factors(asm_plan *plan, int64_t problem, int64_t block, int32_t *kb, double *d,
                     double *U, double *V);

/* Whitened kernel and data of one problem (device, M x N and M); either may be NULL. */
int asm_plan_whitened(asm_plan *plan, int64_t problem, double *Kt, double *gt);

/* Release every device buffer, graph and event of the plan.  NULL is accepted. */
int asm_plan_destroy(asm_plan *plan);

/* Device check of the move primitives, for tests: for each of n entries draws
   delta ~ N(c/d, 1/d^2) truncated to [lo, hi] (lo <= 0 <= hi, d > 0) by inversion at the
   uniform u, with the float64 (precision = ASM_FP64) or float32 (ASM_FP32) device code
   of the samplers.  All arrays device float64 of length n.  Errors: ASM_EINVAL, ASM_EHIP. */
int asm_tn_draw(const double *c, const double *d, const double *lo, const double *hi,
                const double *u, double *out, int64_t n, int32_t precision, void *hip_stream);

/* Device check of the random numbers: out[(s*nblocks + b)*nmodes + i] = the float64 uniform
   of the move (chain, sweep0 + s, b, i) of problem `problem`, for s < nsweeps.  out: device
   float64.  Errors: ASM_EINVAL, ASM_EHIP. */
int asm_uniforms(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep0, int64_t nsweeps,
                 int64_t nblocks, int64_t nmodes, double *out, void *hip_stream);

/* The hierarchy of partitions of Fig. 2 (Sec. IV.C) for N grid points, top level first:
   level l splits the grid into intervals of width w = N / 2^l (one block, then halves, ...),
   shifted by w / 2 on the even levels l >= 2 (so that the grid centre is not a boundary
   there); the boundaries are floor(N (2j + s) / 2^(l+1)), s = 1 on shifted levels, the
   blocked levels run while w >= 2, and the last level is the single points (components
   sampling).  Levels with a block longer than max_block (> 0) are left out.  Host code only
   (no GPU call).  Writes *levels and *n_starts (= B + levels); level_blocks (host, >= 64
   entries) and starts (host, >= *n_starts entries) may be NULL to query the sizes, and
   are filled in the layout of asm_problem.level_blocks and block_start.
   Errors: ASM_EINVAL (N < 1 or N > 2^24). */
int asm_hierarchy(int64_t N, int64_t max_block, int64_t *levels, int64_t *n_starts,
                  int64_t *level_blocks, int64_t *starts);

/* Message of the last failing call on this thread ("" if none). */
const char *asm_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int asm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ASM_H */
