// Host side of the C ABI declared in include/asm.h: validation, plan construction, the
// sweep loop (direct launches or a replayed hipGraph), finalisation and the VJP.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"
#include "rng_tn.h"

using namespace asmk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(ASM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// dynamic LDS a sampler workgroup may use (160 KB per CU, less room for static variables)
constexpr size_t kLdsBudget = 160 * 1024 - 1024;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct asm_plan {
    hipStream_t stream = nullptr;
    int device = -1;          // the device current at creation, where every buffer lives
    asm_options opt{};
    int64_t P = 0;
    std::vector<ProbDesc> probs;
    std::vector<BlockDesc> blocks;
    std::vector<TileDesc> tiles;
    std::vector<int64_t> n_prefix, m_prefix;
    std::vector<int32_t> slot_group;
    std::vector<double> slot_count;
    int64_t total_chains = 0, total_n = 0, total_m = 0;
    int64_t max_cross_tiles = 0, max_m = 0;
    int parts = 1;           // cross-moment partial sums per chain group (splits = groups x parts)
    int64_t cross_words = 0;
    double *Qb = nullptr;     // range bases of the problems' K~ (float32 plans with want_vjp)
    double *WY = nullptr;     // [(Q^T K~)^T | Q^T g~] (or [K~^T | g~]) per problem: snapshot residuals
    int64_t max_mx = 0;       // the largest number of residual coordinates over the problems
    bool any_rank = false;    // a problem whose moments are taken in its range basis
    double *vjp_scratch = nullptr;
    // float32 plans with want_vjp: per-sweep snapshots of A of the accumulated sweeps of a
    // launch, and the residual coordinates formed from them, reduced after each launch into
    // the cross moments on the sampler's stream
    float *snapA = nullptr, *snapR = nullptr;
    int64_t *snap_first = nullptr;   // the sweep of the first snapshot row (device)
    int64_t snap_rows = 0, max_snap_tiles = 0, snap_words_a = 0, snap_words_r = 0;
    int64_t max_nb = 0, max_nbp = 0, max_kb = 0, max_n = 0;
    int64_t lds_off_d = 0, lds_off_u = 0, lds_off_unif = 0, lds_off_ce = 0;   // float32 sampler LDS
    int32_t kce = 4;
    int pf = 0, prefetch = 0;   // prefetch words per thread of the instance; whether used
    int u_lds = 0;
    int roles = 1;           // 2: the two-role sampler (sample32p.h)
    int64_t p_off_vwd = 0, p_off_d = 0, p_off_u = 0, p_off_vwz = 0, p_off_und = 0, p_off_unz = 0, p_off_h = 0,
            p_off_ce = 0;
    int64_t p_du_word = 0;
    int32_t p_wd = 0, p_wu = 0, p_kd = 0, p_zs = 0;
    bool unbounded = false;  // a zero mode with V of one sign (found when packing)
    int ept = 0, rpt = 0;    // compiled float32 instance: components and residual entries per lane
    int fp32 = 1;
    int lanes = 16, chains_per_wg = 16, grid32 = 0;
    int units_per_tile = 1;  // float32: wavefronts (accumulator slots) per tile
    size_t lds32 = 0, lds64 = 0;
    bool any_cov = false;
    bool any_levels = false;   // a problem with a hierarchy of partitions
    float *wm1f = nullptr;     // float32 exponents w_n - 1 of the gamma priors (float32 plans)
    // the float32 sampler's extended instances: hierarchies and gamma priors
    bool ext() const { return any_levels || any_prior || any_con; }
    std::vector<int32_t> lvl;  // level table (pairs: first block of the problem's, count)
    std::vector<ConTask> ctasks;          // constrained blocks (setup)
    std::vector<int64_t> ctask_svd;       // their decomposition tasks
    ConTask *ctasks_d = nullptr;
    double *hv = nullptr;                 // their Householder vectors
    int64_t hv_words = 0, kq_words = 0, vp_words = 0;
    int32_t *d_lvl = nullptr;
    bool ran = false;
    int64_t sweep = 0;      // absolute sweep counter (host mirror)
    std::vector<void *> allocs;

    // device buffers
    ProbDesc *d_probs = nullptr;
    BlockDesc *d_blocks = nullptr;
    TileDesc *d_tiles = nullptr;
    int64_t *d_nprefix = nullptr, *d_mprefix = nullptr;
    int32_t *d_chain_problem = nullptr, *d_chain_local = nullptr;
    double *Kt = nullptr, *gt = nullptr, *Lc = nullptr, *sigma = nullptr;
    double *V64 = nullptr, *U64 = nullptr, *d64 = nullptr;
    float4 *F32 = nullptr;
    float *U32 = nullptr;
    ChunkLayout chunk{};
    float *A32 = nullptr, *r32 = nullptr;
    double *A64 = nullptr, *r64 = nullptr, *chi2 = nullptr, *chi2_prev = nullptr, *drift = nullptr;
    double *accA = nullptr, *accA2 = nullptr, *slot_count_d = nullptr;
    double *shape = nullptr;   // gamma-prior shapes (problems with a prior, at off_n)
    bool any_prior = false;
    bool any_con = false;      // a problem with a linear constraint c . A = F
    double *con = nullptr;     // the constraint vectors c (at off_n)
    int32_t *slot_group_d = nullptr;
    double *cross = nullptr;
    unsigned long long *counters = nullptr;
    int *flags = nullptr, *queue = nullptr;
    int64_t *sweep_d = nullptr;

    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // events around each sampler launch of a run (pairs), reused across runs
    std::vector<hipEvent_t> tev;
    size_t tev_used = 0;
    bool timing = false;
    int64_t timed_sweeps = 0;
    // use_graph: one refresh cycle of the float32 sampler captured per kind (burn-in or
    // accumulating, with or without VJP snapshots) and replayed; recaptured per run
    hipGraphExec_t gexec[8] = {};
    hipGraphExec_t gexec_refresh = nullptr;   // the refresh of a cycle, replayed after the sampler
    int64_t gburnin[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    hipStream_t gstream = nullptr;   // capture stream when the plan's stream is the null stream
    int64_t graph_replays = 0;
};

namespace {

template <typename T>
int dalloc(asm_plan *pl, T **out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) return fail(ASM_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
    pl->allocs.push_back(p);
    *out = static_cast<T *>(p);
    return ASM_OK;
}

#define TRY(expr)              \
    do {                       \
        int rc_ = (expr);      \
        if (rc_ != ASM_OK) return rc_; \
    } while (0)

// The blocks of a problem, level after level, and the levels' block ranges.
struct Partition {
    std::vector<int64_t> n0, nb;          // per block (all levels)
    std::vector<int32_t> lfirst, lcount;  // per level
};

int parse_partition(const asm_problem &q, int64_t p, Partition *out) {
    out->n0.clear();
    out->nb.clear();
    out->lfirst.clear();
    out->lcount.clear();
    if (q.levels < 0 || q.levels > 64) return fail(ASM_EINVAL, "problem %lld: levels must be in [0, 64]", (long long)p);
    const int64_t L = q.levels > 1 ? q.levels : 1;
    if (L > 1 && !q.level_blocks) return fail(ASM_EINVAL, "problem %lld: level_blocks is required with levels > 1", (long long)p);
    if (q.B < 1 || !q.block_start) return fail(ASM_EINVAL, "problem %lld: need B >= 1 blocks", (long long)p);
    if (q.B > 65535) return fail(ASM_EINVAL, "problem %lld: more than 65535 blocks", (long long)p);
    int64_t at = 0, total = 0;
    for (int64_t l = 0; l < L; ++l) {
        const int64_t Bl = L > 1 ? q.level_blocks[l] : q.B;
        if (Bl < 1 || total + Bl > q.B)
            return fail(ASM_EINVAL, "problem %lld: level_blocks must be >= 1 and sum to B", (long long)p);
        const int64_t *cut = q.block_start + at;
        if (cut[0] != 0 || cut[Bl] != q.N)
            return fail(ASM_EINVAL, "problem %lld: block_start must run from 0 to N (level %lld)", (long long)p, (long long)l);
        out->lfirst.push_back((int32_t)total);
        out->lcount.push_back((int32_t)Bl);
        for (int64_t b = 0; b < Bl; ++b) {
            const int64_t nb = cut[b + 1] - cut[b];
            if (nb < 1) return fail(ASM_EINVAL, "problem %lld: blocks must be non-empty and increasing", (long long)p);
            if (nb > 65535) return fail(ASM_EINVAL, "problem %lld: block larger than 65535", (long long)p);
            out->n0.push_back(cut[b]);
            out->nb.push_back(nb);
        }
        at += Bl + 1;
        total += Bl;
    }
    if (total != q.B) return fail(ASM_EINVAL, "problem %lld: level_blocks must sum to B", (long long)p);
    return ASM_OK;
}

int validate(const asm_problem *pr, int64_t n, const asm_options *o) {
    if (!pr || n < 1) return fail(ASM_EINVAL, "need at least one problem");
    if (!o) return fail(ASM_EINVAL, "options are required");
    if (o->chains < 1) return fail(ASM_EINVAL, "chains must be >= 1");
    if (o->burnin < 0 || o->sweeps < 1) return fail(ASM_EINVAL, "burnin >= 0 and sweeps >= 1 required");
    if (o->precision != ASM_FP64 && o->precision != ASM_FP32)
        return fail(ASM_EINVAL, "precision must be ASM_FP64 or ASM_FP32");
    if (o->refresh_every < 0) return fail(ASM_EINVAL, "refresh_every must be >= 0");
    if (o->start != ASM_START_FLAT && o->start != ASM_START_NNLS && o->start != ASM_START_NNLS_NOISED)
        return fail(ASM_EINVAL, "start must be ASM_START_FLAT, ASM_START_NNLS or ASM_START_NNLS_NOISED");
    if (o->groups < 0 || o->groups > 64) return fail(ASM_EINVAL, "groups must be in [1, 64]");
    if (o->lanes_per_chain != 0 && o->lanes_per_chain != 4 && o->lanes_per_chain != 8 &&
        o->lanes_per_chain != 16 && o->lanes_per_chain != 32 && o->lanes_per_chain != 64)
        return fail(ASM_EINVAL, "lanes_per_chain must be 0, 4, 8, 16, 32 or 64");
    if (o->roles < 0 || o->roles > 3) return fail(ASM_EINVAL, "roles must be 0, 1, 2 or 3");
    if (o->chains_per_workgroup < 0 || o->chains_per_workgroup > 512 ||
        (o->chains_per_workgroup & (o->chains_per_workgroup - 1)) != 0)
        return fail(ASM_EINVAL, "chains_per_workgroup must be 0 or a power of two up to 512");
    if (o->u_rows != 0 && o->u_rows != 1) return fail(ASM_EINVAL, "u_rows must be 0 or 1");
    if (o->chains > (1ll << 31) || o->burnin + o->sweeps > (1ll << 31))
        return fail(ASM_EINVAL, "chains and sweeps must fit the 32-bit random-number counter");
    for (int64_t p = 0; p < n; ++p) {
        const asm_problem &q = pr[p];
        if (q.M < 1 || q.N < 1) return fail(ASM_EINVAL, "problem %lld: M and N must be >= 1", (long long)p);
        if (q.M > 4096) return fail(ASM_EINVAL, "problem %lld: M > 4096 is not supported", (long long)p);
        if (!q.K || !q.G) return fail(ASM_EINVAL, "problem %lld: K and G are required", (long long)p);
        if ((q.sigma == nullptr) == (q.cov == nullptr))
            return fail(ASM_EINVAL, "problem %lld: give exactly one of sigma and cov", (long long)p);
        Partition part;
        TRY(parse_partition(q, p, &part));
        for (int64_t b = 0; b < q.B; ++b)
            if (q.k && q.k[b] < 0) return fail(ASM_EINVAL, "problem %lld: k must be >= 0", (long long)p);
    }
    return ASM_OK;
}

int check_flags(asm_plan *pl, int *hflags) {
    HIPCHK(hipMemcpyAsync(hflags, pl->flags, sizeof(int), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    return ASM_OK;
}

// tiles of the float32 sampler: consecutive chains within one error-bar group; each
// wavefront of a tile (64 / lanes chains) accumulates into its own slot
void build_tiles(asm_plan *pl) {
    pl->tiles.clear();
    pl->slot_group.clear();
    pl->slot_count.clear();
    const int cpw = pl->chains_per_wg;
    const int gw = 64 / pl->lanes;                 // chains per wavefront
    pl->units_per_tile = (cpw + gw - 1) / gw;      // wavefronts per tile
    for (int64_t p = 0; p < pl->P; ++p) {
        ProbDesc &pd = pl->probs[p];
        const int64_t C = pd.C, G = pd.groups;
        pd.off_tab = (int64_t)pl->slot_group.size();
        int64_t nunits = 0;
        // a wavefront's chains share one accumulator slot, so they must lie in one chain
        // group; tiles may span groups when every group starts on a wavefront boundary (else
        // each group gets tiles of its own, the last one partly filled)
        bool span = pd.batches == 1;
        for (int64_t g = 1; g < G && span; ++g) span = (g * C / G) % gw == 0;
        const int64_t ngr = (pd.batches > 1 || span) ? 1 : G;
        int64_t gu = 0;   // with spanning tiles: the group of the current unit
        for (int64_t g = 0; g < ngr; ++g) {
            const int64_t c0 = ngr == 1 ? 0 : g * C / G;
            const int64_t c1 = ngr == 1 ? C : (g + 1) * C / G;
            for (int64_t c = c0; c < c1; c += cpw) {
                TileDesc t;
                t.problem = (int32_t)p;
                t.chain0 = (int32_t)c;
                t.nchains = (int32_t)std::min<int64_t>(cpw, c1 - c);
                t.slot = (int32_t)(nunits * pd.batches);
                pl->tiles.push_back(t);
                for (int w = 0; w < pl->units_per_tile; ++w) {
                    const int64_t nc = std::max<int64_t>(0, std::min<int64_t>(gw, t.nchains - (int64_t)w * gw));
                    // the unit's group: that of its first chain (of the tile's last one when
                    // the unit is empty; it then counts no chain)
                    const int64_t cu = nc > 0 ? c + (int64_t)w * gw : c + t.nchains - 1;
                    if (span)
                        while (gu + 1 < G && (gu + 1) * C / G <= cu) ++gu;
                    else
                        gu = g;
                    for (int64_t bt = 0; bt < pd.batches; ++bt) {
                        pl->slot_group.push_back((int32_t)(pd.batches > 1 ? bt : gu));
                        pl->slot_count.push_back((double)nc);
                    }
                    ++nunits;
                }
            }
        }
        pd.nslot = nunits * pd.batches;
    }
}

// slots of the float64 sampler: one unit per chain
void build_chain_slots(asm_plan *pl) {
    pl->slot_group.clear();
    pl->slot_count.clear();
    for (int64_t p = 0; p < pl->P; ++p) {
        ProbDesc &pd = pl->probs[p];
        pd.off_tab = (int64_t)pl->slot_group.size();
        for (int64_t c = 0; c < pd.C; ++c)
            for (int64_t bt = 0; bt < pd.batches; ++bt) {
                pl->slot_group.push_back((int32_t)(pd.batches > 1 ? bt : c * pd.groups / pd.C));
                pl->slot_count.push_back(1.0);
            }
        pd.nslot = pd.C * pd.batches;
    }
}

// sample counts per slot: chains of the slot times the sweeps of its batch
void finish_slot_counts(asm_plan *pl) {
    const int64_t S = pl->opt.sweeps;
    for (int64_t p = 0; p < pl->P; ++p) {
        const ProbDesc &pd = pl->probs[p];
        for (int64_t sl = 0; sl < pd.nslot; ++sl) {
            double &cnt = pl->slot_count[pd.off_tab + sl];
            if (pd.batches > 1) {
                const int64_t bt = sl % pd.batches, G = pd.batches;
                // sweeps s' in [0, S) with floor(s' G / S) == bt
                const int64_t lo = (bt * S + G - 1) / G, hi = ((bt + 1) * S + G - 1) / G;
                cnt *= (double)(hi - lo);
            } else {
                cnt *= (double)S;
            }
        }
    }
}

SampleArgs make_args(asm_plan *pl) {
    SampleArgs a{};
    a.probs = pl->d_probs;
    a.blocks = pl->d_blocks;
    a.tiles = pl->d_tiles;
    a.ntiles = (int64_t)pl->tiles.size();
    a.Kt = pl->Kt;
    a.gt = pl->gt;
    a.V64 = pl->V64;
    a.U64 = pl->U64;
    a.d64 = pl->d64;
    a.F32 = pl->F32;
    a.U32 = pl->U32;
    a.chunk_words = pl->chunk.words;
    a.A32 = pl->A32;
    a.r32 = pl->r32;
    a.A64 = pl->A64;
    a.r64 = pl->r64;
    a.chi2 = pl->chi2;
    a.drift = pl->drift;
    a.accA = pl->accA;
    a.accA2 = pl->accA2;
    a.counters = pl->counters;
    a.flags = pl->flags;
    a.queue = pl->queue;
    a.sweep = pl->sweep_d;
    a.seed = pl->opt.seed;
    a.lds_off_d = pl->lds_off_d;
    a.lds_off_u = pl->lds_off_u;
    a.lds_off_unif = pl->lds_off_unif;
    a.lds_off_ce = pl->lds_off_ce;
    a.kce = pl->kce;
    a.p_off_ce = pl->p_off_ce;
    a.u_lds = pl->u_lds;
    a.prefetch = pl->prefetch;
    a.p_off_vwd = pl->p_off_vwd;
    a.p_off_d = pl->p_off_d;
    a.p_off_u = pl->p_off_u;
    a.p_off_vwz = pl->p_off_vwz;
    a.p_off_und = pl->p_off_und;
    a.p_off_unz = pl->p_off_unz;
    a.p_off_h = pl->p_off_h;
    a.p_du_word = pl->p_du_word;
    a.p_wd = pl->p_wd;
    a.p_wu = pl->p_wu;
    a.p_kd = pl->p_kd;
    a.p_zs = pl->p_zs;
    a.lvl = pl->d_lvl;
    a.shape = pl->shape;
    a.hier = pl->ext() ? 1 : 0;
    a.prior = pl->any_prior ? 1 : 0;
    a.wm1f = pl->wm1f;
    return a;
}

// r = g~ - K~ A for every chain, and chi^2 = |r|^2 (optionally folding the drift)
int refresh(asm_plan *pl, bool measure_drift) {
    if (measure_drift && pl->fp32)
        HIPCHK(launch_rownorm(pl->d_probs, pl->d_chain_problem, pl->d_chain_local, pl->total_chains,
                              pl->r32, pl->r64, pl->fp32, pl->chi2_prev, nullptr, nullptr, pl->stream));
    if (pl->fp32 && pl->any_con)   // float32 chains back onto c . A = F
        HIPCHK(launch_con_fix(pl->d_probs, pl->d_chain_problem, pl->d_chain_local, pl->total_chains, pl->con,
                              pl->A32, pl->stream));
    HIPCHK(launch_refresh_all(pl->d_probs, pl->P, pl->opt.chains, pl->max_m, pl->Kt, pl->gt, pl->A32,
                              pl->r32, pl->A64, pl->r64, pl->fp32, pl->stream));
    HIPCHK(launch_rownorm(pl->d_probs, pl->d_chain_problem, pl->d_chain_local, pl->total_chains,
                          pl->r32, pl->r64, pl->fp32, pl->chi2,
                          measure_drift && pl->fp32 ? pl->chi2_prev : nullptr,
                          measure_drift && pl->fp32 ? pl->drift : nullptr, pl->stream));
    return ASM_OK;
}

// One segment of nsw sweeps starting at the device sweep counter; advances the counter.
int segment(asm_plan *pl, int64_t nsw, int accumulate, int64_t burnin_abs, bool snap) {
    SampleArgs a = make_args(pl);
    if (snap) {
        a.snapA = pl->snapA;
        a.snap_rows = pl->snap_rows;
        a.snap_first = pl->snap_first;
    }
    a.nsw = nsw;
    a.accumulate = accumulate;
    a.burnin = burnin_abs;
    a.sweeps = pl->opt.sweeps;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pl->timing) {
        while (pl->tev.size() < pl->tev_used + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            pl->tev.push_back(e);
        }
        e0 = pl->tev[pl->tev_used++];
        e1 = pl->tev[pl->tev_used++];
        HIPCHK(hipEventRecord(e0, pl->stream));
    }
    if (pl->fp32) {
        a.refresh_every = 0;
        if (pl->roles == 2)
            HIPCHK(launch_sample32p(a, pl->ept, pl->rpt, pl->grid32, pl->lds32, pl->stream));
        else if (pl->roles == 3)
            HIPCHK(launch_sample32w(a, pl->ept, pl->rpt, pl->grid32, pl->lds32, pl->stream));
        else
            HIPCHK(launch_sample32_inst(a, pl->lanes, pl->ept, pl->rpt, pl->chains_per_wg, pl->grid32,
                                    pl->lds32, pl->stream));
    } else {
        a.refresh_every = pl->opt.refresh_every;
        HIPCHK(launch_sample64_grid(a, pl->total_chains, pl->d_chain_problem, pl->d_chain_local,
                                    pl->lds64, pl->stream));
    }
    if (pl->timing) {
        HIPCHK(hipEventRecord(e1, pl->stream));
        pl->timed_sweeps += nsw;
    }
    HIPCHK(launch_bump(pl->sweep_d, nsw, pl->queue, pl->stream));
    return ASM_OK;
}

// The stream that runs the sampler: the plan's, or the private capture stream of graph mode
// when the plan's stream is the null stream.
hipStream_t main_stream(asm_plan *pl) { return pl->stream ? pl->stream : (pl->gstream ? pl->gstream : pl->stream); }

// After the sampler wrote the snapshots of nsnap sweeps: the residual coordinates of every
// snapshot state, then their cross moments with A, on the sampler's stream (beside the
// sampler, whose launches hold the register file, they only stretched its launches).
int snap_reduce(asm_plan *pl, int64_t nsnap, int64_t burnin_abs) {
    hipStream_t ms = main_stream(pl);
    HIPCHK(launch_project(pl->d_probs, pl->P, nsnap * pl->opt.chains, pl->max_mx, nsnap, pl->WY, pl->snapA,
                          pl->snapR, ms));
    HIPCHK(launch_cross_snap(pl->d_probs, pl->P, pl->max_snap_tiles, (int)pl->opt.groups, pl->parts, nsnap,
                             pl->snapA, pl->snapR, pl->snap_first, burnin_abs, pl->opt.sweeps, pl->cross, ms));
    return ASM_OK;
}

// One refresh cycle of the float32 sampler (R sweeps starting at a multiple of R): the
// sampler launch (writing the snapshots when snap), the sweep-counter bump and the
// float64 refresh.  With use_graph the sampler and bump are captured once per run and kind,
// and the refresh once per plan, as two graphs replayed one after the other (the
// sampler graph between timing events); they hold kernel launches only (no memsets, no host
// work), and every argument is the same for each cycle of the run (the kernels read the
// sweep counter from device memory).
int capture(asm_plan *pl, hipGraphExec_t *exec, const std::function<int()> &body) {
    if (!pl->stream && !pl->gstream) HIPCHK(hipStreamCreate(&pl->gstream));
    // capture on the plan's stream, or on a private stream when that is the null stream
    hipStream_t user = pl->stream;
    pl->stream = main_stream(pl);
    const bool timing = pl->timing;
    pl->timing = false;
    HIPCHK(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeRelaxed));
    const int brc = body();
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(pl->stream, &g);
    pl->timing = timing;
    pl->stream = user;
    if (brc != ASM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return brc;
    }
    HIPCHK(ee);
    const hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(ie);
    return ASM_OK;
}

int cycle(asm_plan *pl, int64_t R, int accumulate, int64_t burnin_abs, bool snap) {
    if (!pl->opt.use_graph) {
        TRY(segment(pl, R, accumulate, burnin_abs, snap));
        TRY(refresh(pl, true));
        return ASM_OK;
    }
    const int key = (accumulate ? 1 : 0) | (snap ? 2 : 0);
    if (!pl->gexec[key] || pl->gburnin[key] != burnin_abs) {
        if (pl->gexec[key]) HIPCHK(hipGraphExecDestroy(pl->gexec[key]));
        pl->gexec[key] = nullptr;
        TRY(capture(pl, &pl->gexec[key], [&]() { return segment(pl, R, accumulate, burnin_abs, snap); }));
        pl->gburnin[key] = burnin_abs;
    }
    if (!pl->gexec_refresh) TRY(capture(pl, &pl->gexec_refresh, [&]() { return refresh(pl, true); }));
    hipStream_t ms = main_stream(pl);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pl->timing) {
        while (pl->tev.size() < pl->tev_used + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            pl->tev.push_back(e);
        }
        e0 = pl->tev[pl->tev_used++];
        e1 = pl->tev[pl->tev_used++];
        HIPCHK(hipEventRecord(e0, ms));
    }
    HIPCHK(hipGraphLaunch(pl->gexec[key], ms));
    if (pl->timing) {
        HIPCHK(hipEventRecord(e1, ms));
        pl->timed_sweeps += R;
    }
    HIPCHK(hipGraphLaunch(pl->gexec_refresh, ms));
    ++pl->graph_replays;
    return ASM_OK;
}

// Run sweeps [sweep, sweep + total) with accumulation from burnin_abs on (if accumulate).
int sweep_loop(asm_plan *pl, int64_t total, int accumulate, int64_t burnin_abs) {
    const int64_t R = pl->opt.refresh_every;
    const int64_t end = pl->sweep + total;
    const bool vjp = accumulate && pl->opt.want_vjp;
    const bool snapping = vjp && pl->fp32;   // float32: the cross moments come from snapshots
    if (snapping && !pl->snapA) return fail(ASM_ESTATE, "plan has no snapshot buffers");
    while (pl->sweep < end) {
        const int64_t s = pl->sweep;
        // whole refresh cycles of the float32 sampler go through cycle() (a graph replay with
        // use_graph); they must not straddle the end of burn-in and must fit the snapshots
        if (pl->fp32 && R > 0 && s % R == 0 && s + R <= end && (s >= burnin_abs || s + R <= burnin_abs) &&
            (!(snapping && s >= burnin_abs) || pl->snap_rows >= R)) {
            const bool snap = snapping && s >= burnin_abs;
            TRY(cycle(pl, R, accumulate, burnin_abs, snap));
            if (snap) TRY(snap_reduce(pl, R, burnin_abs));
            pl->sweep += R;
            continue;
        }
        int64_t seg = end - s;
        if (pl->fp32 && R > 0) seg = std::min(seg, R - s % R);   // stop where a refresh is due
        if (!pl->fp32 && seg > 256) seg = 256;
        if (vjp && s + seg > burnin_abs && s < burnin_abs) seg = burnin_abs - s;   // burn-in apart
        // float32: as many sweeps as the snapshot rows hold; float64 with want_vjp: one sweep,
        // whose state the cross-moment kernel reads directly
        if (snapping && s >= burnin_abs) seg = std::min(seg, pl->snap_rows);
        else if (vjp && s >= burnin_abs) seg = 1;
        if (seg < 1) seg = 1;
        const bool snap = snapping && s >= burnin_abs;
        TRY(segment(pl, seg, accumulate, burnin_abs, snap));
        pl->sweep += seg;
        if (snap) {
            TRY(snap_reduce(pl, seg, burnin_abs));
        } else if (vjp && s >= burnin_abs) {
            // the sweep just sampled: its chain groups, or its batch of sweeps
            const int bgroup = pl->opt.chains < pl->opt.groups
                                   ? (int)((s - burnin_abs) * pl->opt.groups / pl->opt.sweeps) : -1;
            HIPCHK(launch_cross_all(pl->d_probs, pl->P, pl->max_cross_tiles, (int)pl->opt.groups, pl->parts, bgroup,
                                    pl->A32, pl->r32, pl->A64, pl->r64, pl->fp32, pl->cross, pl->stream));
        }
        if (pl->fp32 && R > 0 && pl->sweep % R == 0) TRY(refresh(pl, true));
    }
    return ASM_OK;
}

// The float32 sampler's configuration for a plan created with lanes_per_chain = 0: for every
// width with a compiled instance that fits the problems, the automatic configuration and its
// neighbours (half and twice the chains per workgroup, the U rows read from global memory
// instead of LDS, one role instead of two) are timed on throwaway plans (2 warm-up sweeps,
// then 24 timed sweeps on the plan's stream) and the fastest is kept, per shape of the batch
// (problem sizes, partitions, k, chains, the options fixed by the caller) for the rest of the
// process.  Every configuration samples the same chains.
struct TuneConf {
    int L = 16, cpw = 0, u_rows = 0, roles = 0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneConf> g_tune_cache;
// set while the tuner creates its throwaway plans: they only advance, so they get no
// snapshot buffers
thread_local bool t_probe_plan = false;
// The block factors and the NNLS start depend on the problems alone, not on the sampler's
// configuration, so the tuner's throwaway plans (of one batch) compute them once and copy them
// afterwards (problems without a constraint, whose factors the constraint's map rewrites)
struct ProbeShare {
    double *V64 = nullptr, *U64 = nullptr, *d64 = nullptr, *init = nullptr;
    int *has_init = nullptr;
    size_t nV = 0, nU = 0, nd = 0, nN = 0;
    std::vector<int32_t> kb;
    bool factors = false, start = false;
    ~ProbeShare() {
        for (void *q : {(void *)V64, (void *)U64, (void *)d64, (void *)init, (void *)has_init})
            if (q) (void)hipFree(q);
    }
};
thread_local ProbeShare *t_probe_share = nullptr;

int tune_sampler(const asm_problem *pr, int64_t n, const asm_options *o, void *hip_stream, TuneConf *best) {
    std::string key = std::to_string(o->chains) + ":" + std::to_string(o->refresh_every) + ":" +
                      std::to_string(o->start) + ":" + std::to_string(o->chains_per_workgroup) + ":" +
                      std::to_string(o->u_rows) + ":" + std::to_string(o->roles);
    int64_t max_nb = 0, max_m = 0;
    int hier = 0;
    for (int64_t p = 0; p < n; ++p) {
        key += "|" + std::to_string(pr[p].M) + "," + std::to_string(pr[p].N) + "," + (pr[p].cov ? "c" : "s");
        max_m = std::max(max_m, pr[p].M);
        Partition part;
        TRY(parse_partition(pr[p], p, &part));
        key += ";" + std::to_string(part.lcount.size());
        hier |= (part.lcount.size() > 1 || pr[p].prior_shape || pr[p].constraint_c) ? 1 : 0;
        for (int64_t b = 0; b < pr[p].B; ++b) {
            const int64_t nb = part.nb[b];
            max_nb = std::max(max_nb, nb);
            key += "," + std::to_string(part.n0[b]) + "+" + std::to_string(nb) + ":" +
                   std::to_string(pr[p].k ? pr[p].k[b] : -1);
        }
        key += std::string(pr[p].prior_shape ? "p" : "") + (pr[p].constraint_c ? "c" : "");
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return ASM_OK;
        }
    }
    std::vector<int> cand;
    for (int L : {4, 8, 16, 32, 64}) {
        int e, r, f;
        if (sample32_pick(L, max_nb, max_m, hier, &e, &r, &f) == 0) cand.push_back(L);
    }
    if (cand.empty()) return fail(ASM_EINVAL, "block of %lld points or %lld data points too large for the float32 sampler",
                                  (long long)max_nb, (long long)max_m);
    TuneConf chosen;
    chosen.L = cand[0];
    chosen.cpw = o->chains_per_workgroup;
    chosen.u_rows = o->u_rows;
    chosen.roles = o->roles;
    float best_ms = -1.0f;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    ProbeShare share;
    struct ShareScope {
        ~ShareScope() { t_probe_share = nullptr; }
    } share_scope;
    t_probe_share = &share;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // time one configuration; fills the configuration the plan actually took
    auto probe = [&](const TuneConf &c, TuneConf *took) -> float {
        asm_options so = *o;
        so.lanes_per_chain = c.L;
        so.chains_per_workgroup = c.cpw;
        so.u_rows = c.u_rows;
        so.roles = c.roles;
        so.want_vjp = 0;
        so.use_graph = 0;
        asm_plan *sp = nullptr;
        t_probe_plan = true;
        const int crc = asm_plan_create(pr, n, &so, hip_stream, &sp);
        t_probe_plan = false;
        if (crc != ASM_OK) return -1.0f;
        float ms = -1.0f;
        if (asm_plan_advance(sp, 2) == ASM_OK && hipEventRecord(e0, st) == hipSuccess &&
            asm_plan_advance(sp, 24) == ASM_OK && hipEventRecord(e1, st) == hipSuccess &&
            hipEventSynchronize(e1) == hipSuccess)
            (void)hipEventElapsedTime(&ms, e0, e1);
        if (took) {
            took->L = c.L;
            took->cpw = sp->chains_per_wg;
            took->u_rows = sp->u_lds ? 0 : 1;
            took->roles = sp->roles;
        }
        asm_plan_destroy(sp);
        return ms;
    };
    auto consider = [&](const TuneConf &c, float ms) {
        if (ms > 0.0f && (best_ms < 0.0f || ms < best_ms)) {
            best_ms = ms;
            chosen = c;
        }
    };
    for (int L : cand) {
        TuneConf a;
        a.L = L;
        a.cpw = o->chains_per_workgroup;
        a.u_rows = o->u_rows;
        a.roles = o->roles;
        TuneConf took;
        const float ms = probe(a, &took);
        if (ms <= 0.0f) continue;
        took.roles = a.roles == 0 ? 0 : took.roles;   // keep the automatic choice automatic
        consider(took, ms);
        if (cand.size() == 1 && o->chains_per_workgroup == 0 && o->u_rows == 0 && o->roles == 0 &&
            took.cpw <= 64 / L && took.u_rows == 1)
            break;   // nothing to vary
        std::vector<TuneConf> alt;
        if (o->roles == 0 && (took.roles == 2 || took.roles == 3)) {   // one role, automatic workgroup
            TuneConf c = a;
            c.roles = 1;
            alt.push_back(c);
        }
        if (o->chains_per_workgroup == 0) {
            for (int f : {2, 0}) {   // half and twice the automatic workgroup, one role
                const int cpw = f ? took.cpw / f : took.cpw * 2;
                if (cpw < 1 || (L * cpw) % 64 != 0 || L * cpw > 512) continue;
                TuneConf c = a;
                c.cpw = cpw;
                c.roles = o->roles == 2 ? 2 : 1;
                if (c.roles == 2 && cpw != 16) continue;
                alt.push_back(c);
            }
        }
        if (o->u_rows == 0 && took.u_rows == 0) {   // U rows from global memory
            TuneConf c = a;
            c.u_rows = 1;
            alt.push_back(c);
        }
        for (const TuneConf &c : alt) consider(c, probe(c, nullptr));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = chosen;
    *best = chosen;
    return ASM_OK;
}

}  // namespace

extern "C" {

const char *asm_last_error(void) { return g_err.c_str(); }

int asm_version(void) { return 100; }

int asm_hierarchy(int64_t N, int64_t max_block, int64_t *levels, int64_t *n_starts, int64_t *level_blocks,
                  int64_t *starts) {
    g_err.clear();
    if (!levels || !n_starts) return fail(ASM_EINVAL, "levels and n_starts are required");
    if (N < 1 || N > (1LL << 24)) return fail(ASM_EINVAL, "N must be in [1, 2^24]");
    int64_t nl = 0, ns = 0;
    // one level: its cuts (0 < c < N) in increasing order, then N
    auto emit = [&](const std::vector<int64_t> &cuts) {
        int64_t widest = 0, prev = 0;
        for (int64_t c : cuts) {
            widest = std::max(widest, c - prev);
            prev = c;
        }
        if (max_block > 0 && widest > max_block) return;
        if (level_blocks) level_blocks[nl] = (int64_t)cuts.size();
        if (starts) {
            starts[ns] = 0;
            for (size_t j = 0; j < cuts.size(); ++j) starts[ns + 1 + (int64_t)j] = cuts[j];
        }
        ns += (int64_t)cuts.size() + 1;
        ++nl;
    };
    std::vector<int64_t> cuts;
    for (int l = 0; (N >> (l + 1)) >= 1 && l < 62; ++l) {   // width N / 2^l >= 2
        const int64_t den = 1LL << (l + 1);
        const int64_t shift = (l >= 2 && l % 2 == 0) ? 1 : 0;   // every other level, by half a width
        cuts.clear();
        for (int64_t j = 0;; ++j) {
            const int64_t c = (N * (2 * j + shift)) / den;   // N <= 2^24 and 2j + 1 <= 2N + 1
            if (c >= N) break;
            if (c > 0) cuts.push_back(c);
        }
        cuts.push_back(N);
        emit(cuts);
    }
    cuts.clear();
    for (int64_t c = 1; c <= N; ++c) cuts.push_back(c);   // the single points
    emit(cuts);
    *levels = nl;
    *n_starts = ns;
    return ASM_OK;
}

int asm_plan_destroy(asm_plan *pl) {
    if (!pl) return ASM_OK;
    if (pl->gexec_refresh) (void)hipGraphExecDestroy(pl->gexec_refresh);
    for (auto &g : pl->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (pl->gstream) (void)hipStreamDestroy(pl->gstream);
    for (auto &e : pl->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : pl->tev) (void)hipEventDestroy(e);
    for (void *p : pl->allocs) (void)hipFree(p);
    delete pl;
    return ASM_OK;
}

int asm_plan_create(const asm_problem *pr, int64_t n, const asm_options *o, void *hip_stream,
                    asm_plan **out) {
    g_err.clear();
    if (!out) return fail(ASM_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(validate(pr, n, o));
    asm_options tuned;
    if (o->precision == ASM_FP32 && o->lanes_per_chain == 0) {
        TuneConf c;
        TRY(tune_sampler(pr, n, o, hip_stream, &c));
        tuned = *o;
        tuned.lanes_per_chain = c.L;
        tuned.chains_per_workgroup = c.cpw;
        tuned.u_rows = c.u_rows;
        tuned.roles = c.roles;
        o = &tuned;
    }
    asm_plan *pl = new asm_plan();
    int rc = ASM_OK;
    struct Guard {
        asm_plan *&p;
        int &rc;
        ~Guard() {
            if (rc != ASM_OK) asm_plan_destroy(p);
        }
    } guard{pl, rc};
#define STEP(expr)                 \
    do {                           \
        rc = (expr);               \
        if (rc != ASM_OK) return rc; \
    } while (0)
#define HSTEP(expr)                                                                    \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            rc = fail(ASM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));               \
            return rc;                                                                 \
        }                                                                              \
    } while (0)

    pl->stream = static_cast<hipStream_t>(hip_stream);
    HSTEP(hipGetDevice(&pl->device));
    pl->opt = *o;
    if (pl->opt.groups == 0) pl->opt.groups = 32;
    pl->P = n;
    pl->fp32 = o->precision == ASM_FP32;
    for (auto &e : pl->ev) HSTEP(hipEventCreate(&e));
    (void)set_sample32_lds_limit(160 * 1024);
    (void)allow_lds_sample32p(160 * 1024);
    (void)allow_lds_sample32w(160 * 1024);
    (void)set_sample64_lds_limit();
    (void)hipGetLastError();

    // ---- sizes and offsets ----
    int64_t offK = 0, offm = 0, offn = 0, offA = 0, offr = 0, offc = 0, offL = 0, offcross = 0;
    int64_t offV = 0, offU = 0, offd = 0, offwork = 0;
    std::vector<SvdTask> tasks;
    std::vector<int64_t> blockM;
    const int64_t C = o->chains;
    const int64_t G = pl->opt.groups;
    pl->n_prefix.push_back(0);
    pl->m_prefix.push_back(0);
    for (int64_t p = 0; p < n; ++p) {
        const asm_problem &q = pr[p];
        ProbDesc pd{};
        pd.M = q.M;
        pd.N = q.N;
        pd.B = q.B;
        pd.C = C;
        pd.off_K = offK;
        pd.off_m = offm;
        pd.off_n = offn;
        pd.off_A = offA;
        pd.off_r = offr;
        pd.off_c = offc;
        pd.off_blk = (int64_t)pl->blocks.size();
        pd.off_cross = offcross;
        pd.off_L = offL;
        pd.groups = (int32_t)G;
        pd.batches = C < G ? G : 1;
        pd.has_cov = q.cov != nullptr;
        pd.index = (uint32_t)p;
        pd.has_prior = q.prior_shape != nullptr;
        pl->any_prior |= pd.has_prior != 0;
        // a linear constraint (Sec. IV.E): its vector is read here, since it decides how many
        // modes each block has
        std::vector<double> cvec;
        if (q.constraint_c) {
            cvec.resize(q.N);
            HSTEP(hipMemcpy(cvec.data(), q.constraint_c, q.N * sizeof(double), hipMemcpyDeviceToHost));
            bool any = false;
            for (double x : cvec) {
                if (!std::isfinite(x)) { rc = fail(ASM_EDOMAIN, "problem %lld: constraint_c must be finite", (long long)p); return rc; }
                any |= x != 0.0;
            }
            if (!any || !std::isfinite(q.constraint_value)) {
                rc = fail(ASM_EINVAL, "problem %lld: constraint_c must not vanish and F must be finite", (long long)p);
                return rc;
            }
            pd.has_con = 1;
            pd.con_value = q.constraint_value;
            pl->any_con = true;
        }
        pl->any_cov |= pd.has_cov;
        Partition part;
        STEP(parse_partition(q, p, &part));
        pd.levels = (int64_t)part.lcount.size();
        pd.off_lvl = (int64_t)pl->lvl.size() / 2;
        for (size_t l = 0; l < part.lcount.size(); ++l) {
            pl->lvl.push_back(part.lfirst[l]);
            pl->lvl.push_back(part.lcount[l]);
        }
        pl->any_levels |= pd.levels > 1;
        for (int64_t b = 0; b < q.B; ++b) {
            BlockDesc bd{};
            bd.n0 = part.n0[b];
            bd.nb = part.nb[b];
            // under a constraint, a block with a non-zero share c_b has nb - 1 modes
            bool cb = false;
            for (int64_t j = 0; j < bd.nb && !cvec.empty(); ++j) cb |= cvec[bd.n0 + j] != 0.0;
            bd.nm = cb ? bd.nb - 1 : bd.nb;
            const int64_t kmax = std::min(q.M, bd.nm);
            bd.off_V = offV;
            bd.off_U = offU;
            bd.off_d = offd;
            offV += bd.nb * bd.nb;
            offU += kmax * q.M;
            offd += kmax;
            SvdTask t{};
            t.M = q.M;
            t.N = q.N;
            t.off_K = offK;
            t.n0 = bd.n0;
            t.nb = bd.nb;
            t.kreq = q.k ? q.k[b] : -1;
            t.off_V = bd.off_V;
            t.off_U = bd.off_U;
            t.off_d = bd.off_d;
            t.off_work = offwork;
            t.block = (int64_t)pl->blocks.size();
            if (cb && bd.nm > 0) {
                // decompose K~_b Q_b (M x nm, at a place in the kernel array fixed below) into
                // V' (nm x nm, in V64 after the modes); k_con_map forms V = Q_b V'
                ConTask ct{};
                ct.M = q.M;
                ct.N = q.N;
                ct.off_K = offK;
                ct.n0 = bd.n0;
                ct.nb = bd.nb;
                ct.off_c = offn + bd.n0;
                ct.off_v = pl->hv_words;
                ct.off_kq = pl->kq_words;   // relative until the kernel array's size is known
                ct.off_vp = pl->vp_words;   // relative until the mode array's size is known
                ct.off_V = bd.off_V;
                pl->hv_words += bd.nb + 1;
                t.N = bd.nm;
                t.n0 = 0;
                t.nb = bd.nm;
                t.off_K = pl->kq_words;      // relative, as above
                t.off_V = pl->vp_words;
                pl->kq_words += q.M * bd.nm;
                pl->vp_words += bd.nm * bd.nm;
                pl->ctasks.push_back(ct);
                pl->ctask_svd.push_back((int64_t)tasks.size());
            }
            offwork += svd_work_doubles(q.M, std::max<int64_t>(bd.nm, 1));
            if (bd.nm > 0) tasks.push_back(t);   // a one-point block under the constraint has no mode
            blockM.push_back(q.M);
            pl->blocks.push_back(bd);
            pl->max_nb = std::max(pl->max_nb, bd.nb);
        }
        offK += q.M * q.N;
        offm += q.M;
        offn += q.N;
        offA += C * q.N;
        offr += C * q.M;
        offc += C;
        if (pd.has_cov) offL += q.M * q.M;
        pl->max_m = std::max(pl->max_m, q.M);
        pl->max_cross_tiles = std::max(pl->max_cross_tiles, ((q.M + 31) / 32) * ((q.N + 32) / 32));
        pl->n_prefix.push_back(offn);
        pl->m_prefix.push_back(offm);
        pl->probs.push_back(pd);
    }
    pl->total_chains = offc;
    pl->total_n = offn;
    // the constrained blocks' matrices after the whitened kernels and their V' after the modes
    for (size_t j = 0; j < pl->ctasks.size(); ++j) {
        ConTask &ct = pl->ctasks[j];
        SvdTask &t = tasks[pl->ctask_svd[j]];
        ct.off_kq += offK;
        ct.off_vp += offV;
        t.off_K = ct.off_kq;
        t.off_V = ct.off_vp;
    }
    pl->total_m = offm;
    if (pl->fp32 && o->want_vjp && !t_probe_plan) {
        // the cross moments of the VJP come from per-sweep snapshots of A and the residual
        // coordinates formed from them: rows for every accumulated sweep of a launch (at most
        // refresh_every or 64 sweeps, and at most half of the free device memory), padded to
        // whole 16-byte words
        int64_t per_row = 0;
        for (auto &pd : pl->probs)
            per_row += pd.C * ((pd.N + 3) / 4 * 4 + (pd.M + 3) / 4 * 4) * (int64_t)sizeof(float);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)16 << 30;
        (void)hipGetLastError();
        const int64_t cap = (int64_t)(free_b / 2);
        const int64_t want_rows = o->refresh_every > 0 ? o->refresh_every : 64;
        pl->snap_rows = std::max<int64_t>(1, std::min<int64_t>(want_rows, cap / std::max<int64_t>(per_row, 1)));
        for (auto &pd : pl->probs) {
            pd.off_sa = pl->snap_words_a;
            pd.off_sr = pl->snap_words_r;
            pl->snap_words_a += pl->snap_rows * pd.C * ((pd.N + 3) / 4 * 4);
            pl->snap_words_r += pl->snap_rows * pd.C * ((pd.M + 3) / 4 * 4);
            pl->max_snap_tiles = std::max(pl->max_snap_tiles, cross_snap_tiles(pd.M, pd.N));
        }
    }
    if (o->want_vjp) {
        // cross moments in partial sums per (chain group, part): the groups give the VJP its
        // error bar, the parts the parallelism
        int cus = 256, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        (void)hipGetLastError();
        if (pl->fp32) {
            // (tile, split) workgroups: four fit a CU beside the sampler, about four rounds
            const int64_t want = 16LL * cus / std::max<int64_t>(1, pl->max_snap_tiles * G);
            pl->parts = (int)std::max<int64_t>(1, std::min<int64_t>(8, want));
        } else {
            // enough (tile, split) wavefronts to fill the chip, at least 8 chains per part
            const int64_t want = (2048 + pl->max_cross_tiles * G - 1) / (pl->max_cross_tiles * G);
            pl->parts = (int)std::max<int64_t>(1, std::min<int64_t>({want, 8, std::max<int64_t>(1, C / (8 * G))}));
        }
    }

    // ---- allocations ----
    double *work = nullptr, *tmpN = nullptr;
    int32_t *kb_d = nullptr;
    int64_t *blockM_d = nullptr;
    int *has_init_d = nullptr;
    SvdTask *tasks_d = nullptr;
    STEP(dalloc(pl, &pl->Kt, offK + pl->kq_words));
    STEP(dalloc(pl, &pl->gt, offm));
    STEP(dalloc(pl, &pl->sigma, offm));
    if (pl->any_cov) STEP(dalloc(pl, &pl->Lc, offL));
    STEP(dalloc(pl, &pl->V64, offV + pl->vp_words));
    STEP(dalloc(pl, &pl->U64, offU));
    STEP(dalloc(pl, &pl->d64, offd));
    STEP(dalloc(pl, &work, offwork));
    STEP(dalloc(pl, &kb_d, pl->blocks.size()));
    STEP(dalloc(pl, &blockM_d, blockM.size()));
    STEP(dalloc(pl, &tasks_d, tasks.size()));
    STEP(dalloc(pl, &tmpN, offn));
    STEP(dalloc(pl, &has_init_d, n));
    STEP(dalloc(pl, &pl->flags, 1));
    STEP(dalloc(pl, &pl->queue, 8));   // one counter per tile range
    STEP(dalloc(pl, &pl->sweep_d, 1));
    STEP(dalloc(pl, &pl->counters, 3));
    if (pl->any_prior) STEP(dalloc(pl, &pl->shape, offn));
    STEP(dalloc(pl, &pl->chi2, offc));
    STEP(dalloc(pl, &pl->chi2_prev, offc));
    STEP(dalloc(pl, &pl->drift, offc));
    STEP(dalloc(pl, &pl->d_chain_problem, offc));
    STEP(dalloc(pl, &pl->d_chain_local, offc));
    STEP(dalloc(pl, &pl->d_nprefix, n + 1));
    STEP(dalloc(pl, &pl->d_mprefix, n + 1));
    if (pl->fp32) {
        // 1024 spare floats past the last chain: the eight-lane sampler loads a block's
        // components as whole rows of its lanes (up to 127 entries past the block's end)
        STEP(dalloc(pl, &pl->A32, offA + 1024));
        STEP(dalloc(pl, &pl->r32, offr));
    } else {
        STEP(dalloc(pl, &pl->A64, offA));
        STEP(dalloc(pl, &pl->r64, offr));
    }
    if (pl->fp32 && o->want_vjp && !t_probe_plan) {
        STEP(dalloc(pl, &pl->snapA, pl->snap_words_a));
        STEP(dalloc(pl, &pl->snapR, pl->snap_words_r));
        STEP(dalloc(pl, &pl->snap_first, 1));
    }
    if (o->want_vjp) STEP(dalloc(pl, &pl->vjp_scratch, vjp_scratch_doubles(n, offm, (int)G)));
    hipStream_t st = pl->stream;
    HSTEP(hipMemsetAsync(pl->flags, 0, sizeof(int), st));
    HSTEP(hipMemsetAsync(pl->sweep_d, 0, sizeof(int64_t), st));
    HSTEP(hipMemsetAsync(pl->queue, 0, 8 * sizeof(int), st));
    HSTEP(hipMemsetAsync(pl->counters, 0, 3 * sizeof(unsigned long long), st));
    HSTEP(hipMemsetAsync(pl->drift, 0, offc * sizeof(double), st));

    // ---- input checks (device data) ----
    std::vector<int> has_init(n, 0);
    for (int64_t p = 0; p < n; ++p) {
        const asm_problem &q = pr[p];
        HSTEP(launch_check_finite(q.K, q.M * q.N, pl->flags, 1, st));
        HSTEP(launch_check_finite(q.G, q.M, pl->flags, 1, st));
        if (q.sigma) HSTEP(launch_check_positive(q.sigma, q.M, pl->flags, 2, st));
        if (q.cov) HSTEP(launch_check_finite(q.cov, q.M * q.M, pl->flags, 1, st));
        if (q.prior_shape) {
            HSTEP(launch_check_positive(q.prior_shape, q.N, pl->flags, 4, st));
            HSTEP(hipMemcpyAsync(pl->shape + pl->probs[p].off_n, q.prior_shape, q.N * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
        }
        if (q.init) {
            HSTEP(launch_check_finite(q.init, q.N, pl->flags, 1, st));
            HSTEP(hipMemcpyAsync(tmpN + pl->probs[p].off_n, q.init, q.N * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
            has_init[p] = 1;
        }
    }
    int hflags = 0;
    STEP(check_flags(pl, &hflags));
    if (hflags & 2) { rc = fail(ASM_EDOMAIN, "non-finite value in K, G, cov or init"); return rc; }
    if (hflags & 4) { rc = fail(ASM_EDOMAIN, "sigma must be positive and finite"); return rc; }
    if (hflags & 16) { rc = fail(ASM_EDOMAIN, "prior_shape must be positive and finite"); return rc; }
    if (pl->fp32 && pl->any_prior) {
        // the float32 sampler's exponents w_n - 1 (problems without a prior: 0)
        std::vector<double> w(offn, 1.0);
        for (int64_t p = 0; p < n; ++p)
            if (pr[p].prior_shape)
                HSTEP(hipMemcpy(w.data() + pl->probs[p].off_n, pr[p].prior_shape, pr[p].N * sizeof(double),
                                hipMemcpyDeviceToHost));
        std::vector<float> f(offn);
        for (int64_t i = 0; i < offn; ++i) f[i] = (float)(w[i] - 1.0);
        STEP(dalloc(pl, &pl->wm1f, offn));
        HSTEP(hipMemcpy(pl->wm1f, f.data(), offn * sizeof(float), hipMemcpyHostToDevice));
    }
    if (std::any_of(has_init.begin(), has_init.end(), [](int v) { return v; })) {
        std::vector<double> h(offn);
        HSTEP(hipMemcpy(h.data(), tmpN, offn * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < n; ++p)
            if (has_init[p])
                for (int64_t i = 0; i < pr[p].N; ++i)
                    if (h[pl->probs[p].off_n + i] < 0.0) {
                        rc = fail(ASM_EDOMAIN, "problem %lld: init must be >= 0", (long long)p);
                        return rc;
                    }
    }

    HSTEP(hipEventRecord(pl->ev[0], st));
    // ---- whitening ----
    for (int64_t p = 0; p < n; ++p) {
        const asm_problem &q = pr[p];
        const ProbDesc &pd = pl->probs[p];
        if (q.sigma) {
            HSTEP(launch_whiten_diag(q.K, q.G, q.sigma, q.M, q.N, pl->Kt + pd.off_K, pl->gt + pd.off_m, st));
            HSTEP(hipMemcpyAsync(pl->sigma + pd.off_m, q.sigma, q.M * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
        } else {
            HSTEP(launch_cholesky(q.cov, q.M, pl->Lc + pd.off_L, pl->flags, 3, st));
            HSTEP(launch_trsm_lower(pl->Lc + pd.off_L, q.M, q.K, q.N, q.N, pl->Kt + pd.off_K, st));
            HSTEP(launch_trsm_lower(pl->Lc + pd.off_L, q.M, q.G, 1, 1, pl->gt + pd.off_m, st));
        }
    }
    STEP(check_flags(pl, &hflags));
    if (hflags & 8) { rc = fail(ASM_EDOMAIN, "covariance is not symmetric positive definite"); return rc; }

    // ---- block decompositions ----
    ProbeShare *share = (t_probe_plan && !pl->any_con) ? t_probe_share : nullptr;
    const size_t nV = (size_t)(offV + pl->vp_words);
    std::vector<int32_t> kb(pl->blocks.size());
    if (share && share->factors && share->nV == nV && share->nU == (size_t)offU && share->nd == (size_t)offd &&
        share->kb.size() == kb.size()) {
        HSTEP(hipMemcpyAsync(pl->V64, share->V64, nV * sizeof(double), hipMemcpyDeviceToDevice, st));
        HSTEP(hipMemcpyAsync(pl->U64, share->U64, offU * sizeof(double), hipMemcpyDeviceToDevice, st));
        HSTEP(hipMemcpyAsync(pl->d64, share->d64, offd * sizeof(double), hipMemcpyDeviceToDevice, st));
        kb = share->kb;
    } else {
    HSTEP(hipMemsetAsync(kb_d, 0, pl->blocks.size() * sizeof(int32_t), st));   // blocks with no mode
    if (pl->any_con) {
        STEP(dalloc(pl, &pl->con, offn));
        STEP(dalloc(pl, &pl->hv, pl->hv_words));
        STEP(dalloc(pl, &pl->ctasks_d, pl->ctasks.size()));
        for (int64_t p = 0; p < n; ++p)
            if (pr[p].constraint_c)
                HSTEP(hipMemcpyAsync(pl->con + pl->probs[p].off_n, pr[p].constraint_c, pr[p].N * sizeof(double),
                                     hipMemcpyDeviceToDevice, st));
        HSTEP(hipMemcpyAsync(pl->ctasks_d, pl->ctasks.data(), pl->ctasks.size() * sizeof(ConTask),
                             hipMemcpyHostToDevice, st));
        HSTEP(launch_con_prep(pl->ctasks_d, (int64_t)pl->ctasks.size(), pl->Kt, pl->con, pl->Kt, pl->hv, st));
    }
    HSTEP(hipMemcpyAsync(tasks_d, tasks.data(), tasks.size() * sizeof(SvdTask), hipMemcpyHostToDevice, st));
    HSTEP(launch_block_svd_tasks(tasks_d, (int64_t)tasks.size(), pl->Kt, work, pl->V64, pl->U64,
                                 pl->d64, kb_d, st));
    if (pl->any_con)
        HSTEP(launch_con_map(pl->ctasks_d, (int64_t)pl->ctasks.size(), pl->hv, pl->V64, pl->V64, st));
    HSTEP(hipMemcpyAsync(kb.data(), kb_d, kb.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HSTEP(hipStreamSynchronize(st));
    if (share && !share->factors) {
        if (!share->V64) HSTEP(hipMalloc(&share->V64, nV * sizeof(double)));
        if (!share->U64) HSTEP(hipMalloc(&share->U64, std::max<int64_t>(offU, 1) * sizeof(double)));
        if (!share->d64) HSTEP(hipMalloc(&share->d64, std::max<int64_t>(offd, 1) * sizeof(double)));
        HSTEP(hipMemcpyAsync(share->V64, pl->V64, nV * sizeof(double), hipMemcpyDeviceToDevice, st));
        HSTEP(hipMemcpyAsync(share->U64, pl->U64, offU * sizeof(double), hipMemcpyDeviceToDevice, st));
        HSTEP(hipMemcpyAsync(share->d64, pl->d64, offd * sizeof(double), hipMemcpyDeviceToDevice, st));
        share->nV = nV;
        share->nU = (size_t)offU;
        share->nd = (size_t)offd;
        share->kb = kb;
        share->factors = true;
    }
    }
    for (size_t b = 0; b < kb.size(); ++b) pl->blocks[b].kb = kb[b];

    // ---- range bases and cross-moment sums (want_vjp) ----
    if (o->want_vjp) {
        if (pl->fp32) {
            // the VJP's moments of the float32 plans are taken in the coordinates of a basis of
            // range(K~), from the data modes of each problem's first partition
            constexpr int kMaxRank = 128;
            std::vector<int64_t> cfirst(1, 0), colU, colD, woff;
            int64_t wtot = 0, qtot = 0, maxm = 0;
            for (int64_t p = 0; p < n; ++p) {
                ProbDesc &pd = pl->probs[p];
                const int32_t lc = pl->lvl[2 * pd.off_lvl + 1];
                for (int32_t b = 0; b < lc; ++b) {
                    const BlockDesc &bd = pl->blocks[pd.off_blk + b];
                    for (int64_t i = 0; i < bd.kb; ++i) {
                        colU.push_back(bd.off_U + i * pd.M);
                        colD.push_back(bd.off_d + i);
                    }
                }
                const int64_t K = (int64_t)colU.size() - cfirst.back();
                cfirst.push_back((int64_t)colU.size());
                woff.push_back(wtot);
                wtot += std::max<int64_t>(1, K) * pd.M;
                pd.off_q = qtot;
                qtot += pd.M * std::min<int64_t>({pd.M, std::max<int64_t>(K, 1), (int64_t)kMaxRank});
                maxm = std::max(maxm, pd.M);
            }
            double *rwork = nullptr;
            int64_t *cf_d = nullptr, *cu_d = nullptr, *cd_d = nullptr, *wo_d = nullptr;
            int32_t *rk_d = nullptr;
            ProbDesc *pb_d = nullptr;
            STEP(dalloc(pl, &rwork, wtot));
            STEP(dalloc(pl, &pl->Qb, qtot));
            STEP(dalloc(pl, &cf_d, cfirst.size()));
            STEP(dalloc(pl, &cu_d, colU.size()));
            STEP(dalloc(pl, &cd_d, colD.size()));
            STEP(dalloc(pl, &wo_d, woff.size()));
            STEP(dalloc(pl, &rk_d, n));
            STEP(dalloc(pl, &pb_d, n));
            HSTEP(hipMemcpyAsync(pb_d, pl->probs.data(), n * sizeof(ProbDesc), hipMemcpyHostToDevice, st));
            HSTEP(hipMemcpyAsync(cf_d, cfirst.data(), cfirst.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
            if (!colU.empty()) {
                HSTEP(hipMemcpyAsync(cu_d, colU.data(), colU.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
                HSTEP(hipMemcpyAsync(cd_d, colD.data(), colD.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
            }
            HSTEP(hipMemcpyAsync(wo_d, woff.data(), woff.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
            HSTEP(launch_range_basis(pb_d, n, maxm, cf_d, cu_d, cd_d, pl->U64, pl->d64, wo_d, rwork, pl->Qb, rk_d,
                                     kMaxRank, st));
            std::vector<int32_t> rk(n);
            HSTEP(hipMemcpyAsync(rk.data(), rk_d, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            HSTEP(hipStreamSynchronize(st));
            for (int64_t p = 0; p < n; ++p) {
                pl->probs[p].rank_r = rk[p];
                pl->any_rank |= rk[p] > 0;
            }
            // the scratch of the basis is not needed again
            for (void *q : {(void *)rwork, (void *)cf_d, (void *)cu_d, (void *)cd_d, (void *)wo_d, (void *)rk_d,
                            (void *)pb_d}) {
                auto it = std::find(pl->allocs.begin(), pl->allocs.end(), q);
                if (it != pl->allocs.end()) pl->allocs.erase(it);
                HSTEP(hipFree(q));
            }
            pl->max_snap_tiles = 0;
            int64_t wy = 0, maxe = 0;
            for (auto &pd : pl->probs) {
                const int64_t Mx = pd.rank_r > 0 ? pd.rank_r : pd.M;
                pl->max_snap_tiles = std::max(pl->max_snap_tiles, cross_snap_tiles(Mx, pd.N));
                pl->max_mx = std::max(pl->max_mx, Mx);
                pd.off_w = wy;
                wy += Mx * (pd.N + 1);
                maxe = std::max(maxe, Mx * (pd.N + 1));
            }
            // the maps from a sampled state to its residual coordinates
            STEP(dalloc(pl, &pl->WY, wy));
            ProbDesc *pw_d = nullptr;
            STEP(dalloc(pl, &pw_d, n));
            HSTEP(hipMemcpyAsync(pw_d, pl->probs.data(), n * sizeof(ProbDesc), hipMemcpyHostToDevice, st));
            HSTEP(launch_resid_map(pw_d, n, maxe, pl->Kt, pl->gt, pl->Qb, pl->WY, st));
            HSTEP(hipStreamSynchronize(st));
            {
                auto it = std::find(pl->allocs.begin(), pl->allocs.end(), (void *)pw_d);
                if (it != pl->allocs.end()) pl->allocs.erase(it);
                HSTEP(hipFree(pw_d));
            }
        }
        int64_t offx = 0;
        for (auto &pd : pl->probs) {
            pd.off_cross = offx;
            offx += (int64_t)G * pl->parts * (pd.rank_r > 0 ? pd.rank_r : pd.M) * (pd.N + 1);
        }
        pl->cross_words = offx;
        STEP(dalloc(pl, &pl->cross, offx));
    }

    // ---- chain -> problem tables ----
    {
        std::vector<int32_t> cp(offc), cl(offc);
        for (int64_t p = 0; p < n; ++p)
            for (int64_t c = 0; c < C; ++c) {
                cp[pl->probs[p].off_c + c] = (int32_t)p;
                cl[pl->probs[p].off_c + c] = (int32_t)c;
            }
        HSTEP(hipMemcpyAsync(pl->d_chain_problem, cp.data(), offc * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HSTEP(hipMemcpyAsync(pl->d_chain_local, cl.data(), offc * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HSTEP(hipMemcpyAsync(pl->d_nprefix, pl->n_prefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HSTEP(hipMemcpyAsync(pl->d_mprefix, pl->m_prefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HSTEP(hipStreamSynchronize(st));
    }

    // ---- sampler configuration ----
    int max_cu = 256;
    {
        int dev = 0;
        HSTEP(hipGetDevice(&dev));
        HSTEP(hipDeviceGetAttribute(&max_cu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    if (pl->fp32) {
        int L = o->lanes_per_chain;
        if (o->roles == 3) {
            // the eight-lane sampler (sample32w.h)
            if (L != 0 && L != 8) {
                rc = fail(ASM_EINVAL, "roles 3 (the eight-lane sampler) needs lanes_per_chain 8 or 0");
                return rc;
            }
            L = 8;
        }
        if (L == 0) {
            // aim for about one wavefront per SIMD (4 per CU) across all chains
            const double chains_per_simd = (double)pl->total_chains / (4.0 * max_cu);
            const double want = 64.0 / std::max(1.0, chains_per_simd);
            L = want >= 48 ? 64 : want >= 24 ? 32 : want >= 12 ? 16 : want >= 6 ? 8 : 4;
        }
        int ept = 0, rpt = 0, pf = 0;
        {
            // the requested width first, then wider ones, then narrower ones
            const int order[] = {L, 16, 32, 8, 4, 64};
            bool found = false;
            for (int cand : order) {
                if ((o->lanes_per_chain != 0 || o->roles == 3) && cand != L) continue;
                if (sample32_pick(cand, pl->max_nb, pl->max_m, pl->ext() ? 1 : 0, &ept, &rpt, &pf) == 0) {
                    L = cand;
                    found = true;
                    break;
                }
            }
            if (!found) {
                rc = fail(ASM_EINVAL, "block of %lld points or %lld data points too large for the float32 sampler",
                          (long long)pl->max_nb, (long long)pl->max_m);
                return rc;
            }
        }
        // the eight-lane sampler (sample32w.h): asked for with roles 3, or taken in automatic
        // mode for eight lanes per chain with the automatic workgroup and U rows in LDS, when
        // one of its instances holds the sizes and its staging area fits the LDS with 64 chains
        bool wide = false;
        {
            int64_t mkb = 0;
            for (auto &bd : pl->blocks) mkb = std::max(mkb, bd.kb);
            int we = 0, wr = 0;
            bool ok = L == 8 && !pl->ext() && (o->roles == 0 || o->roles == 3) &&
                      (o->chains_per_workgroup == 0 || o->chains_per_workgroup == 64) && o->u_rows == 0 &&
                      sample32w_pick(pl->max_nb, pl->max_m, mkb, &we, &wr) == 0;
            if (ok) {
                const size_t need = (size_t)(pl->max_nb + 2) * we * 8 * sizeof(float2) + (size_t)(mkb + 3) / 4 * 16 +
                                    (size_t)mkb * wr * 8 * sizeof(float) +
                                    (size_t)64 * std::max<int64_t>(mkb, 1) * sizeof(float);
                ok = need <= kLdsBudget;
            }
            if (ok) {
                wide = true;
                ept = we;
                rpt = wr;
                pf = 0;
            } else if (o->roles == 3) {
                rc = fail(ASM_EINVAL, "roles 3 (the eight-lane sampler) needs one partition per problem with no prior "
                                      "or constraint, blocks of at most 128 points with at most 32 data modes, at most "
                                      "416 data points, 64 chains per workgroup, U rows in LDS, and its staging area "
                                      "within the LDS");
                return rc;
            }
        }
        pl->lanes = L;
        pl->ept = ept;
        pl->rpt = rpt;
        pl->pf = pf;
        const int64_t row = (int64_t)ept * L;   // components per staged row
        const int64_t mp = (int64_t)rpt * L;
        pl->max_nbp = row;
        int64_t offU32 = 0;
        for (auto &bd : pl->blocks) {
            bd.nbp = row;
            bd.mp = mp;
            bd.off_U32 = offU32;
            offU32 += std::max<int64_t>(bd.kb, 1) * mp;   // mp is a multiple of 4
        }
        STEP(dalloc(pl, &pl->U32, offU32));
        // LDS of a workgroup: the staging area (the block's (V, w) rows with two spare rows
        // for the rows loaded ahead, its singular values, and its U rows when they fit) and
        // one uniform row per chain.  Each block's packed chunk is the image of the staging
        // area.
        int64_t max_kb = 0, max_n = 0;
        for (auto &bd : pl->blocks) max_kb = std::max(max_kb, bd.kb);
        for (auto &pd : pl->probs) max_n = std::max(max_n, pd.N);
        pl->max_kb = max_kb;
        pl->max_n = max_n;
        // centre/step rows: two halves of kce floats per chain; the eight-lane sampler keeps
        // one slot per data mode (the step overwrites the centre)
        pl->kce = wide ? (int32_t)std::max<int64_t>(1, max_kb) : (int32_t)std::max<int64_t>(4, (max_kb + 3) / 4 * 4);
        const size_t vw_bytes = (size_t)(pl->max_nb + 2) * row * sizeof(float2);
        const size_t d_bytes = (size_t)(max_kb + 3) / 4 * 16;
        const size_t u_bytes = (size_t)max_kb * mp * sizeof(float);
        auto layout = [&](int cpw, bool with_u) {
            size_t off = vw_bytes;
            pl->lds_off_d = (int64_t)off;
            off += d_bytes;
            pl->lds_off_u = (int64_t)off;
            if (with_u) off += u_bytes;
            off = (off + 15) / 16 * 16;
            pl->lds_off_unif = (int64_t)off;
            if (!wide)   // the eight-lane sampler holds its uniforms in registers
                off += (size_t)cpw * row * sizeof(float) * (pl->any_prior ? 2 : 1);   // prior: acceptance rows
            pl->lds_off_ce = (int64_t)off;
            off += (size_t)cpw * (wide ? 1 : 2) * pl->kce * sizeof(float);
            return off;
        };
        // chains per workgroup: enough workgroups for every CU, at most 512 threads (256 for
        // the prefetching instances, compiled for one wavefront per SIMD)
        int cpw = (pf > 0 ? 256 : 512) / L;
        if (wide) {
            cpw = 64;
        } else if (o->chains_per_workgroup > 0) {
            cpw = o->chains_per_workgroup;
            if ((L * cpw) % 64 != 0 || L * cpw > (pf > 0 ? 256 : 512)) {
                rc = fail(ASM_EINVAL, "chains_per_workgroup %d with %d lanes per chain: the threads must be a multiple "
                                      "of 64 and at most %d", cpw, L, pf > 0 ? 256 : 512);
                return rc;
            }
        } else {
            while (cpw > 64 / L) {
                const int64_t wgs = (pl->total_chains + cpw - 1) / cpw;
                if (layout(cpw, false) <= kLdsBudget && wgs >= max_cu) break;
                cpw /= 2;
            }
        }
        pl->chains_per_wg = cpw;
        pl->u_lds = (wide || (o->u_rows == 0 && layout(cpw, true) <= kLdsBudget)) ? 1 : 0;
        pl->lds32 = layout(cpw, pl->u_lds);
        if (pl->lds32 > kLdsBudget) {
            rc = fail(ASM_EINVAL, "block factors need %zu bytes of LDS (limit 160 KB)", pl->lds32);
            return rc;
        }
        // the packed chunks (one per block, the image of the staging area)
        pl->chunk.rows = pl->max_nb + 2;
        pl->chunk.row = row;
        pl->chunk.d_len = (max_kb + 3) / 4 * 4;
        pl->chunk.u_rows = pl->u_lds ? max_kb : 0;
        pl->chunk.mp = mp;
        pl->chunk.words = (int64_t)(vw_bytes + d_bytes + (pl->u_lds ? u_bytes : 0)) / 16;
        pl->chunk.compact = pl->ext() ? 1 : 0;   // the extended instances stage packed chunks
        int64_t f32_words = 0;
        if (!pl->chunk.compact) {
            for (size_t k = 0; k < pl->blocks.size(); ++k) pl->blocks[k].off_chunk = (int64_t)k * pl->chunk.words;
            f32_words = (int64_t)pl->blocks.size() * pl->chunk.words;
        } else {
            // each block's image packed to its size (nm + 2 rows, round4(kb) values, kb U rows),
            // the blocks back to back, so that consecutive blocks of a level are one copy
            std::vector<int64_t> words(pl->blocks.size());
            for (size_t k = 0; k < pl->blocks.size(); ++k) {
                const BlockDesc &bd = pl->blocks[k];
                words[k] = ((bd.nm + 2) * row * 8 + (bd.kb + 3) / 4 * 16 + (pl->u_lds ? bd.kb * mp * 4 : 0)) / 16;
                pl->blocks[k].off_chunk = f32_words;
                f32_words += words[k];
            }
            // groups: consecutive blocks of one level whose images fit the staging area together
            // and whose uniforms (four per Philox call) fit one uniform row, staged and drawn at
            // once (many small blocks share one pair of barriers)
            const int64_t cap = pl->lds_off_unif / 16;
            for (auto &pd : pl->probs) {
                for (int64_t l = 0; l < pd.levels; ++l) {
                    const int64_t f = pd.off_blk + pl->lvl[2 * (pd.off_lvl + l)];
                    const int64_t c = pl->lvl[2 * (pd.off_lvl + l) + 1];
                    int64_t k = f;
                    while (k < f + c) {
                        int64_t n = 0, w = 0, u = 0;
                        while (k + n < f + c) {
                            const int64_t wn = words[k + n], un = (pl->blocks[k + n].nm + 3) / 4 * 4;
                            if (n > 0 && (w + wn > cap || u + un > row)) break;
                            w += wn;
                            u += un;
                            ++n;
                        }
                        pl->blocks[k].grp_n = (int32_t)n;
                        pl->blocks[k].grp_words = (int32_t)w;
                        for (int64_t j = 1; j < n; ++j) pl->blocks[k + j].grp_n = pl->blocks[k + j].grp_words = 0;
                        k += n;
                    }
                }
            }
        }
        STEP(dalloc(pl, &pl->F32, f32_words));
        // the next block's chunk is prefetched into registers when it fits the instance's
        // per-thread budget (not with a hierarchy, whose blocks are staged to their own size)
        pl->prefetch = (pf > 0 && L * cpw <= 256 && pl->chunk.words <= (int64_t)pf * L * cpw && !pl->ext()) ? 1 : 0;
        // two roles (data modes of the next block beside the zero modes of this one) when the
        // instance, the partitions (two blocks or more) and the staging areas allow it
        {
            int pe = 0, pr = 0, pfr = 0, pfu = 0, pfz = 0;
            // (in automatic mode only with enough chains for a 16-chain workgroup per CU)
            bool ok = o->roles != 1 && L == 16 && (o->chains_per_workgroup == 0 || o->chains_per_workgroup == 16) &&
                      (o->roles == 2 || pl->total_chains >= 16LL * max_cu) &&
                      sample32p_pick(pl->max_nb, pl->max_m, pl->u_lds, &pe, &pr, &pfr, &pfu, &pfz) == 0 &&
                      pe == ept && pr == rpt;
            // one partition of two blocks or more, no prior, no constraint (the two roles run
            // every mode of a block, and the zero role's rows are those of an unconstrained block)
            for (auto &pd : pl->probs) ok = ok && pd.B >= 2 && pd.levels == 1 && !pd.has_prior && !pd.has_con;
            const int64_t rw = row / 2;   // 16-byte words per (V, w) row
            // zero modes the data role runs per block, balancing the two roles: a data move
            // costs about kDataOverZero zero moves at 201 data points and blocks of 100 points,
            // scaled by the ratio of the algorithmic counts (2 M + 3 N_b + 40 against 3 N_b + 10)
            // where that ratio is larger
            const double kDataOverZero = pl->u_lds ? 2.6 : 3.0;
            const double kRatio201 = (2.0 * 201 + 3.0 * 100 + 40.0) / (3.0 * 100 + 10.0);
            double zsum = 0.0;
            for (auto &bd : pl->blocks) {
                const double ratio = (2.0 * (double)pl->max_m + 3.0 * (double)bd.nb + 40.0) / (3.0 * (double)bd.nb + 10.0);
                const double dz = kDataOverZero * std::max(1.0, ratio / kRatio201);
                zsum += 0.5 * ((double)(bd.nb - bd.kb) - dz * (double)bd.kb);
            }
            int64_t zs = (int64_t)std::lround(zsum / std::max<size_t>(1, pl->blocks.size()));
            // the data role's rows (0..max k + zs + 1) must fit its prefetch registers
            zs = std::max<int64_t>(0, std::min<int64_t>(zs, 256LL * pfr / rw - 2 - max_kb));
            int64_t zrows = 0, ke_max = 0;
            for (auto &bd : pl->blocks) {
                const int64_t ke = std::min(bd.kb + zs, bd.nb);
                ke_max = std::max(ke_max, ke);
                zrows = std::max(zrows, bd.nb + 2 - ke);
            }
            const int64_t wd = (ke_max + 2) * rw, wu = (pl->chunk.d_len + (pl->u_lds ? max_kb * mp : 0)) / 4;
            ok = ok && wd <= 256LL * pfr && wu <= 256LL * pfu && zrows * rw <= 256LL * pfz;
            size_t off = 0;
            auto take = [&](size_t bytes) {
                const size_t at = off;
                off = (off + bytes + 15) / 16 * 16;
                return (int64_t)at;
            };
            pl->p_off_vwd = take((size_t)wd * 16);
            pl->p_off_d = take((size_t)wu * 16);
            pl->p_off_u = pl->p_off_d + pl->chunk.d_len * (int64_t)sizeof(float);
            pl->p_off_vwz = take((size_t)zrows * rw * 16);
            pl->p_kd = (int32_t)((ke_max + 3) / 4 * 4);
            pl->p_off_und = take((size_t)16 * pl->p_kd * sizeof(float));
            pl->p_off_unz = take((size_t)16 * row * sizeof(float));
            pl->p_off_h = take((size_t)16 * row * sizeof(float));
            pl->p_off_ce = take((size_t)16 * 2 * pl->kce * sizeof(float));
            ok = ok && off <= kLdsBudget;
            if (ok) {
                pl->roles = 2;
                pl->chains_per_wg = 256 / L;   // the two-role kernel's workgroup: 16 chains
                pl->lds32 = off;
                pl->p_wd = (int32_t)wd;
                pl->p_wu = (int32_t)wu;
                pl->p_du_word = pl->chunk.rows * rw;
                pl->p_zs = (int32_t)zs;
            } else if (o->roles == 2) {
                rc = fail(ASM_EINVAL, "two roles need 16 lanes per chain, a two-role instance for the sizes, two "
                                      "blocks or more per problem, no hierarchy, prior or constraint, and the "
                                      "staging areas in LDS");
                return rc;
            }
        }
        if (wide) pl->roles = 3;
        build_tiles(pl);
        pl->grid32 = (int)std::min<int64_t>((int64_t)pl->tiles.size(), (int64_t)max_cu * 2);
        STEP(dalloc(pl, &pl->d_tiles, pl->tiles.size()));
        HSTEP(hipMemcpyAsync(pl->d_tiles, pl->tiles.data(), pl->tiles.size() * sizeof(TileDesc),
                             hipMemcpyHostToDevice, st));
    } else {
        int64_t maxlds = 0;
        for (auto &pd : pl->probs) maxlds = std::max(maxlds, (pd.N + pd.M) * (int64_t)sizeof(double));
        if (maxlds > (int64_t)kLdsBudget) {
            rc = fail(ASM_EINVAL, "float64 sampler holds N + M doubles in LDS: at most 20480");
            return rc;
        }
        pl->lds64 = (size_t)maxlds;
        pl->lanes = 64;
        pl->chains_per_wg = 1;
        build_chain_slots(pl);
    }
    finish_slot_counts(pl);
    int64_t slot_elems = 0;
    for (auto &pd : pl->probs) {
        pd.off_slot = slot_elems;
        slot_elems += pd.nslot * pd.N;
    }
    STEP(dalloc(pl, &pl->accA, slot_elems));
    STEP(dalloc(pl, &pl->accA2, slot_elems));
    STEP(dalloc(pl, &pl->slot_group_d, pl->slot_group.size()));
    STEP(dalloc(pl, &pl->slot_count_d, pl->slot_count.size()));
    HSTEP(hipMemcpyAsync(pl->slot_group_d, pl->slot_group.data(), pl->slot_group.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HSTEP(hipMemcpyAsync(pl->slot_count_d, pl->slot_count.data(), pl->slot_count.size() * sizeof(double), hipMemcpyHostToDevice, st));

    // ---- device tables ----
    STEP(dalloc(pl, &pl->d_probs, pl->probs.size()));
    STEP(dalloc(pl, &pl->d_blocks, pl->blocks.size()));
    STEP(dalloc(pl, &pl->d_lvl, pl->lvl.size()));
    HSTEP(hipMemcpyAsync(pl->d_lvl, pl->lvl.data(), pl->lvl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HSTEP(hipMemcpyAsync(pl->d_probs, pl->probs.data(), pl->probs.size() * sizeof(ProbDesc), hipMemcpyHostToDevice, st));
    HSTEP(hipMemcpyAsync(pl->d_blocks, pl->blocks.data(), pl->blocks.size() * sizeof(BlockDesc), hipMemcpyHostToDevice, st));
    HSTEP(hipMemcpyAsync(blockM_d, blockM.data(), blockM.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HSTEP(hipMemcpyAsync(has_init_d, has_init.data(), n * sizeof(int), hipMemcpyHostToDevice, st));

    // ---- start from the non-negative least-squares fit where asked ----
    if ((o->start == ASM_START_NNLS || o->start == ASM_START_NNLS_NOISED) && share && share->start &&
        share->nN == (size_t)offn) {
        HSTEP(hipMemcpyAsync(tmpN, share->init, offn * sizeof(double), hipMemcpyDeviceToDevice, st));
        HSTEP(hipMemcpyAsync(has_init_d, share->has_init, n * sizeof(int), hipMemcpyDeviceToDevice, st));
    } else if (o->start == ASM_START_NNLS || o->start == ASM_START_NNLS_NOISED) {
        std::vector<int> use(n, 0);
        std::vector<int64_t> woff(n, 0);
        int64_t wtot = 0;
        for (int64_t p = 0; p < n; ++p) {
            use[p] = has_init[p] ? 0 : 1;
            woff[p] = wtot;
            if (use[p]) wtot += nnls_work_doubles(pr[p].M, pr[p].N);
        }
        if (wtot > 0) {
            double *nw = nullptr;
            int *use_d = nullptr;
            int64_t *woff_d = nullptr;
            STEP(dalloc(pl, &nw, wtot));
            STEP(dalloc(pl, &use_d, n));
            STEP(dalloc(pl, &woff_d, n));
            HSTEP(hipMemcpyAsync(use_d, use.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
            HSTEP(hipMemcpyAsync(woff_d, woff.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, st));
            const double *g = pl->gt;
            if (o->start == ASM_START_NNLS_NOISED) {
                double *gn = nullptr;
                STEP(dalloc(pl, &gn, offm));
                HSTEP(launch_noise_data(pl->d_probs, n, pl->gt, gn, o->seed, st));
                g = gn;
            }
            HSTEP(launch_nnls(pl->d_probs, n, use_d, pl->Kt, g, nw, woff_d, 0.01, tmpN,
                              has_init_d, st));
        }
        if (share && !share->start) {
            if (!share->init) HSTEP(hipMalloc(&share->init, std::max<int64_t>(offn, 1) * sizeof(double)));
            if (!share->has_init) HSTEP(hipMalloc(&share->has_init, std::max<int64_t>(n, 1) * sizeof(int)));
            HSTEP(hipMemcpyAsync(share->init, tmpN, offn * sizeof(double), hipMemcpyDeviceToDevice, st));
            HSTEP(hipMemcpyAsync(share->has_init, has_init_d, n * sizeof(int), hipMemcpyDeviceToDevice, st));
            share->nN = (size_t)offn;
            share->start = true;
        }
    }

    // ---- float32 packing, start state, first residual ----
    if (pl->fp32)
        HSTEP(launch_pack32_blocks(pl->d_blocks, blockM_d, (int64_t)pl->blocks.size(), pl->V64,
                                   pl->U64, pl->d64, pl->chunk, pl->F32, pl->U32, pl->flags, st));
    HSTEP(launch_init_state2(pl->d_probs, n, o->chains, pl->Kt, pl->gt, tmpN, has_init_d, pl->A64, pl->A32,
                             pl->fp32, st));
    if (pl->any_con) {
        std::vector<int32_t> which;
        for (int64_t p = 0; p < n; ++p)
            if (pl->probs[p].has_con) which.push_back((int32_t)p);
        int32_t *which_d = nullptr;
        STEP(dalloc(pl, &which_d, which.size()));
        HSTEP(hipMemcpyAsync(which_d, which.data(), which.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HSTEP(launch_con_start(pl->d_probs, which_d, (int64_t)which.size(), pl->con, pl->A64, pl->A32, pl->fp32,
                               pl->flags, 5, st));
        STEP(check_flags(pl, &hflags));
        if (hflags & 32) {
            rc = fail(ASM_EDOMAIN, "the start moved onto the constraint has a negative component: pass an init");
            return rc;
        }
    }
    STEP(refresh(pl, false));
    HSTEP(hipEventRecord(pl->ev[1], st));
    HSTEP(hipStreamSynchronize(st));
    if (pl->fp32) {
        // the float32 sampler relies on every zero mode having a finite interval
        STEP(check_flags(pl, &hflags));
        pl->unbounded = (hflags & 1) != 0;
    }
    *out = pl;
    return ASM_OK;
#undef STEP
#undef HSTEP
}

int asm_plan_advance(asm_plan *pl, int64_t sweeps) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (sweeps < 0) return fail(ASM_EINVAL, "sweeps must be >= 0");
    if (sweeps == 0) return ASM_OK;
    if (pl->unbounded) return fail(ASM_EUNBOUNDED, "a zero mode has an unbounded interval: improper posterior");
    TRY(sweep_loop(pl, sweeps, 0, 0));
    int hflags = 0;
    TRY(check_flags(pl, &hflags));
    if (hflags & 1) return fail(ASM_EUNBOUNDED, "a zero mode has an unbounded interval: improper posterior");
    return ASM_OK;
}

int asm_plan_run(asm_plan *pl, double *mean, double *stderr_, double *post_sd, asm_stats *stats) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (!mean || !stderr_) return fail(ASM_EINVAL, "mean and stderr_ are required");
    if (pl->unbounded) return fail(ASM_EUNBOUNDED, "a zero mode has an unbounded interval: improper posterior");
    hipStream_t st = pl->stream;
    const int64_t slot_elems = pl->probs.back().off_slot + pl->probs.back().nslot * pl->probs.back().N;
    HIPCHK(hipMemsetAsync(pl->accA, 0, slot_elems * sizeof(double), st));
    HIPCHK(hipMemsetAsync(pl->accA2, 0, slot_elems * sizeof(double), st));
    HIPCHK(hipMemsetAsync(pl->counters, 0, 3 * sizeof(unsigned long long), st));
    if (pl->opt.want_vjp) HIPCHK(hipMemsetAsync(pl->cross, 0, pl->cross_words * sizeof(double), st));
    HIPCHK(hipEventRecord(pl->ev[2], st));
    const int64_t run_first = pl->sweep;
    const int64_t burnin_abs = pl->sweep + pl->opt.burnin;
    pl->timing = true;
    pl->tev_used = 0;
    pl->timed_sweeps = 0;
    pl->graph_replays = 0;
    int lrc = sweep_loop(pl, pl->opt.burnin + pl->opt.sweeps, 1, burnin_abs);
    pl->timing = false;
    TRY(lrc);
    HIPCHK(hipEventRecord(pl->ev[3], st));
    HIPCHK(launch_finalize(pl->d_probs, pl->P, pl->d_nprefix, pl->total_n, pl->accA, pl->accA2,
                           pl->slot_group_d, pl->slot_count_d, mean, stderr_, post_sd, nullptr, st));
    int hflags = 0;
    TRY(check_flags(pl, &hflags));
    pl->ran = true;
    if (stats) {
        memset(stats, 0, sizeof *stats);
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, pl->ev[0], pl->ev[1]));
        stats->setup_ms = ms;
        HIPCHK(hipEventElapsedTime(&ms, pl->ev[2], pl->ev[3]));
        stats->sample_ms = ms;
        double mm = 0, dm = 0;
        const int64_t nsw = pl->opt.burnin + pl->opt.sweeps;
        for (auto &pd : pl->probs) {
            // modes per sweep of each level (N per level, fewer under a constraint)
            double nm_sum = 0.0;
            for (int64_t l = 0; l < pd.levels; ++l) {
                const int32_t f = pl->lvl[2 * (pd.off_lvl + l)], c = pl->lvl[2 * (pd.off_lvl + l) + 1];
                for (int32_t b = f; b < f + c; ++b) nm_sum += (double)pl->blocks[pd.off_blk + b].nm;
            }
            mm += (double)pd.C * (double)nsw * nm_sum / (double)pd.levels;
            // data modes per sweep of each level, and the levels the run's sweeps sampled
            std::vector<double> kbl(pd.levels, 0.0);
            for (int64_t l = 0; l < pd.levels; ++l) {
                const int32_t f = pl->lvl[2 * (pd.off_lvl + l)], c = pl->lvl[2 * (pd.off_lvl + l) + 1];
                for (int32_t b = f; b < f + c; ++b) kbl[l] += (double)pl->blocks[pd.off_blk + b].kb;
            }
            if (pd.levels == 1) {
                dm += (double)pd.C * (double)nsw * kbl[0];
            } else {
                for (int64_t s = run_first; s < run_first + nsw; ++s)
                    dm += (double)pd.C * kbl[sweep_level(pl->opt.seed, pd.index, (uint32_t)s, (uint32_t)pd.levels)];
            }
        }
        stats->mode_moves = mm;
        stats->data_moves = dm;
        std::vector<double> dr(pl->total_chains);
        HIPCHK(hipMemcpy(dr.data(), pl->drift, dr.size() * sizeof(double), hipMemcpyDeviceToHost));
        stats->chi2_drift_max = dr.empty() ? 0.0 : *std::max_element(dr.begin(), dr.end());
        unsigned long long cnt[3];
        HIPCHK(hipMemcpy(cnt, pl->counters, sizeof cnt, hipMemcpyDeviceToHost));
        stats->clamped = (int64_t)cnt[0];
        stats->frozen = (int64_t)cnt[1];
        stats->rejected = (int64_t)cnt[2];
        stats->lanes_per_chain = pl->lanes;
        stats->chains_per_block = pl->chains_per_wg;
        double smp = 0.0;
        for (size_t i = 0; i + 1 < pl->tev_used; i += 2) {
            float t = 0;
            HIPCHK(hipEventElapsedTime(&t, pl->tev[i], pl->tev[i + 1]));
            smp += t;
        }
        stats->sampler_ms = smp;
        stats->sampler_launches = (int64_t)(pl->tev_used / 2);
        stats->sampler_sweeps = pl->timed_sweeps;
        stats->graph_replays = pl->graph_replays;
        stats->roles = pl->roles;
    }
    if (hflags & 1) return fail(ASM_EUNBOUNDED, "a zero mode has an unbounded interval: improper posterior");
    return ASM_OK;
}

int asm_plan_vjp(asm_plan *pl, const double *v, double *grad_G, double *grad_se) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (!pl->opt.want_vjp) return fail(ASM_ESTATE, "plan was created without want_vjp");
    if (!pl->ran) return fail(ASM_ESTATE, "asm_plan_run must come before asm_plan_vjp");
    if (!v || !grad_G) return fail(ASM_EINVAL, "v and grad_G are required");
    hipStream_t st = pl->stream;
    HIPCHK(launch_vjp(pl->d_probs, pl->P, pl->d_mprefix, pl->total_m, pl->max_m, (int)pl->opt.groups, pl->parts,
                      pl->cross, pl->accA, pl->slot_group_d, pl->slot_count_d, pl->Qb, pl->sigma, pl->Lc, v,
                      pl->vjp_scratch, grad_G, grad_se, st));
    HIPCHK(hipStreamSynchronize(st));
    return ASM_OK;
}

// ---- the VJP without allocation ----
// The intermediate products of the VJP (per-group moment rows, centred moments, their images
// under -T^T) live in this file-scope array instead of the plan's own buffer, for callers
// that may not allocate.  Each device holds its own copy; host code reaches it only through
// the address hipGetSymbolAddress returns on that device.  Every kernel of the VJP writes the
// scratch entries it later reads, so nothing needs clearing between calls.
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 23;   // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
int noalloc_scratch(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(ASM_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ASM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return ASM_OK;
}

}  // namespace

int asm_plan_vjp_noalloc(asm_plan *pl, const double *v, double *grad_G, double *grad_se) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (!pl->opt.want_vjp) return fail(ASM_ESTATE, "plan was created without want_vjp");
    if (!pl->ran) return fail(ASM_ESTATE, "asm_plan_run must come before asm_plan_vjp_noalloc");
    if (!v || !grad_G) return fail(ASM_EINVAL, "v and grad_G are required");
    const int64_t need = vjp_scratch_doubles(pl->P, pl->total_m, (int)pl->opt.groups);
    if (need > kNoAllocScratchDoubles)
        return fail(ASM_EINVAL,
                    "the VJP needs %lld scratch doubles ((4 groups + 2) x sum M + 2 problems x groups), more "
                    "than the %lld of asm_plan_vjp_noalloc; use asm_plan_vjp",
                    (long long)need, (long long)kNoAllocScratchDoubles);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != pl->device)
        return fail(ASM_EINVAL, "device %d is current, the plan lives on device %d", dev, pl->device);
    double *ws = nullptr;
    TRY(noalloc_scratch(dev, &ws));
    HIPCHK(launch_vjp(pl->d_probs, pl->P, pl->d_mprefix, pl->total_m, pl->max_m, (int)pl->opt.groups, pl->parts,
                      pl->cross, pl->accA, pl->slot_group_d, pl->slot_count_d, pl->Qb, pl->sigma, pl->Lc, v, ws,
                      grad_G, grad_se, pl->stream));
    return ASM_OK;
}

int asm_plan_group_means(asm_plan *pl, double *mean, double *stderr_, double *group_means) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (!pl->ran) return fail(ASM_ESTATE, "asm_plan_run must come before asm_plan_group_means");
    if (!mean || !stderr_ || !group_means) return fail(ASM_EINVAL, "mean, stderr_ and group_means are required");
    HIPCHK(launch_finalize(pl->d_probs, pl->P, pl->d_nprefix, pl->total_n, pl->accA, pl->accA2, pl->slot_group_d,
                           pl->slot_count_d, mean, stderr_, nullptr, group_means, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    return ASM_OK;
}

int asm_plan_state(asm_plan *pl, int64_t problem, double *A, double *r, double *chi2) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (problem < 0 || problem >= pl->P) return fail(ASM_EINVAL, "problem index out of range");
    if (pl->fp32) {
        // the float32 sampler carries no running chi^2: report |r|^2 of the carried residual
        HIPCHK(launch_rownorm(pl->d_probs, pl->d_chain_problem, pl->d_chain_local, pl->total_chains,
                              pl->r32, pl->r64, 1, pl->chi2_prev, nullptr, nullptr, pl->stream));
    }
    HIPCHK(launch_state64(pl->d_probs, problem, pl->probs[problem], pl->A32, pl->r32, pl->A64,
                          pl->r64, pl->fp32 ? pl->chi2_prev : pl->chi2, pl->fp32, A, r, chi2,
                          pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    return ASM_OK;
}

int asm_plan_factors(asm_plan *pl, int64_t problem, int64_t block, int32_t *kb, double *d,
                     double *U, double *V) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (problem < 0 || problem >= pl->P) return fail(ASM_EINVAL, "problem index out of range");
    const ProbDesc &pd = pl->probs[problem];
    if (block < 0 || block >= pd.B) return fail(ASM_EINVAL, "block index out of range");
    const BlockDesc &bd = pl->blocks[pd.off_blk + block];
    if (kb) *kb = (int32_t)bd.kb;
    hipStream_t st = pl->stream;
    if (d && bd.kb) HIPCHK(hipMemcpyAsync(d, pl->d64 + bd.off_d, bd.kb * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (U && bd.kb) {
        // stored mode-major (kb x M); returned M x kb
        std::vector<double> h(bd.kb * pd.M), t(bd.kb * pd.M);
        HIPCHK(hipMemcpyAsync(h.data(), pl->U64 + bd.off_U, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t i = 0; i < bd.kb; ++i)
            for (int64_t m = 0; m < pd.M; ++m) t[m * bd.kb + i] = h[i * pd.M + m];
        HIPCHK(hipMemcpyAsync(U, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (V) {
        std::vector<double> h(bd.nb * bd.nb), t(bd.nb * bd.nb);
        HIPCHK(hipMemcpyAsync(h.data(), pl->V64 + bd.off_V, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t i = 0; i < bd.nb; ++i)   // a block under a constraint has nm < nb modes
            for (int64_t q = 0; q < bd.nb; ++q) t[q * bd.nb + i] = i < bd.nm ? h[i * bd.nb + q] : 0.0;
        HIPCHK(hipMemcpyAsync(V, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return ASM_OK;
}

int asm_plan_whitened(asm_plan *pl, int64_t problem, double *Kt, double *gt) {
    g_err.clear();
    if (!pl) return fail(ASM_EINVAL, "plan is NULL");
    if (problem < 0 || problem >= pl->P) return fail(ASM_EINVAL, "problem index out of range");
    const ProbDesc &pd = pl->probs[problem];
    if (Kt) HIPCHK(hipMemcpyAsync(Kt, pl->Kt + pd.off_K, pd.M * pd.N * sizeof(double), hipMemcpyDeviceToDevice, pl->stream));
    if (gt) HIPCHK(hipMemcpyAsync(gt, pl->gt + pd.off_m, pd.M * sizeof(double), hipMemcpyDeviceToDevice, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    return ASM_OK;
}

int asm_tn_draw(const double *c, const double *d, const double *lo, const double *hi,
                const double *u, double *out, int64_t n, int32_t precision, void *hip_stream) {
    g_err.clear();
    if (n < 0 || (n > 0 && (!c || !d || !lo || !hi || !u || !out)))
        return fail(ASM_EINVAL, "bad arguments");
    if (precision != ASM_FP64 && precision != ASM_FP32) return fail(ASM_EINVAL, "bad precision");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIPCHK(launch_tn_draw(c, d, lo, hi, u, out, n, precision, st));
    HIPCHK(hipStreamSynchronize(st));
    return ASM_OK;
}

int asm_uniforms(uint64_t seed, int64_t problem, int64_t chain, int64_t sweep0, int64_t nsweeps,
                 int64_t nblocks, int64_t nmodes, double *out, void *hip_stream) {
    g_err.clear();
    if (!out || nsweeps < 0 || nblocks < 0 || nmodes < 0 || nblocks > 65535 || nmodes > 65535)
        return fail(ASM_EINVAL, "bad arguments");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIPCHK(launch_uniforms(seed, problem, chain, sweep0, nsweeps, nblocks, nmodes, out, st));
    HIPCHK(hipStreamSynchronize(st));
    return ASM_OK;
}

}  // extern "C"
