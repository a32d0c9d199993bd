"""Benchmark of the blocked-modes sampler on one MI355X.

One step is one pass of the whole hot path over one synthetic continuation problem, by
default the large workload (beta = 50, 401 imaginary times with exponentially correlated
noise, whitened by its Cholesky factor, 4000 Lorentzian grid points in 32 blocks of 125 with
up to 30 data modes, sigma = 1e-4, 16384 chains, 1000 burn-in and 5000 measured sweeps,
float32 chain state, refresh cycles replayed from a hipGraph):
    whitening -> float64 block SVDs -> float32 packing -> NNLS start -> sweeps with float64
    residual refreshes every 64 sweeps -> float64 accumulation of <A> (and of the moments of
    Cov(r~, A)) -> error bars -> VJP d<A>/dG v, with its error bar, for a seeded cotangent v.
The problem arrays are on the GPU before the timed region starts.

Prints one JSON line (see the fields below).  Only one GPU is supported.

    python bench.py [--steps K] [--warmup W] [--no-vjp] [--no-cpu]
    python bench.py --workload single     # beta = 20, 201 points, 800 grid points, 4096 chains
    python bench.py --workload batched    # 256 uneven continuations in one launch
    python bench.py --copy-probe          # a plain 1 GiB device copy, to calibrate HBM counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 float32 lanes x 2.4 GHz, one operation per lane per cycle (no packed
# float32 arithmetic; a fused multiply-add counts as one operation)
PEAK_LANE_OPS = 256 * 64 * 2.4e9
SAMPLER_SOURCES = ["sample32.h", "sample32_l16.hip", "sample32p.h", "sample32p_l16.hip", "sample32w.h", "sample32w_l8.hip",
                   "tn32.h", "tn32_coef.h",
                   "rng_tn.h", "internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "{kernel}_{workload}.md")
WORKLOAD_FILE_NAMES = {"large": "large", "single": "single_continuation"}


def lane_ops_per_sweep(M, blocks, s_tn=40, s_u=10):
    """Algorithmic lane-operations of one chain-sweep.

    A move of a block with nb grid points costs 3 operations per component (the ratio that
    bounds the step, its min/max into the interval, the update of A); a data move adds 2 per
    data point (c = U_i . r and the update of r) and s_tn for the truncated-normal draw, a
    zero move s_u for the flat draw.
    """
    ops = 0
    for nb, kb in blocks:
        ops += kb * (2 * M + 3 * nb + s_tn) + (nb - kb) * (3 * nb + s_u)
    return ops


def sampler_source_hash():
    h = hashlib.sha256()
    for name in SAMPLER_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_01379_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per sampler launch from the committed counter summary of that kernel on that
    workload, if it was taken on the current sampler sources (else None)."""
    try:
        with open(TRAFFIC_FILE.format(kernel=kernel, workload=WORKLOAD_FILE_NAMES.get(workload, workload))) as f:
            for line in f:
                line = line.strip()
                if line.startswith("{") and '"sources"' in line:
                    rec = json.loads(line)
                    if rec.get("sources") == sampler_source_hash():
                        return rec
    except OSError:
        pass
    return None


class _DevProblem:
    def __init__(self, p, device):
        import torch
        self.K = torch.as_tensor(p.K, dtype=torch.float64, device=device)
        self.G = torch.as_tensor(p.G, dtype=torch.float64, device=device)
        self.sigma = None if p.sigma is None else torch.as_tensor(p.sigma, dtype=torch.float64, device=device)
        self.cov = None if p.cov is None else torch.as_tensor(p.cov, dtype=torch.float64, device=device)
        self.block_start = p.block_start
        self.levels = getattr(p, "levels", None)
        self.prior_shape = getattr(p, "prior_shape", None)
        self.constraint_c = getattr(p, "constraint_c", None)
        self.constraint_value = getattr(p, "constraint_value", 0.0)
        self.k = p.k
        self.init = None


def cpu_baseline(prob, seconds_target=20.0):
    """The CPU oracle on the host cores, on a bounded sample of the same workload."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = max(1, min(threads, os.cpu_count() or 1, 64))
    prep = oracle.prepare(prob)
    chains = 4 * threads
    # calibrate on a short run, then size the sample to about seconds_target
    t = time.time()
    oracle.run(prep, chains=threads, burnin=0, sweeps=20, threads=threads, groups=1)
    dt = max(time.time() - t, 1e-3)
    sec_per_sweep = dt / 20.0 * (chains / threads)   # seconds per sweep of all sample chains
    sweeps = int(max(20, min(5000, seconds_target / sec_per_sweep)))
    t = time.time()
    oracle.run(prep, chains=chains, burnin=0, sweeps=sweeps, threads=threads, groups=4)
    dt = time.time() - t
    moves = chains * sweeps * prob.N
    return {"value": moves / dt, "unit": "mode-moves/s", "cores": threads, "kind": "oracle",
            "chain_sweeps_per_s": chains * sweeps / dt,
            "sample": f"{chains} chains x {sweeps} sweeps of the same problem from the flat start "
                      f"({moves:.3g} moves, {dt:.1f} s, float64)"}


def copy_probe():
    """A plain device copy of 1 GiB, three times: the FETCH_SIZE / WRITE_SIZE counters of
    this kernel calibrate the counters of the sampler."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 4 * n, "repeats": 3}))


def micro():
    """On-chip rates of one MI355X: float32 fused multiply-adds per second, and LDS read
    bytes per second for 4-, 8- and 16-byte reads per lane, each word read by one lane or by
    the four 16-lane groups of a wavefront (the samplers' pattern)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1912_01379_amd", "libasm_micro.so"))
    lib.micro_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.zeros(64 * cus, dtype=torch.float32, device="cuda:0")
    ms = ctypes.c_double()
    out = {"cus": cus}

    def run(kind, iters, grid, share=1):
        rc = lib.micro_run(kind, iters, grid, share, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"micro_run({kind}) failed: {rc}")
        return ms.value * 1e-3

    for wpc in (4, 8, 16):   # 256-thread workgroups: 4 waves each
        grid = cus * wpc // 4
        iters = 20000
        t = run(0, iters, grid)
        out[f"valu_fma_per_s_{wpc}waves_per_cu"] = grid * 256 * iters * 16 / t
    for kind, width in ((1, 4), (2, 8), (3, 16)):
        for share in (1, 4):
            grid = cus * 2   # two workgroups of 64 KiB per CU, 8 waves
            iters = 4000
            t = run(kind, iters, grid, share)
            out[f"lds_read_b{8 * width}_share{share}_bytes_per_s"] = grid * 256 * iters * 8 * width / t
    lib.micro_run2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p]

    def run2(kind, iters, grid, src=None, dst=None):
        rc = lib.micro_run2(kind, iters, grid, src, dst, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"micro_run2({kind}) failed: {rc}")
        return ms.value * 1e-3

    grid = cus * 4
    t = run2(4, 10000, grid)
    out["valu_fp64_fma_per_s_16waves_per_cu"] = grid * 256 * 10000 * 16 / t
    t = run2(5, 20000, grid)
    out["mfma_f64_flop_per_s"] = grid * 4 * 20000 * 8 * 2048 / t
    n = (1 << 30) // 16   # 1 GiB of float4 words
    src = torch.ones(4 * n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    t = run2(6, n, cus * 8, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()))
    out["hbm_copy_bytes_per_s"] = 2 * 16 * n / t   # read + write
    del src, dst
    out["lds_bytes_per_clk_per_cu_at_2.4GHz"] = {k: v / (cus * 2.4e9) for k, v in out.items() if k.startswith("lds")}
    out["valu_lane_ops_per_clk_per_cu_at_2.4GHz"] = out["valu_fma_per_s_8waves_per_cu"] / (cus * 2.4e9)
    print(json.dumps({"micro": out}))


def batched(args):
    """The batched workload: 256 continuations of uneven size (M in [51, 201], N in
    [200, 1000], B = round(N / 100) blocks, k = min(20, N_b)), 256 chains each, in one
    persistent launch per refresh cycle, replayed from a hipGraph; lanes per chain tuned."""
    import torch
    import workloads
    import paper_1912_01379_amd as pk
    dev = torch.device("cuda:0")
    probs = workloads.batched_datasets(256)
    dps = [_DevProblem(p, dev) for p in probs]
    chains = 256
    sweeps_total = args.burnin + args.sweeps

    def step():
        plan = pk.Plan(dps, chains=chains, burnin=args.burnin, sweeps=args.sweeps, seed=2025,
                       precision="fp32", refresh_every=64, want_vjp=False, groups=32,
                       lanes_per_chain=args.lanes, use_graph=True, start="nnls", device=dev)
        res = plan.run()
        torch.cuda.synchronize()
        # algorithmic lane-operations of one sweep of every chain of the batch
        ops = 0.0
        for j, p in enumerate(probs):
            blocks = []
            for b in range(len(p.block_start) - 1):
                nb = int(p.block_start[b + 1] - p.block_start[b])
                blocks.append((nb, plan.factors(j, b, nb)[0]))
            ops += chains * lane_ops_per_sweep(p.M, blocks)
        plan.close()
        return res, ops

    for w in range(args.warmup):
        step()
        print(f"warmup step {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res, ops_sweep = step()
        print(f"step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = res.stats
    moves = chains * sweeps_total * sum(p.N for p in probs)
    avg_launch_s = st["sampler_ms"] * 1e-3 / max(1, st["sampler_launches"])
    ops_per_launch = ops_sweep * st["sampler_sweeps"] / max(1, st["sampler_launches"])
    kernel = {2: "k_sample32p", 3: "k_sample32w"}.get(st.get("roles", 1), "k_sample32")
    out = {"metric": "mode-moves/s", "value": moves * args.steps / elapsed, "unit": "mode-moves/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batched: 256 continuations, M in [51,201], N in [200,1000], "
                                  "B = round(N/100), k <= 20, 256 chains each, fp32, NNLS start, hipGraph",
                      "chains_total": chains * len(probs), "burnin": args.burnin, "sweeps": args.sweeps,
                      "lanes_per_chain": st["lanes_per_chain"], "chains_per_workgroup": st["chains_per_block"],
                      "roles": st.get("roles", 1), "graph_replays": st["graph_replays"]},
           "roofline": {"bound": "alu", "achieved": ops_per_launch / avg_launch_s, "peak": PEAK_LANE_OPS,
                        "unit": "lane-op/s", "frac": ops_per_launch / avg_launch_s / PEAK_LANE_OPS,
                        "traffic": None, "kernel": kernel, "ops_per_chain_sweep_batch": ops_sweep,
                        "avg_launch_ms": avg_launch_s * 1e3, "launches_per_step": st["sampler_launches"]},
           "setup_ms": st["setup_ms"], "sample_ms": st["sample_ms"]}
    print(json.dumps(out))


def conductivity(args):
    """The paper's own test case (optical conductivity, bosonic kernel, Sec. III) on both grids
    of Fig. 3 (40 and 120 points) with components, modes, blocked modes on one partition of
    4 blocks, and blocked modes on the hierarchy of Fig. 2 (a random level per sweep):
    mode-moves/s, ESS/s and the median step size Delta_i of Fig. 3.  Then Fig. 7 (Sec. V.C):
    the flat prior of a grid of spacing 0.2 (60 points) simulated on the 120-point grid with
    gamma shapes 1/2, and the 120-point grid simulated on the 60-point one with shapes 2,
    compared through the averages over each pair of fine intervals."""
    import torch
    import workloads
    import paper_1912_01379_amd as pk
    dev = torch.device("cuda:0")
    rows, means = {}, {}
    cases = [(f"N{n}_{name}", n, nb, 0.1, name == "hierarchy", None)
             for n in (40, 120)
             for name, nb in (("components", n), ("modes", 1), ("blocked4", 4), ("hierarchy", 1))]
    cases += [("N60s2_blocked4", 60, 4, 0.2, False, None), ("N120_prior60", 120, 4, 0.1, False, 0.5),
              ("N60s2_prior120", 60, 4, 0.2, False, 2.0), ("N60s2_noise120", 60, 4, 0.2, False, "noise"),
              ("N120_hierarchy_sumrule", 120, 1, 0.1, True, "sumrule")]
    for key, n, nb, step, hier, shape in cases:
        if args.cases and key not in args.cases.split(","):
            continue
        p = workloads.optical_conductivity(n, nb, step=step)
        if hier:
            p.levels = pk.hierarchy(n)
        if shape == "sumrule":
            # Sec. IV.E: the sum rule sum_n w_n sigma_n = (pi / 2) Pi(0) imposed exactly
            p.constraint_c = np.asarray(p.weights, np.float64)
            p.constraint_value = math.pi / 2.0 * float(p.G[0])
        elif shape == "noise":
            # Sec. V.C's cheap variant: the data variance scaled by 120 / 60 instead of the shapes
            p.sigma = p.sigma * math.sqrt(120 / 60)
        elif shape is not None:
            p.prior_shape = np.full(n, shape)
        dp = _DevProblem(p, dev)
        plan = pk.Plan([dp], chains=args.chains, burnin=args.burnin, sweeps=args.sweeps, seed=2026,
                       precision="fp32", refresh_every=64, groups=32, lanes_per_chain=args.lanes,
                       start="nnls", use_graph=False, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the sampler's lane-operations per chain-sweep, averaged over the levels (uniform)
        parts = p.levels if p.levels is not None else [p.block_start]
        ops, blk = [], 0
        for cuts in parts:
            lv = []
            for b in range(len(cuts) - 1):
                nb = int(cuts[b + 1] - cuts[b])
                lv.append((nb, plan.factors(0, blk, nb)[0]))
                blk += 1
            ops.append(lane_ops_per_sweep(p.M, lv))
        st = res.stats
        us_sweep = 1e3 * st["sampler_ms"] / max(1, st["sampler_sweeps"])
        frac = float(np.mean(ops)) * args.chains / (us_sweep * 1e-6) / PEAK_LANE_OPS
        se, sd = res.stderr.cpu().numpy(), res.post_sd.cpu().numpy()
        ess = (sd / se) ** 2
        prev = plan.state(0)[0].cpu().numpy()
        steps = []
        for _ in range(50):
            plan.advance(1)
            cur = plan.state(0)[0].cpu().numpy()
            steps.append(np.linalg.norm(cur - prev, axis=1) / np.linalg.norm(prev, axis=1))
            prev = cur
        plan.close()
        means[key] = (res.mean.cpu().numpy(), se)
        rows[key] = {
            "mode_moves_per_s": args.chains * (args.burnin + args.sweeps) * n / dt,
            "rejected_frac": res.stats["rejected"] / max(1.0, res.stats["mode_moves"]),
            "ess_per_s_min": float(np.nanmin(ess)) / dt, "ess_per_s_median": float(np.nanmedian(ess)) / dt,
            "median_step": float(np.median(np.concatenate(steps))),
            "sampler_us_per_sweep": us_sweep, "alu_frac": frac,
            "lanes_per_chain": res.stats["lanes_per_chain"], "roles": res.stats["roles"]}
        print(f"{key} done", file=sys.stderr, flush=True)

    # Fig. 7: relative L2 distance of the averages, fine grids compared through the average of
    # each pair of fine intervals (the coarse interval they make up)
    pair = lambda m: m.reshape(-1, 2).mean(axis=1)
    rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
    fig7 = {}
    if all(k in means for k in ("N120_prior60", "N60s2_blocked4", "N120_blocked4")):
        fig7["coarse_flat_simulated_on_fine"] = {
            "rel_l2_to_coarse_flat": rel(pair(means["N120_prior60"][0]), means["N60s2_blocked4"][0]),
            "fine_flat_rel_l2_to_coarse_flat": rel(pair(means["N120_blocked4"][0]), means["N60s2_blocked4"][0])}
    if all(k in means for k in ("N60s2_prior120", "N60s2_blocked4", "N120_blocked4")):
        fig7["fine_flat_simulated_on_coarse"] = {
            "rel_l2_to_fine_flat": rel(means["N60s2_prior120"][0], pair(means["N120_blocked4"][0])),
            "coarse_flat_rel_l2_to_fine_flat": rel(means["N60s2_blocked4"][0], pair(means["N120_blocked4"][0]))}
    if all(k in means for k in ("N60s2_noise120", "N120_blocked4")):
        fig7["fine_flat_by_noise_scaling_on_coarse"] = {
            "rel_l2_to_fine_flat": rel(means["N60s2_noise120"][0], pair(means["N120_blocked4"][0]))}
    if all(k in means for k in ("N120_hierarchy_sumrule", "N120_hierarchy")):
        # Sec. IV.E: the sum rule is strongly represented in the data
        fig7["sum_rule_imposed_rel_l2_to_free"] = rel(means["N120_hierarchy_sumrule"][0], means["N120_hierarchy"][0])
    main_row = rows.get("N120_hierarchy", next(iter(rows.values())))
    print(json.dumps({"metric": "mode-moves/s", "value": main_row["mode_moves_per_s"], "unit": "mode-moves/s",
                      "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "optical conductivity (Sec. III): 60 bosonic Matsubara points, "
                                             "beta 15, relative noise 1e-3, grids of 40 and 120 points; value: "
                                             "120 points, Fig. 2 hierarchy",
                                 "chains": args.chains, "burnin": args.burnin, "sweeps": args.sweeps},
                      "cases": rows, "fig7": fig7}))


def fig6_grid_dependence(dev, chains=4096, burnin=2000, sweeps=10000, lanes=16):
    """Sec. V.B, Fig. 6: the model-2 test case on 64-point grids (uniform with spacing 0.125,
    cutoff 8; Gaussian alpha = 4, exponential beta = 3, Lorentzian gamma = 2.5) at relative
    noise 1e-3 and 1e-2, with the Fig. 2 hierarchy.  Reported per grid: the w-weighted relative
    L2 distance of the average to the exact sigma; per pair of non-uniform grids: their
    averages interpolated to 120 frequencies in [0.05, 6], the largest |difference| / combined
    error bar, the fraction of frequencies beyond 3 error bars and the relative L2 difference.
    Also the width dependence (Gaussian alpha = 3 against 5) beside the cutoff dependence
    (uniform spacing 0.125 against 0.25, cutoffs 8 and 16) at noise 1e-3."""
    import paper_1912_01379_amd as pk
    import workloads
    from paper_1912_01379_amd import grids
    wc = np.linspace(0.05, 6.0, 120)

    def average(srel, fam, par, step=0.125):
        g = None if fam == "uniform" else grids.grid(fam, par, 64)
        p = workloads.optical_conductivity(64, 1, model=2, sigma_rel=srel, step=step, grid=g)
        p.levels = pk.hierarchy(64, max_block=128)
        plan = pk.Plan([_DevProblem(p, dev)], chains=chains, burnin=burnin, sweeps=sweeps, seed=2029,
                       precision="fp32", refresh_every=64, groups=32, lanes_per_chain=lanes, start="nnls",
                       device=dev)
        r = plan.run()
        m, se = r.mean.cpu().numpy(), r.stderr.cpu().numpy()
        plan.close()
        ex = p.A_true
        d = math.sqrt(np.sum(p.weights * (m - ex) ** 2) / np.sum(p.weights * ex ** 2))
        return p.omega, m, se, d

    def pair(r1, r2):
        a, b = np.interp(wc, r1[0], r1[1]), np.interp(wc, r2[0], r2[1])
        z = np.abs(a - b) / np.hypot(np.interp(wc, r1[0], r1[2]), np.interp(wc, r2[0], r2[2]))
        return {"max_z": float(z.max()), "frac_beyond_3": float(np.mean(z > 3.0)),
                "rel_l2": float(math.sqrt(np.sum((a - b) ** 2) / np.sum((0.5 * (a + b)) ** 2)))}

    out = {}
    fams = (("uniform", 0.0), ("gaussian", 4.0), ("exponential", 3.0), ("lorentzian", 2.5))
    for srel in (1e-3, 1e-2):
        res = {f: average(srel, f, par) for f, par in fams}
        out[f"noise{srel:g}"] = {
            "rel_l2_to_exact": {f: res[f][3] for f, _ in fams},
            "pairs": {f"{f1}-{f2}": pair(res[f1], res[f2])
                      for i, (f1, _) in enumerate(fams[1:]) for f2, _ in fams[i + 2:]}}
    out["width_vs_cutoff"] = {"gaussian3-gaussian5": pair(average(1e-3, "gaussian", 3.0), average(1e-3, "gaussian", 5.0)),
                              "uniform0.125-uniform0.25": pair(average(1e-3, "uniform", 0.0),
                                                               average(1e-3, "uniform", 0.0, step=0.25))}
    return out


def grid_study(args):
    """Sec. V-VI on the model-2 test case (Figs. 4, 6, 8, 9, 10): the mean chi^2 / M of the
    sampled spectra on uniform grids of step 0.1 with growing cutoff, and on Lorentzian
    (width 2.5) and Gaussian (width 2.4) grids of growing N, with the Fig. 2 hierarchy (blocks
    up to 128 points); and the default-model fit of Fig. 9 for each grid family."""
    import torch
    import workloads
    import paper_1912_01379_amd as pk
    from paper_1912_01379_amd import grids
    dev = torch.device("cuda:0")
    rows = {}
    cases = [("uniform_cutoff%g" % (0.1 * n), n, None) for n in (40, 80, 120, 240)]
    cases += [("lorentzian2.5_N%d" % n, n, ("lorentzian", 2.5)) for n in (32, 64, 128, 256, 512)]
    cases += [("gaussian2.4_N%d" % n, n, ("gaussian", 2.4)) for n in (32, 64, 128, 256, 512)]
    t_all = time.perf_counter()
    moves = 0.0
    for key, n, fam in cases:
        g = None if fam is None else grids.grid(fam[0], fam[1], n)
        p = workloads.optical_conductivity(n, 1, model=2, grid=g)
        p.levels = pk.hierarchy(n, max_block=128)
        dp = _DevProblem(p, dev)
        plan = pk.Plan([dp], chains=args.chains, burnin=args.burnin, sweeps=args.sweeps, seed=2027,
                       precision="fp32", refresh_every=64, groups=32, lanes_per_chain=args.lanes,
                       start="nnls", device=dev)
        res = plan.run()
        chi2 = plan.state(0)[2].cpu().numpy() / len(p.G)
        moves += res.stats["mode_moves"]
        rows[key] = {"N": n, "chi2_over_M_mean": float(np.mean(chi2)), "chi2_over_M_p90": float(np.percentile(chi2, 90)),
                     "sample_ms": res.stats["sample_ms"]}
        plan.close()
        print(f"{key} done", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t_all
    p = workloads.optical_conductivity(40, 1, model=2)
    wm = 2.0 * np.pi * np.arange(len(p.G)) / 15.0
    fit = {}
    for fam, b in (("gaussian", (0.5, 10.0)), ("exponential", (0.3, 10.0)), ("lorentzian", (0.1, 10.0)),
                   ("uniform", (1.0, 20.0))):
        par, sse = grids.fit_default_model(fam, p.G, wm, b)
        fit[fam] = {"best_parameter": par, "sse": sse}
    print(json.dumps({"metric": "mode-moves/s", "value": moves / dt, "unit": "mode-moves/s", "n_gpus": 1,
                      "steps": 1, "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "grid study (Secs. V-VI): optical conductivity model 2, uniform, "
                                             "Lorentzian and Gaussian grids, Fig. 2 hierarchy",
                                 "chains": args.chains, "burnin": args.burnin, "sweeps": args.sweeps},
                      "cases": rows, "fig9_default_model_fit": fit,
                      "fig6_grid_dependence": fig6_grid_dependence(dev, args.chains, args.burnin, args.sweeps,
                                                                   args.lanes or 16)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=None)
    ap.add_argument("--burnin", type=int, default=None)
    ap.add_argument("--chains", type=int, default=None)
    ap.add_argument("--no-vjp", action="store_true")
    ap.add_argument("--no-overhead", action="store_true",
                    help="skip the untimed forward without the VJP's moments")
    ap.add_argument("--no-split", action="store_true", help="skip the untimed split-half equilibration check")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--micro", action="store_true", help="on-chip VALU and LDS rates")
    ap.add_argument("--workload", choices=["large", "single", "batched", "conductivity", "grids"],
                    default="large")
    ap.add_argument("--graph", action="store_true", help="replay refresh cycles from a hipGraph")
    ap.add_argument("--cases", default="", help="conductivity workload: comma list such as N120_hierarchy")
    ap.add_argument("--hierarchy", action="store_true",
                    help="single-continuation workload on the Fig. 2 hierarchy instead of its 8 blocks")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; use --gpus 1"}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.micro:
        micro()
        return
    if args.workload not in ONE_PROBLEM:
        # the other workloads' defaults
        args.burnin = 2000 if args.burnin is None else args.burnin
        args.sweeps = args.sweeps or 10000
        args.chains = args.chains or 4096
    if args.workload == "batched":
        batched(args)
        return
    if args.workload == "conductivity":
        conductivity(args)
        return
    if args.workload == "grids":
        grid_study(args)
        return

    one_problem(args)


# the two one-problem workloads: chains, burn-in, measured sweeps, and whether cycles replay
# from a hipGraph by default
ONE_PROBLEM = {
    "large": dict(chains=16384, burnin=1000, sweeps=5000, graph=True),
    "single": dict(chains=4096, burnin=2000, sweeps=10000, graph=False),
}


def one_problem(args):
    """One continuation problem per step: the large workload (beta = 50, 401 correlated data
    points whitened by their Cholesky factor, 4000 grid points in 32 blocks of 125 with up to 30
    data modes, 16384 chains) or the single-continuation workload (beta = 20, 201 points, 800
    grid points in 8 blocks of 100 with up to 20 data modes, 4096 chains); forward and VJP."""
    import torch
    import workloads
    import paper_1912_01379_amd as pk

    dev = torch.device("cuda:0")
    d = ONE_PROBLEM[args.workload]
    chains = args.chains or d["chains"]
    burnin = d["burnin"] if args.burnin is None else args.burnin
    sweeps = args.sweeps or d["sweeps"]
    use_graph = d["graph"] or args.graph
    if args.workload == "large":
        prob = workloads.large_workload()
        label = ("large: beta=50, M=401 correlated (length 5) whitened by Cholesky, N=4000 Lorentzian grid, "
                 "32 blocks x 125, k<=30, sigma=1e-4, fp32 chains, NNLS start")
    else:
        prob = workloads.single_continuation()
        label = ("single continuation: beta=20, M=201, N=800 Lorentzian grid, "
                 + ("Fig. 2 hierarchy of 7 levels (8 to 800 blocks)" if args.hierarchy else "8 blocks x 100")
                 + ", k<=20, sigma=1e-4, fp32 chains, NNLS start")
        if args.hierarchy:
            # the Fig. 2 hierarchy of the 800-point grid, levels of blocks up to 128 points (the
            # float32 instances' largest block): 8 blocks of 100 down to the single points
            prob.levels = pk.hierarchy(prob.N, max_block=128)
            prob.k = np.full(prob.B, 20, np.int32)
    v = torch.as_tensor(workloads.differentiation_cotangent(prob.N), dtype=torch.float64, device=dev)
    dp = _DevProblem(prob, dev)
    want_vjp = not args.no_vjp

    def step(vjp=want_vjp):
        plan = pk.Plan([dp], chains=chains, burnin=burnin, sweeps=sweeps, seed=2024,
                       precision="fp32", refresh_every=64, want_vjp=vjp, groups=32,
                       lanes_per_chain=args.lanes, start="nnls", use_graph=use_graph, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = plan.vjp(v, stderr=True) if vjp else None
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        blocks, blk = [], 0   # per level: (N_b, k_b) of its blocks
        for cuts in prob.partitions():
            lv = []
            for b in range(len(cuts) - 1):
                nb = int(cuts[b + 1] - cuts[b])
                lv.append((nb, plan.factors(0, blk, nb)[0]))
                blk += 1
            blocks.append(lv)
        plan.close()
        return res, (t1 - t0), (t2 - t1), blocks, g

    for w in range(args.warmup):
        step()
        print(f"warmup step {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    outs = []
    for k in range(args.steps):
        outs.append(step())
        print(f"step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    res, fwd_s, vjp_s, blocks, g = outs[-1]
    st = res.stats
    sweeps_total = burnin + sweeps
    moves_per_step = chains * sweeps_total * prob.N
    # levels are drawn uniformly: per-sweep counts averaged over the levels
    data_per_step = chains * sweeps_total * float(np.mean([sum(k for _, k in lv) for lv in blocks]))
    value = moves_per_step * args.steps / elapsed
    step_s = elapsed / args.steps
    # roofline of the sampler kernel from its own launch events
    ops_sweep = float(np.mean([lane_ops_per_sweep(prob.M, lv) for lv in blocks]))
    avg_launch_s = st["sampler_ms"] * 1e-3 / max(1, st["sampler_launches"])
    ops_per_launch = ops_sweep * chains * st["sampler_sweeps"] / max(1, st["sampler_launches"])
    achieved = ops_per_launch / avg_launch_s
    kernel = {2: "k_sample32p", 3: "k_sample32w"}.get(st.get("roles", 1), "k_sample32")
    tr = measured_traffic(kernel, args.workload)
    se = res.stderr.cpu().numpy()
    sd = res.post_sd.cpu().numpy()
    ess = (sd / se) ** 2
    tau = chains * sweeps / ess
    # the forward alone (untimed): what accumulating the VJP's moments costs the forward
    fwd_novjp_s = None
    if want_vjp and not args.no_overhead:
        fwd_novjp_s = step(vjp=False)[1]
        print("forward without the VJP's moments done", file=sys.stderr, flush=True)

    # equilibration (untimed): the same chains' averages over the first and the second half of
    # the measured sweeps, z = |<A>_1 - <A>_2| / sqrt(se_1^2 + se_2^2) per grid point; a drift
    # of the chains between the halves (a burn-in too short for the slowest points) shows as
    # z well above the few units of chance
    split = None
    if not args.no_split:
        plan = pk.Plan([dp], chains=chains, burnin=0, sweeps=sweeps // 2, seed=2025, precision="fp32",
                       refresh_every=64, want_vjp=False, groups=32, lanes_per_chain=args.lanes, start="nnls",
                       use_graph=use_graph, device=dev)
        plan.advance(burnin)
        h1 = plan.run()
        m1, s1 = h1.mean.cpu().numpy(), h1.stderr.cpu().numpy()
        h2 = plan.run()
        m2, s2 = h2.mean.cpu().numpy(), h2.stderr.cpu().numpy()
        plan.close()
        z = np.abs(m1 - m2) / np.sqrt(s1 ** 2 + s2 ** 2)
        ok = np.isfinite(z)
        slow = np.argsort(np.where(np.isfinite(tau), tau, -1.0))[::-1][:10]
        split = {"burnin": burnin, "sweeps_per_half": sweeps // 2, "max_z": float(np.max(z[ok])),
                 "frac_z_above_3": float(np.mean(z[ok] > 3.0)), "median_z": float(np.median(z[ok])),
                 "z_at_10_slowest_points": [round(float(z[i]), 2) for i in slow],
                 "tau_int_at_10_slowest_points": [round(float(tau[i]), 1) for i in slow]}
        print("split-half equilibration check done", file=sys.stderr, flush=True)

    # the plain sampler: float64, one chain per launch
    plain = pk.Plan([dp], chains=1, burnin=0, sweeps=20, seed=7, precision="fp64", groups=1,
                    device=dev)
    pres = plain.run()
    plain.close()
    plain_rate = pres.stats["mode_moves"] / (pres.stats["sample_ms"] * 1e-3)

    out = {
        "metric": "mode-moves/s",
        "value": value,
        "unit": "mode-moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": label, "chains": chains, "burnin": burnin, "sweeps": sweeps,
                   "vjp": want_vjp, "hipgraph": use_graph, "lanes_per_chain": st["lanes_per_chain"],
                   "chains_per_workgroup": st["chains_per_block"], "roles": st.get("roles", 1),
                   "data_modes_per_block": [k for _, k in blocks[0]] if len(blocks) == 1 else None},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "lane-op/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": None if tr is None else tr["bytes_per_launch"],
                     "kernel": kernel, "ops_per_chain_sweep": ops_sweep,
                     "ops_per_launch": ops_per_launch, "avg_launch_ms": avg_launch_s * 1e3,
                     "launches_per_step": st["sampler_launches"]},
        "chain_sweeps_per_s": chains * sweeps_total * args.steps / elapsed,
        "data_moves_per_s": data_per_step * args.steps / elapsed,
        "zero_moves_per_s": (moves_per_step - data_per_step) * args.steps / elapsed,
        "ess_per_s": {"min": float(np.nanmin(ess)) / step_s, "median": float(np.nanmedian(ess)) / step_s},
        "tau_int_sweeps": {"max": float(np.nanmax(tau)), "median": float(np.nanmedian(tau))},
        "forward_ms": fwd_s * 1e3,
        "vjp_ms": vjp_s * 1e3 if want_vjp else None,
        "vjp_over_forward": (vjp_s / fwd_s) if want_vjp else None,
        "forward_ms_without_vjp_moments": None if fwd_novjp_s is None else fwd_novjp_s * 1e3,
        "vjp_moments_forward_overhead": None if fwd_novjp_s is None else fwd_s / fwd_novjp_s - 1.0,
        "vjp_rel_stderr_median": (float(np.median(g[1].cpu().numpy() / np.abs(g[0].cpu().numpy()).max()))
                                  if g is not None else None),
        "setup_ms": st["setup_ms"],
        "sampler_ms_per_step": st["sampler_ms"],
        "graph_replays": st["graph_replays"],
        "chi2_drift_max": st["chi2_drift_max"],
        "split_half": split,
        "plain_fp64_mode_moves_per_s": plain_rate,
        "speedup_vs_plain": value / plain_rate,
    }
    if not args.no_cpu:
        cb = cpu_baseline(prob)
        out["cpu_baseline"] = cb
        out["speedup_vs_cpu_oracle"] = value / cb["value"]
        # the oracle runs the same Markov chain (same moves, same integrated autocorrelation
        # time), so its effective samples per second are its chain-sweeps per second over tau
        tau_med = float(np.nanmedian(tau))
        out["cpu_oracle_ess_per_s_median"] = cb["chain_sweeps_per_s"] / tau_med
    print(json.dumps(out))


if __name__ == "__main__":
    main()
