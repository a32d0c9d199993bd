"""Benchmark of the blocked-modes sampler on one MI355X.

One step is one pass of the whole hot path over one synthetic continuation problem of
the single-continuation workload (beta = 20, 201 imaginary times, 800 Lorentzian grid
points in 8 blocks of 100 with up to 20 data modes, sigma = 1e-4, 4096 chains, 2000
burn-in and 10000 measured sweeps, float32 chain state):
    whitening -> float64 block SVDs -> float32 packing -> NNLS start -> sweeps with float64
    residual refreshes every 64 sweeps -> float64 accumulation of <A> and of Cov(r~, A) ->
    error bars -> VJP d<A>/dG v for a seeded cotangent v.
The problem arrays are on the GPU before the timed region starts.

Prints one JSON line (see the fields below).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 64 * 2.4e9   # MI355X: 256 CUs x 64 fp32 lanes x 2.4 GHz (non-packed)


def lane_ops_per_sweep(M, blocks):
    """Algorithmic lane-operations of one chain-sweep.

    Per move of a block with nb components: 4 per component (ratio to the stored
    reciprocal, min/max into the interval, fused update, clamp) plus the scalar draw
    (4 for a flat draw, 40 for the truncated normal); a data move adds 2 per data point
    (the dot product U_i . r and the residual update).
    """
    ops = 0
    for nb, kb in blocks:
        ops += kb * (4 * nb + 2 * M + 40) + (nb - kb) * (4 * nb + 4)
    return ops


class _DevProblem:
    def __init__(self, p, device):
        import torch
        self.K = torch.as_tensor(p.K, dtype=torch.float64, device=device)
        self.G = torch.as_tensor(p.G, dtype=torch.float64, device=device)
        self.sigma = None if p.sigma is None else torch.as_tensor(p.sigma, dtype=torch.float64, device=device)
        self.cov = None if p.cov is None else torch.as_tensor(p.cov, dtype=torch.float64, device=device)
        self.block_start = p.block_start
        self.k = p.k
        self.init = None


def cpu_baseline(prob, seconds_target=15.0):
    """The CPU oracle on the host cores, on a bounded sample of the same workload."""
    import oracle
    threads = min(os.cpu_count() or 1, 64)
    prep = oracle.prepare(prob)
    chains = 4 * threads
    # calibrate on a short run, then size the sample to about seconds_target
    t = time.time()
    oracle.run(prep, chains=threads, burnin=0, sweeps=20, threads=threads, groups=1)
    dt = max(time.time() - t, 1e-3)
    per_chain_sweep = dt / (20.0 * threads / threads)   # seconds per sweep of `threads` chains
    sweeps = int(max(20, min(5000, seconds_target / (per_chain_sweep * chains / threads))))
    t = time.time()
    oracle.run(prep, chains=chains, burnin=0, sweeps=sweeps, threads=threads, groups=4)
    dt = time.time() - t
    moves = chains * sweeps * prob.N
    return {"value": moves / dt, "unit": "mode-moves/s", "cores": threads, "kind": "oracle",
            "sample": f"{chains} chains x {sweeps} sweeps of the same problem from the flat start "
                      f"({moves:.3g} moves, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=10000)
    ap.add_argument("--burnin", type=int, default=2000)
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--no-vjp", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lanes", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)

    import torch
    import workloads
    import paper_1912_01379_amd as pk

    dev = torch.device("cuda:0")
    prob = workloads.config2()
    v = torch.as_tensor(workloads.config4_cotangent(prob.N), dtype=torch.float64, device=dev)
    dp = _DevProblem(prob, dev)
    want_vjp = not args.no_vjp

    def step():
        plan = pk.Plan([dp], chains=args.chains, burnin=args.burnin, sweeps=args.sweeps, seed=2024,
                       precision="fp32", refresh_every=64, want_vjp=want_vjp, groups=32,
                       lanes_per_chain=args.lanes, start="nnls", device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = plan.vjp(v) if want_vjp else None
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        blocks = []
        for b in range(prob.B):
            nb = int(prob.block_start[b + 1] - prob.block_start[b])
            k = plan.factors(0, b, nb)[0]
            blocks.append((nb, k))
        plan.close()
        return res, (t1 - t0), (t2 - t1), blocks, g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    outs = []
    for _ in range(args.steps):
        outs.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    res, fwd_s, vjp_s, blocks, _ = outs[-1]
    st = res.stats
    moves_per_step = args.chains * (args.burnin + args.sweeps) * prob.N
    value = moves_per_step * args.steps / elapsed
    # roofline of the sampler kernel from its own launch events
    ops_sweep = lane_ops_per_sweep(prob.M, blocks)
    achieved = ops_sweep * args.chains * st["sampler_sweeps"] / (st["sampler_ms"] * 1e-3)
    mean = res.mean.cpu().numpy()
    se = res.stderr.cpu().numpy()
    sd = res.post_sd.cpu().numpy()
    ess = (sd / se) ** 2
    step_s = elapsed / args.steps

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
        "config": {"workload": "single continuation: beta=20, M=201, N=800 Lorentzian grid, "
                               "8 blocks x 100, k<=20, sigma=1e-4, fp32 chains, NNLS start",
                   "chains": args.chains, "burnin": args.burnin, "sweeps": args.sweeps,
                   "vjp": want_vjp, "lanes_per_chain": st["lanes_per_chain"],
                   "chains_per_workgroup": st["chains_per_block"],
                   "data_modes_per_block": [k for _, k in blocks]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "lane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                     "kernel": "k_sample32", "ops_per_chain_sweep": ops_sweep,
                     "sampler_ms_per_step": st["sampler_ms"],
                     "avg_launch_ms": st["sampler_ms"] / max(1, st["sampler_launches"])},
        "ess_per_s": {"min": float(np.nanmin(ess)) / step_s, "median": float(np.nanmedian(ess)) / step_s},
        "forward_ms": fwd_s * 1e3,
        "vjp_ms": vjp_s * 1e3 if want_vjp else None,
        "vjp_over_forward": (vjp_s / fwd_s) if want_vjp else None,
        "setup_ms": st["setup_ms"],
        "chi2_drift_max": st["chi2_drift_max"],
        "plain_fp64_mode_moves_per_s": plain_rate,
        "speedup_vs_plain": value / plain_rate,
    }
    if not args.no_cpu:
        cb = cpu_baseline(prob)
        out["cpu_baseline"] = cb
        out["speedup_vs_cpu_oracle"] = value / cb["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
