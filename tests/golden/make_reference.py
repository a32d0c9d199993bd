"""Write the stored oracle averages used by the GPU parity tests.

Only the CPU oracle and the seeded workload generators are called.  Each file holds the
oracle's average spectrum <A> (the estimate of Eq. (MCint) by blocked modes sampling,
Sec. IV.C) and its standard error over independent chain groups, for a fixed protocol
(chains, burn-in, sweeps, seed, start model) that the GPU test repeats with its own chains.
The single-continuation reference starts from the NNLS start of Sec. IV.D, so that both sides average
over the equilibrated chain rather than over the slow relaxation from a flat start.

    python tests/golden/make_reference.py [plain] [single] [batched_1] [batched_2] [batched_3] [differentiation] [large]

The large-workload reference (401 correlated data points whitened by their Cholesky factor, 4000
grid points in 32 blocks, Sec. IV and Sec. IV.C) takes about half an hour on 8 cores.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

THREADS = int(os.environ.get("ORACLE_THREADS", "0")) or None

PROTOCOLS = {
    "plain": dict(problem="plain_one_chain", chains=64, burnin=200, sweeps=2000, seed=11, groups=32,
                 refresh_every=64),
    # 512 chains: the reference's error bars are then about a third of those of the float32
    # run it is compared with, so a bias of one reference error bar is visible
    "single": dict(problem="single_continuation", chains=512, burnin=500, sweeps=2000, seed=12, groups=32,
                 refresh_every=64, start="nnls"),
    "large": dict(problem="large_workload", chains=256, burnin=1000, sweeps=5000, seed=15, groups=32,
                 refresh_every=64, start="nnls"),
    # the differentiation workload: the single-continuation problem with its seeded cotangent v; J^T v
    # (Sec. II, Eq. (PI) differentiated in the data), its error bar over the chain groups and
    # the value of every group (their covariance carries the strong correlation between the
    # entries of J^T v, which the parity test needs)
    "differentiation": dict(problem="single_continuation", chains=1024, burnin=500, sweeps=2000, seed=14, groups=32,
                 refresh_every=64, start="nnls", vjp="differentiation_cotangent"),
}
# three uneven datasets of the batched workload (N = 396, 670, 407 in 4, 7, 4 blocks); 256
# chains, so that the reference error bars are half those of a 64-chain run
for _i in (1, 2, 3):
    PROTOCOLS[f"batched_{_i}"] = dict(problem="batched_dataset", index=_i, chains=256, burnin=500,
                                   sweeps=2000, seed=30 + _i, groups=32, refresh_every=64,
                                   start="nnls")


def make(name):
    proto = PROTOCOLS[name]
    gen = getattr(workloads, proto["problem"])
    prob = gen(proto["index"]) if "index" in proto else gen()
    prep = oracle.prepare(prob)
    t = time.time()
    init = oracle.nnls_start(prep) if proto.get("start") == "nnls" else None
    v = getattr(workloads, proto["vjp"])(prep.N) if "vjp" in proto else None
    res = oracle.run(prep, chains=proto["chains"], burnin=proto["burnin"], sweeps=proto["sweeps"],
                     seed=proto["seed"], groups=proto["groups"], refresh_every=proto["refresh_every"],
                     init=init, threads=THREADS, vjp_v=v)
    dt = time.time() - t
    out = os.path.join(HERE, f"{name}_oracle.npz")
    extra = {} if v is None else dict(v=v, vjp=res.vjp, vjp_se=res.vjp_se, vjp_groups=res.vjp_groups)
    np.savez_compressed(out, mean=res.mean, stderr=res.stderr, post_sd=res.post_sd,
                        kb=prep.kb, chi2_final=res.final_chi2, **extra)
    meta = dict(proto, seconds=round(dt, 1), status=res.status, drift_max=res.drift_max,
                what="oracle <A> and standard error over chain groups (Eq. (MCint), Sec. IV.C)")
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(name, "done in", round(dt, 1), "s; kb =", list(prep.kb), flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(PROTOCOLS)):
        make(n)
