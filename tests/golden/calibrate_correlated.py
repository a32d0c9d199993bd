"""Oracle against oracle on the batched workload's three uneven datasets.

The GPU parity test of the batched workload compares spectra of hundreds of strongly
correlated grid points (one slow collective fluctuation of a run moves many points at once),
with error bars from 32 chain groups (Student-t tails).  The pass bounds it uses come from
this null distribution: independent oracle runs (64 chains, other seeds, the reference's
protocol) against the stored 256-chain oracle reference of each dataset, with the same
z-score statistics.  Only the CPU oracle and the workload generators are called.

    python tests/golden/calibrate_correlated.py [replicas]

writes tests/golden/correlated_calibration.json.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import workloads  # noqa: E402
from parity_criteria import zscores  # noqa: E402

THREADS = int(os.environ.get("ORACLE_THREADS", "0")) or None


def main(replicas=12):
    out = {"what": "oracle (64 chains, other seeds) against the stored 256-chain oracle reference, "
                   "per dataset and replica: max |z|, fraction of points with |z| > 3, mean z^2",
           "replicas": replicas, "datasets": {}}
    t0 = time.time()
    for name in ("batched_1", "batched_2", "batched_3"):
        ref = np.load(os.path.join(HERE, f"{name}_oracle.npz"))
        meta = json.load(open(os.path.join(HERE, f"{name}_oracle.json")))
        prob = workloads.batched_dataset(meta["index"])
        prep = oracle.prepare(prob)
        init = oracle.nnls_start(prep)
        rows = []
        for r in range(replicas):
            res = oracle.run(prep, chains=64, burnin=meta["burnin"], sweeps=meta["sweeps"],
                             seed=5000 + 100 * meta["index"] + r, groups=meta["groups"],
                             refresh_every=meta["refresh_every"], init=init, threads=THREADS)
            z = zscores(res.mean, res.stderr, ref["mean"], ref["stderr"])
            rows.append(dict(max_z=float(z.max()), frac3=float(np.mean(z > 3.0)),
                             mean_z2=float(np.mean(z ** 2)), n=int(len(z))))
            print(name, r, rows[-1], round(time.time() - t0), "s", flush=True)
        out["datasets"][name] = rows
    allr = [x for rows in out["datasets"].values() for x in rows]
    out["max_of_max_z"] = max(x["max_z"] for x in allr)
    out["max_frac3"] = max(x["frac3"] for x in allr)
    out["max_mean_z2"] = max(x["mean_z2"] for x in allr)
    with open(os.path.join(HERE, "correlated_calibration.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 12)
