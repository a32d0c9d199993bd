"""Pass criteria of the statistical parity tests (shared by the GPU tests and the CPU
calibration of their bounds).

Per grid point z_n = |Delta_n| / sqrt(SE_1^2 + SE_2^2), the error bars from independent chain
groups.  A comparison passes when max z and the number of points beyond 3 stay within bounds;
for spectra of many strongly correlated points the mean of z^2 is bounded as well, which
catches a bias shared by many points.
"""
import numpy as np


def zscores(m1, s1, m2, s2):
    z = np.abs(np.asarray(m1) - np.asarray(m2)) / np.sqrt(np.asarray(s1) ** 2 + np.asarray(s2) ** 2)
    return z[np.isfinite(z)]


def zscore_ok(m1, s1, m2, s2, frac=0.01, zmax=4.5, n3_min=2, mean_z2=None):
    z = zscores(m1, s1, m2, s2)
    n3 = int(np.sum(z > 3.0))
    ok = float(z.max()) <= zmax and n3 <= max(n3_min, int(frac * len(z)))
    if mean_z2 is not None:
        ok = ok and float(np.mean(z ** 2)) <= mean_z2
    return ok, (float(z.max()), n3, len(z), float(np.mean(z ** 2)))


# Spectra of many strongly correlated points (the batched workload, the conductivity test case
# on a hierarchy): bounds above the spread of the oracle-against-oracle runs of
# tests/golden/calibrate_correlated.py (36 runs: max z up to 5.1, up to 2.5 % of the points
# beyond 3, mean z^2 up to 1.8; its output, correlated_calibration.json, is checked against
# these bounds by a CPU test).
CORRELATED = dict(frac=0.035, zmax=5.5, n3_min=3, mean_z2=2.2)
