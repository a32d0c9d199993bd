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


def principal_t2(delta, ref_groups, rho, k=4):
    """Hotelling's T^2 of a difference of two estimates of a strongly correlated vector, in the
    k leading principal directions of the reference's group values.

    delta: the difference of the two pooled estimates; ref_groups: G x M, the reference's
    estimate from each of its G independent chain groups; rho: the other side's variance over
    the reference's under the null (the same estimator with 1/rho times the chains).  The
    reference's estimate has covariance S / G (S the sample covariance of the group values),
    the difference (1 + rho) S / G.  With e_j, l_j the k leading eigenpairs of S,
      T^2 = sum_j (e_j . delta)^2 / (l_j (1 + rho) / G),
    and (G - k) T^2 / (k (G - 1)) follows F(k, G - k) for Gaussian group values (directions
    taken from S overstate their l_j, which makes the test conservative).  Returns
    (T^2, p value)."""
    from scipy import stats
    X = np.asarray(ref_groups, np.float64)
    G = X.shape[0]
    if not 0 < k < G:
        raise ValueError("need 0 < k < G")
    X = X - X.mean(0)
    S = X.T @ X / (G - 1)
    w, V = np.linalg.eigh(S)
    idx = np.argsort(w)[::-1][:k]
    lam, E = w[idx], V[:, idx]
    proj = E.T @ np.asarray(delta, np.float64)
    t2 = float(np.sum(proj ** 2 / (lam * (1.0 + rho) / G)))
    f = (G - k) * t2 / (k * (G - 1))
    return t2, float(stats.f.sf(f, k, G - k))
