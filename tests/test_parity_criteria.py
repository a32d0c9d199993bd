"""The statistical pass criteria of the GPU parity tests, checked on synthetic Gaussian group
values with a known covariance (host only)."""
import numpy as np

from parity_criteria import principal_t2


def _smooth_cov(M):
    t = np.linspace(0.0, 1.0, M)
    B = np.stack([np.sin((j + 1) * np.pi * t) * 0.5 ** j for j in range(6)], 1)
    S = B @ B.T + 1e-4 * np.eye(M)
    return S, np.linalg.cholesky(S)


def test_principal_t2_size_and_power():
    """Under the null the p value is uniform (rejections at 1 % about 1 %); a shift of five
    standard deviations of the difference along the leading direction is found."""
    rng = np.random.default_rng(7)
    M, G, rho = 201, 32, 0.25
    S, Lc = _smooth_cov(M)
    w, V = np.linalg.eigh(S)
    e1, l1 = V[:, -1], w[-1]

    def trial(shift):
        X = (Lc @ rng.standard_normal((M, G))).T
        other = np.sqrt(rho / G) * (Lc @ rng.standard_normal(M)) + shift * np.sqrt((1 + rho) * l1 / G) * e1
        return principal_t2(other - X.mean(0), X, rho)[1]

    p0 = np.array([trial(0.0) for _ in range(1500)])
    assert 0.004 <= np.mean(p0 < 0.01) <= 0.02
    assert 0.35 <= np.mean(p0 < 0.5) <= 0.65
    p5 = np.array([trial(5.0) for _ in range(300)])
    assert np.mean(p5 < 1e-3) > 0.45


def test_principal_t2_matches_the_one_direction_case():
    """k = 1 with group values along one direction: T^2 is the squared t statistic of the
    difference along it."""
    rng = np.random.default_rng(3)
    G, M = 16, 5
    e = np.array([1.0, 2.0, 0.0, -1.0, 0.5])
    e /= np.linalg.norm(e)
    a = rng.standard_normal(G)
    X = np.outer(a, e)
    d = 0.3 * e
    t2, p = principal_t2(d, X, 0.5, k=1)
    var = np.var(a, ddof=1) * 1.5 / G
    assert np.isclose(t2, 0.09 / var)
    from scipy import stats
    assert np.isclose(p, stats.f.sf(t2, 1, G - 1))
