"""Pins of the FP64 CPU oracle against things other than itself.

Each test fixes a part of the oracle with a result the paper or the mathematics
determines independently: closed forms, quadrature, a library routine that implements
the same special function, or an independent re-derivation of a step in another basis.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import workloads


# --------------------------------------------------------------------------------------
# special functions and the truncated normal
# --------------------------------------------------------------------------------------

def test_mills_ratio_matches_scipy_erfcx(orc):
    # m(x) = Q(x)/phi(x) = sqrt(pi/2) erfcx(x/sqrt 2): two independent implementations
    for x in [0.0, 1e-8, 0.3, 1.0, 2.5, 4.999, 5.0, 5.001, 7.0, 12.0, 30.0, 100.0, 1e4]:
        ref = math.sqrt(math.pi / 2) * special.erfcx(x / math.sqrt(2.0))
        assert abs(orc.mills(x) / ref - 1.0) < 5e-15, x


@pytest.mark.parametrize("r0,t1,t2", [
    (0.0, 0.0, 1e-9), (0.0, -0.3, 0.2), (0.0, 0.0, 1.9), (0.0, 0.0, 2.1), (0.0, -2.1, 0.5),
    (0.0, -5.0, -1.0), (0.0, -np.inf, -3.0), (0.0, -np.inf, 1.0), (0.0, 1.0, np.inf), (0.0, -1.0, np.inf),
    (2.0, 0.0, 0.2), (2.0, 0.0, 1.0), (2.0, 0.5, 3.0), (7.99, 0.0, np.inf), (8.0, 0.0, 0.1),
    (50.0, 0.0, 0.03), (50.0, 0.01, np.inf), (3e3, 0.0, 0.01), (1e-3, 0.0, 1e-6),
    (0.7, 0.0, np.inf), (40.0, 0.0, np.inf)])
def test_mass_matches_quadrature(orc, r0, t1, t2):
    """The scaled normal mass of [r0 + t1, r0 + t2] (both branches, the switch between them,
    infinite ends) against adaptive quadrature of the same integrand."""
    f = lambda t: math.exp(-0.5 * t * (2.0 * r0 + t))
    ref = integrate.quad(f, t1, t2, epsabs=0, epsrel=1e-13, limit=400)[0]
    assert abs(orc.mass(r0, t1, t2) / ref - 1.0) < 5e-14


def test_mass_matches_log_ndtr_in_far_tails(orc):
    """Far above the centre the mass is Q(r0 + t1) - Q(r0 + t2) over phi(r0); scipy's log_ndtr
    gives both tails independently."""
    for r0, t1, t2 in [(10.0, 0.5, 2.0), (30.0, 0.1, 1.0), (37.0, 0.0, np.inf), (200.0, 0.02, 0.5)]:
        lq1 = special.log_ndtr(-(r0 + t1))
        lq2 = special.log_ndtr(-(r0 + t2)) if np.isfinite(t2) else -np.inf
        lphi = stats.norm.logpdf(r0)
        ref = math.exp(lq1 - lphi) * -math.expm1(lq2 - lq1)
        # the reference subtracts logarithms of size (r0 + t1)^2 / 2: that is its resolution
        tol = 2e-14 + 2.0 * np.finfo(float).eps * (r0 + t1) ** 2
        assert abs(orc.mass(r0, t1, t2) / ref - 1.0) < tol, (r0, t1, t2)


def _trunc_cdf(x, c, d, lo, hi):
    """Distribution function F, its complement 1 - F, and the density of N(c/d, 1/d^2)
    restricted to [lo, hi] at x, in 60-digit arithmetic (mpmath), each tail from the side
    where it is small."""
    import mpmath
    mpmath.mp.dps = 60
    c, d, x = mpmath.mpf(c), mpmath.mpf(d), mpmath.mpf(x)
    a = d * mpmath.mpf(lo) - c if np.isfinite(lo) else -mpmath.inf
    b = d * mpmath.mpf(hi) - c if np.isfinite(hi) else mpmath.inf
    z = d * x - c
    if a >= 0:   # above the centre: upper tails
        qa, qb, qz = mpmath.ncdf(-a), mpmath.ncdf(-b), mpmath.ncdf(-z)
        den, F, Fc = qa - qb, qa - qz, qz - qb
    else:
        pa, pb, pz = mpmath.ncdf(a), mpmath.ncdf(b), mpmath.ncdf(z)
        den, F, Fc = pb - pa, pz - pa, pb - pz
    return F / den, Fc / den, d * mpmath.npdf(z) / den


CASES = [(0.0, 1.0, -1.0, 2.0), (5.0, 2.0, -3.0, 0.5), (-40.0, 1.0, 0.0, np.inf),
         (40.0, 1.0, -np.inf, 0.0), (1.0, 1e3, -0.01, 0.02), (0.0, 3.0, -np.inf, 1.0),
         (2.0, 1.0, 0.0, np.inf), (-20.0, 1.0, -1.0, 0.0), (0.4, 0.5, -0.2, 0.1),
         (12.0, 4.0, -1.0, 5.0)]


@pytest.mark.parametrize("c,d,lo,hi", CASES)
def test_tn_inverse_cdf(orc, c, d, lo, hi):
    """The draw at u has distribution-function value u (checked in 60-digit arithmetic)."""
    for k in [1, 3, 1000, 2 ** 30, 2 ** 51, 2 ** 52 - 1000, 2 ** 53 - 3]:
        u = k * 2.0 ** -53
        x = orc.tn_draw(c, d, lo, hi, u)
        assert lo <= x <= hi
        F, Fc, dens = _trunc_cdf(x, c, d, lo, hi)
        err = float(F) - u if u <= 0.5 else float(Fc) - (1.0 - u)
        # what rounding x to a double moves F by (density times a few ulps of x), and the
        # resolution of the standardised ends d lo - c, d hi - c that the draw starts from
        ends = [abs(d * e) for e in (lo, hi) if np.isfinite(e)]
        res = np.spacing(abs(x) + 1e-300) + (np.spacing(abs(c)) + sum(np.spacing(e) for e in ends)) / d
        tol = 1e-13 * min(u, 1.0 - u) + 8.0 * float(dens) * res
        assert abs(err) <= tol, (u, x, err, tol)


def test_tn_narrow_interval_is_tilted_uniform(orc):
    """d -> 0: the Gaussian is almost flat over [lo, hi]; the exact density is exp(-(d x - c)^2/2)."""
    c, d, lo, hi = 0.3, 1e-9, -2.0, 3.0
    for u in [1e-6, 0.25, 0.5, 0.9]:
        x = orc.tn_draw(c, d, lo, hi, u)
        # density ~ exp(c d x) (linear tilt); CDF of the tilt:
        lam = c * d
        ref = lo + math.log1p(u * math.expm1(lam * (hi - lo))) / lam
        assert abs(x - ref) < 1e-12 * (hi - lo)


@pytest.mark.parametrize("c,d,lo,hi", CASES[:8])
def test_tn_mean_by_quantile_integration(orc, c, d, lo, hi):
    """Integral of the quantile function over u equals the closed-form truncated mean."""
    n = 4001
    us = (np.arange(n) + 0.5) / n
    xs = np.array([orc.tn_draw(c, d, lo, hi, float(u)) for u in us])
    mu, tau = c / d, 1.0 / d
    ref = stats.truncnorm.mean((lo - mu) / tau, (hi - mu) / tau, loc=mu, scale=tau)
    spread = stats.truncnorm.std((lo - mu) / tau, (hi - mu) / tau, loc=mu, scale=tau)
    assert abs(xs.mean() - ref) < 2e-3 * spread + 1e-12


# --------------------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------------------

def test_uniforms_open_interval_and_uniform(orc):
    us = np.array([orc.move_uniform(99, 0, c, s, b, i)
                   for c in range(4) for s in range(25) for b in range(4) for i in range(25)])
    assert np.all(us > 0) and np.all(us < 1)
    # (2J+1) 2^-53 exactly
    k = us * 2.0 ** 53
    assert np.all(k == np.round(k)) and np.all(np.round(k) % 2 == 1)
    hist, _ = np.histogram(us, bins=50, range=(0, 1))
    chi2 = float(((hist - len(us) / 50) ** 2 / (len(us) / 50)).sum())
    assert stats.chi2.sf(chi2, 49) > 1e-4
    assert abs(np.corrcoef(us[:-1], us[1:])[0, 1]) < 0.05
    assert len(np.unique(us)) == len(us)


def test_philox_known_answers(orc):
    """Philox4x32-10 against the known-answer vectors published with the generator
    (Salmon et al., SC'11, Random123): zero counter and key, all-ones counter and key, and
    the counter and key taken from the hexadecimal digits of pi."""
    cases = [([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
             ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
             ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
              [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1])]
    for ctr, key, want in cases:
        assert [int(w) for w in orc.philox(ctr, key)] == want


def test_philox_counter_sensitivity(orc):
    base = orc.philox([1, 2, 3, 4], [5, 6])
    for pos in range(4):
        ctr = [1, 2, 3, 4]
        ctr[pos] ^= 1
        out = orc.philox(ctr, [5, 6])
        # every output word changes, and about half of the 128 bits flip
        flips = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, out))
        assert 40 < flips < 88


# --------------------------------------------------------------------------------------
# problems with closed-form or quadrature answers
# --------------------------------------------------------------------------------------

def _problem(K, G, sigma, bstart, k=None):
    M = K.shape[0]
    return workloads.Problem(K=np.asarray(K, float), G=np.asarray(G, float),
                             sigma=np.full(M, float(sigma)), block_start=np.asarray(bstart, np.int64),
                             k=k)


def _within(mc_mean, mc_se, ref, nsig=4.5, floor=1e-12):
    z = np.abs(mc_mean - ref) / np.maximum(mc_se, floor)
    return float(np.max(z))


def test_one_point_grid_is_truncated_normal(orc):
    """N = 1: <A> = mu + s phi(mu/s)/Phi(mu/s) (truncated normal mean)."""
    rng = np.random.default_rng(3)
    k = rng.uniform(0.5, 1.5, 7)
    for mu_over_s in [3.0, 0.2, -2.0, -15.0]:
        s = 1.0 / np.linalg.norm(k)
        mu = mu_over_s * s
        G = k * mu + 0.0
        p = _problem(k[:, None], G, 1.0, [0, 1])
        prep = orc.prepare(p)
        res = orc.run(prep, chains=8, burnin=10, sweeps=20000, groups=16)
        alpha = mu / s
        ref = mu + s * math.exp(stats.norm.logpdf(alpha) - special.log_ndtr(alpha))
        assert _within(res.mean, res.stderr, ref) < 4.5, (mu_over_s, res.mean, ref)


def test_orthogonal_columns_factorise_including_tails(orc):
    """K~ = Q diag(d): independent truncated normals, centres from -40 s to +40 s."""
    rng = np.random.default_rng(5)
    M, N = 12, 6
    Q, _ = np.linalg.qr(rng.standard_normal((M, N)))
    d = np.array([50.0, 20.0, 7.0, 3.0, 1.0, 0.3])
    s = 1.0 / d
    mu = np.array([-40.0, -6.0, -0.5, 0.0, 1.5, 40.0]) * s
    K = Q * d[None, :]
    G = Q @ (d * mu)
    p = _problem(K, G, 1.0, [0, 3, 6])
    prep = orc.prepare(p)
    res = orc.run(prep, chains=8, burnin=10, sweeps=20000, groups=16)
    alpha = mu / s
    ref = mu + s * np.exp(stats.norm.logpdf(alpha) - special.log_ndtr(alpha))
    assert _within(res.mean, res.stderr, ref) < 4.5


def test_sum_rule_only_data_gives_flat_default(orc):
    """K = 1^T, g = 1 (Eq. (def)): <A_n> = E[S]/N, S ~ S^(N-1) exp(-(S-1)^2/2s^2)."""
    N, sig = 8, 0.3
    ws = lambda S, p: S ** (N - 1 + p) * math.exp(-0.5 * ((S - 1.0) / sig) ** 2)
    Z = integrate.quad(lambda S: ws(S, 0), 0, 10)[0]
    ES = integrate.quad(lambda S: ws(S, 1), 0, 10)[0] / Z
    ES2 = integrate.quad(lambda S: ws(S, 2), 0, 10)[0] / Z
    EA = ES / N
    EA2 = ES2 * 2.0 / (N * (N + 1))   # A_n/S ~ Beta(1, N-1)
    for bstart in ([0, 8], [0, 4, 8]):
        p = _problem(np.ones((1, N)), [1.0], sig, bstart)
        prep = orc.prepare(p)
        assert list(prep.kb) == [1] * (len(bstart) - 1)
        res = orc.run(prep, chains=16, burnin=200, sweeps=20000, groups=16)
        assert _within(res.mean, res.stderr, EA) < 4.5, (bstart, res.mean, EA)
        assert np.allclose(res.post_sd, math.sqrt(EA2 - EA * EA), rtol=0.03)


def _chi2_bounds(R):
    """Bounds for the sum of R squared z-scores whose error bars come from 32 chain groups:
    the 0.1% and 99.9% points of chi^2(R), the upper one widened by the Student-t variance
    31/29 of a 31-degree-of-freedom error bar."""
    return stats.chi2.ppf(0.001, R), stats.chi2.ppf(0.999, R) * 31.0 / 29.0


def test_standard_error_is_calibrated_on_closed_forms(orc):
    """The error bar (standard deviation of 32 chain-group means over sqrt(32)) is what every
    parity test divides by.  On two closed forms, 120 seeded replicas each: the one-point grid
    (a truncated normal) and the sum-rule-only data (E[S]/N by quadrature, Eq. (def)), the
    sum of squared z-scores must fall inside chi^2(120).  An error bar inflated by sqrt(2)
    (the sum then sits near 60 against a lower bound of 80) or deflated by it (near 240
    against 185), let alone one off by sqrt(32), lands outside."""
    R = 120
    lo, hi = _chi2_bounds(R)
    # one point: N(mu, s^2) restricted to A >= 0
    k = np.array([0.8, 1.1, 0.6, 1.3])
    s = 1.0 / np.linalg.norm(k)
    mu = 0.4 * s
    p1 = _problem(k[:, None], k * mu, 1.0, [0, 1])
    ref1 = mu + s * math.exp(stats.norm.logpdf(mu / s) - special.log_ndtr(mu / s))
    prep1 = orc.prepare(p1)
    # sum rule on 6 points, one block
    N, sig = 6, 0.3
    ws = lambda S, q: S ** (N - 1 + q) * math.exp(-0.5 * ((S - 1.0) / sig) ** 2)
    ref2 = integrate.quad(lambda S: ws(S, 1), 0, 10)[0] / integrate.quad(lambda S: ws(S, 0), 0, 10)[0] / N
    prep2 = orc.prepare(_problem(np.ones((1, N)), [1.0], sig, [0, N]))
    z1, z2 = [], []
    for r in range(R):
        a = orc.run(prep1, chains=64, burnin=20, sweeps=200, groups=32, seed=7000 + r, threads=4)
        z1.append((a.mean[0] - ref1) / a.stderr[0])
        b = orc.run(prep2, chains=64, burnin=300, sweeps=600, groups=32, seed=9000 + r, threads=4)
        z2.append((b.mean[0] - ref2) / b.stderr[0])
    for z in (np.array(z1), np.array(z2)):
        q = float(np.sum(z ** 2))
        assert lo < q < hi, (q, lo, hi)
        # and no bias: the mean z is within 4 of its own standard error
        assert abs(z.mean()) < 4.0 * z.std(ddof=1) / math.sqrt(R)


def test_sum_rule_only_data_with_a_hierarchy(orc):
    """The same closed form as above, sampled with the hierarchy of Fig. 2 on 8 points (one
    block, halves, the shifted quarters, the components; a random level per sweep)."""
    N, sig = 8, 0.3
    ws = lambda S, p: S ** (N - 1 + p) * math.exp(-0.5 * ((S - 1.0) / sig) ** 2)
    Z = integrate.quad(lambda S: ws(S, 0), 0, 10)[0]
    EA = integrate.quad(lambda S: ws(S, 1), 0, 10)[0] / Z / N
    EA2 = integrate.quad(lambda S: ws(S, 2), 0, 10)[0] / Z * 2.0 / (N * (N + 1))
    p = _problem(np.ones((1, N)), [1.0], sig, [0, N])
    p.levels = orc.hierarchy(N)
    prep = orc.prepare(p)
    assert prep.B == 1 + 2 + 5 + 8 and list(prep.kb) == [1] * prep.B
    res = orc.run(prep, chains=16, burnin=200, sweeps=20000, groups=16)
    assert _within(res.mean, res.stderr, EA) < 4.5, (res.mean, EA)
    assert np.allclose(res.post_sd, math.sqrt(EA2 - EA * EA), rtol=0.03)


def test_hierarchy_partitions_of_fig2(orc):
    """Fig. 2: one block on top, halves below it, the intervals shifted by half their width on
    every other level (so that the grid centre is no boundary there), the single points at the
    bottom.  8 points worked by hand; general N checked for the structure."""
    h = orc.hierarchy(8)
    assert [list(x) for x in h] == [[0, 8], [0, 4, 8], [0, 1, 3, 5, 7, 8], list(range(9))]
    for N in (2, 3, 7, 40, 120, 800, 1000):
        h = orc.hierarchy(N)
        assert list(h[0]) == [0, N] and list(h[-1]) == list(range(N + 1))
        for lvl, cuts in enumerate(h[:-1]):
            assert cuts[0] == 0 and cuts[-1] == N and np.all(np.diff(cuts) > 0)
            w = N / 2 ** lvl
            assert w >= 2
            sizes = np.diff(cuts)
            if lvl >= 2 and lvl % 2 == 0:       # shifted: two half-width end blocks
                assert len(sizes) == 2 ** lvl + 1
                assert abs(sizes[0] - w / 2) < 1 and abs(sizes[-1] - w / 2) < 1
                assert np.all(np.abs(sizes[1:-1] - w) < 1)
                assert N % 2 or N // 2 not in set(cuts.tolist())
            else:
                assert len(sizes) == 2 ** lvl and np.all(np.abs(sizes - w) < 1)
        # below the top, no boundary is shared by every blocked level
        inner = [set(c[1:-1].tolist()) for c in h[1:-1]]
        if len(inner) >= 2:
            assert not set.intersection(*inner)
        assert N < 4 or 2 ** len(h[:-1]) > N // 2   # the blocked levels reach width < 4
    # levels with a block above the limit are left out
    assert [len(x) - 1 for x in orc.hierarchy(800, max_block=128)] == [8, 17, 32, 65, 128, 257, 800]


def test_hierarchy_levels_are_uniform_and_shared(orc):
    """Sec. IV.C: each sweep samples one level chosen at random; the choice is uniform over the
    levels, and differs between problems (keyed like the moves)."""
    L, S = 7, 28000
    lv = np.array([orc.sweep_level(11, 0, s, L) for s in range(S)])
    assert lv.min() == 0 and lv.max() == L - 1
    counts = np.bincount(lv, minlength=L)
    chi2 = float(np.sum((counts - S / L) ** 2 / (S / L)))
    assert chi2 < stats.chi2.ppf(0.9999, L - 1), counts
    # consecutive sweeps are independent: pairs are uniform over L^2 cells
    pairs = np.bincount(lv[:-1] * L + lv[1:], minlength=L * L)
    chi2p = float(np.sum((pairs - (S - 1) / L ** 2) ** 2 / ((S - 1) / L ** 2)))
    assert chi2p < stats.chi2.ppf(0.9999, L * L - 1)
    other = np.array([orc.sweep_level(11, 1, s, L) for s in range(2000)])
    assert np.mean(other == lv[:2000]) < 0.25
    assert all(orc.sweep_level(11, 0, s, 1) == 0 for s in range(50))


def test_hierarchy_keys_moves_by_the_block_within_its_level(orc):
    """Two levels holding the same partition sample exactly as that partition alone: the
    random numbers of a move depend on the block's index within its level, and the factors
    come from the level's own blocks."""
    p = workloads.small_problem(M=21, N=12, nblocks=3)
    prep1 = orc.prepare(p)
    p.levels = [p.block_start, p.block_start]
    prep2 = orc.prepare(p)
    assert prep2.B == 2 * prep1.B
    r1 = orc.run(prep1, chains=3, burnin=0, sweeps=60, groups=3, traj_chain=1)
    r2 = orc.run(prep2, chains=3, burnin=0, sweeps=60, groups=3, traj_chain=1)
    assert np.array_equal(r1.traj_A, r2.traj_A) and np.array_equal(r1.final_r, r2.final_r)
    # a different second level changes exactly the sweeps that pick it
    p.levels = [p.block_start, np.array([0, 5, 12])]
    r3 = orc.run(orc.prepare(p), chains=3, burnin=0, sweeps=60, groups=3, traj_chain=1)
    first = next(s for s in range(60) if orc.sweep_level(1234, 0, s, 2) == 1)
    assert np.array_equal(r3.traj_A[:first], r1.traj_A[:first])
    assert not np.array_equal(r3.traj_A[first], r1.traj_A[first])


def _quad_mean_2d(K, G):
    """<A> over A >= 0 for N = 2 by quadrature (inner integral in closed form)."""
    k1, k2 = K[:, 0], K[:, 1]
    n2 = k2 @ k2
    s = 1.0 / math.sqrt(n2)

    def parts(a1):
        r1 = G - k1 * a1
        m = (k2 @ r1) / n2
        logz = -0.5 * (r1 @ r1 - n2 * m * m) + special.log_ndtr(m / s)
        inner_mean = m + s * math.exp(stats.norm.logpdf(m / s) - special.log_ndtr(m / s))
        return logz, inner_mean

    grid = np.linspace(0, 5, 2001)
    shift = max(parts(a)[0] for a in grid)
    w = lambda a: math.exp(parts(a)[0] - shift)
    Z = integrate.quad(w, 0, np.inf, limit=400, epsrel=1e-12)[0]
    m1 = integrate.quad(lambda a: a * w(a), 0, np.inf, limit=400, epsrel=1e-12)[0] / Z
    m2 = integrate.quad(lambda a: parts(a)[1] * w(a), 0, np.inf, limit=400, epsrel=1e-12)[0] / Z
    return np.array([m1, m2])


def test_two_point_grid_against_quadrature(orc):
    beta = 10.0
    tau = workloads.imaginary_times(11, beta)
    x = np.array([-1.0, 0.5])
    K = workloads.fermionic_kernel(tau, x, beta)
    sig = 0.05
    G = K @ np.array([0.3, 0.02]) + sig * np.random.default_rng(8).standard_normal(11)
    ref = _quad_mean_2d(K / sig, G / sig)
    p = _problem(K, G, sig, [0, 2])
    res = orc.run(orc.prepare(p), chains=16, burnin=100, sweeps=40000, groups=16)
    assert _within(res.mean, res.stderr, ref) < 4.5, (res.mean, ref, res.stderr)
    # two one-point blocks: components sampling, same average
    p2 = _problem(K, G, sig, [0, 1, 2])
    res2 = orc.run(orc.prepare(p2), chains=16, burnin=100, sweeps=40000, groups=16)
    assert _within(res2.mean, res2.stderr, ref) < 4.5, (res2.mean, ref)


def test_three_point_grid_against_quadrature(orc):
    beta = 10.0
    tau = workloads.imaginary_times(11, beta)
    x = np.array([-1.5, 0.0, 1.5])
    K = workloads.fermionic_kernel(tau, x, beta)
    sig = 0.05
    G = K @ np.array([0.3, 0.05, 0.2]) + sig * np.random.default_rng(9).standard_normal(11)
    Kt, gt = K / sig, G / sig
    k3 = Kt[:, 2]
    n3 = k3 @ k3
    s3 = 1.0 / math.sqrt(n3)

    def inner(a1, a2):
        r = gt - Kt[:, 0] * a1 - Kt[:, 1] * a2
        m = (k3 @ r) / n3
        logz = -0.5 * (r @ r - n3 * m * m) + special.log_ndtr(m / s3)
        mean3 = m + s3 * math.exp(stats.norm.logpdf(m / s3) - special.log_ndtr(m / s3))
        return logz, mean3

    # unconstrained optimum as a shift for the exponent
    shift = max(inner(a, b)[0] for a in np.linspace(0, 2, 41) for b in np.linspace(0, 2, 41))
    f = lambda b, a, p: (a if p == 1 else b if p == 2 else (inner(a, b)[1] if p == 3 else 1.0)) \
        * math.exp(inner(a, b)[0] - shift)
    up = 3.0
    Z = integrate.dblquad(lambda b, a: f(b, a, 0), 0, up, 0, up, epsrel=1e-9)[0]
    ref = np.array([integrate.dblquad(lambda b, a: f(b, a, p), 0, up, 0, up, epsrel=1e-9)[0] / Z
                    for p in (1, 2, 3)])
    p = _problem(K, G, sig, [0, 3])
    res = orc.run(orc.prepare(p), chains=16, burnin=100, sweeps=40000, groups=16)
    assert _within(res.mean, res.stderr, ref) < 4.5, (res.mean, ref, res.stderr)


def test_gaussian_limit_mean_and_vjp(orc):
    """Positivity inactive: <A> = (K~^T K~)^-1 K~^T g~, J = Cov K~^T T (closed forms)."""
    p = workloads.gaussian_limit_problem()
    prep = orc.prepare(p)
    res = orc.run(prep, chains=32, burnin=20, sweeps=4000, groups=32, want_cross=True)
    Kt, gt = prep.Kt, prep.gt
    cov = np.linalg.inv(Kt.T @ Kt)
    mean = cov @ Kt.T @ gt
    assert _within(res.mean, res.stderr, mean) < 4.5
    assert np.allclose(res.post_sd, np.sqrt(np.diag(cov)), rtol=0.02)
    J = cov @ Kt.T / p.sigma[None, :]      # d<A>/dG = Cov K~^T T, T = diag(1/sigma)
    v = np.array([1.0, -0.5, 0.25, 2.0])
    ref = J.T @ v
    got = orc.vjp(res, v)
    assert np.linalg.norm(got - ref) < 0.03 * np.linalg.norm(ref)


def test_vjp_standard_error_is_calibrated_on_the_gaussian_limit(orc):
    """The error bar of J^T v (standard deviation over 32 chain groups of each group's own
    covariance estimate, over sqrt(32)) against the closed form J = Cov K~^T T of the Gaussian
    limit: 120 seeded replicas, the sum of squared z-scores of three data points inside
    chi^2(120) each, and the pooled estimate equal to the cross-moment route."""
    p = workloads.gaussian_limit_problem()
    prep = orc.prepare(p)
    Kt = prep.Kt
    cov = np.linalg.inv(Kt.T @ Kt)
    J = cov @ Kt.T / p.sigma[None, :]
    v = np.array([1.0, -0.5, 0.25, 2.0])
    ref = J.T @ v
    R = 120
    lo, hi = _chi2_bounds(R)
    ms = [0, 100, 200]
    z = np.zeros((R, len(ms)))
    for r in range(R):
        res = orc.run(prep, chains=32, burnin=10, sweeps=100, groups=32, seed=300 + r, vjp_v=v,
                      want_cross=(r == 0), threads=4)
        if r == 0:
            assert np.allclose(res.vjp, orc.vjp(res, v), rtol=1e-8, atol=1e-10 * np.abs(ref).max())
        z[r] = (res.vjp[ms] - ref[ms]) / res.vjp_se[ms]
    for j in range(len(ms)):
        q = float(np.sum(z[:, j] ** 2))
        assert lo < q < hi, (ms[j], q, lo, hi)
        assert abs(z[:, j].mean()) < 4.0 * z[:, j].std(ddof=1) / math.sqrt(R)


# --------------------------------------------------------------------------------------
# invariants and structural limits
# --------------------------------------------------------------------------------------

def test_incremental_residual_matches_recomputed(orc):
    p = workloads.small_problem(M=41, N=24, nblocks=2)
    prep = orc.prepare(p)
    res = orc.run(prep, chains=2, burnin=0, sweeps=1000, refresh_every=0, groups=2,
                  traj_chain=0)
    A = res.final_A[0]
    r = prep.gt - prep.Kt @ A
    assert np.linalg.norm(res.final_r[0] - r) <= 1e-10 * np.linalg.norm(r)
    assert abs(res.final_chi2[0] - r @ r) <= 1e-10 * (r @ r)
    assert np.all(res.traj_A >= 0.0)
    chi2_traj = np.array([np.sum((prep.gt - prep.Kt @ a) ** 2) for a in res.traj_A])
    assert np.max(np.abs(chi2_traj - res.traj_chi2) / chi2_traj) < 1e-10


def _components_reference(Kt, gt, f0, seed, sweeps):
    """Components sampling of Eq. (CompChi), written independently (scipy truncnorm)."""
    import oracle as orc
    f = f0.copy()
    traj = []
    for s in range(sweeps):
        for n in range(len(f)):
            kn = Kt[:, n]
            r = gt - Kt @ f
            nn = kn @ kn
            mu = f[n] + (kn @ r) / nn
            sd = 1.0 / math.sqrt(nn)
            u = orc.move_uniform(seed, 0, 0, s, n, 0)
            f[n] = stats.truncnorm.ppf(u, (0.0 - mu) / sd, np.inf, loc=mu, scale=sd)
        traj.append(f.copy())
    return np.array(traj)


def test_one_point_blocks_are_components_sampling(orc):
    beta = 10.0
    tau = workloads.imaginary_times(9, beta)
    x = np.array([-1.0, 0.0, 1.0, 2.0])
    K = workloads.fermionic_kernel(tau, x, beta)
    sig = 0.02
    G = K @ np.array([0.2, 0.4, 0.1, 0.3]) + sig * np.random.default_rng(4).standard_normal(9)
    p = _problem(K, G, sig, [0, 1, 2, 3, 4])
    prep = orc.prepare(p)
    res = orc.run(prep, chains=1, burnin=0, sweeps=20, refresh_every=0, groups=1, traj_chain=0,
                  seed=77)
    ref = _components_reference(prep.Kt, prep.gt, prep.init, 77, 20)
    assert np.max(np.abs(res.traj_A - ref)) < 1e-8 * np.max(np.abs(ref))


def test_single_block_is_modes_sampling_in_e_space(orc):
    """Modes sampling of Sec. IV.B in the e = V^T f basis, written independently."""
    rng = np.random.default_rng(21)
    M, N = 5, 8
    K = rng.standard_normal((M, N)) + 0.5
    G = K @ rng.uniform(0.2, 1.0, N)
    p = _problem(K, G, 0.5, [0, N])
    prep = orc.prepare(p)
    seed = 5
    res = orc.run(prep, chains=1, burnin=0, sweeps=10, refresh_every=0, groups=1, traj_chain=0,
                  seed=seed)
    V = prep.V[0]
    kb = int(prep.kb[0])
    d = np.zeros(N)
    d[:kb] = prep.d[0]
    h = np.zeros(N)
    h[:kb] = prep.U[0].T @ prep.gt
    f = prep.init.copy()
    traj = []
    for s in range(10):
        for i in range(N):
            e = V.T @ f
            Vi = V[:, i]
            # Eq. (modeLimits): max{f/V | V<0} <= e_i - e_i' <= min{f/V | V>0}
            lo_d = np.max(f[Vi < 0] / Vi[Vi < 0]) if np.any(Vi < 0) else -np.inf
            hi_d = np.min(f[Vi > 0] / Vi[Vi > 0]) if np.any(Vi > 0) else np.inf
            lo_e, hi_e = e[i] - hi_d, e[i] - lo_d
            u = orc.move_uniform(seed, 0, 0, s, 0, i)
            if d[i] > 0:
                mu, sd = h[i] / d[i], 1.0 / d[i]
                en = stats.truncnorm.ppf(u, (lo_e - mu) / sd, (hi_e - mu) / sd, loc=mu, scale=sd)
            else:
                en = lo_e + u * (hi_e - lo_e)
            f = np.maximum(f + (en - e[i]) * Vi, 0.0)
        traj.append(f.copy())
    traj = np.array(traj)
    assert np.max(np.abs(res.traj_A - traj)) < 1e-7 * np.max(np.abs(traj))


def test_block_factors_are_an_orthonormal_svd(orc):
    p = workloads.single_continuation()
    prep = orc.prepare(p)
    for b in range(prep.B):
        s0, s1 = prep.bstart[b], prep.bstart[b + 1]
        Kb = prep.Kt[:, s0:s1]
        V = prep.V[b]
        kb = prep.kb[b]
        assert 1 <= kb <= 20
        assert np.allclose(V.T @ V, np.eye(V.shape[0]), atol=1e-12)
        assert np.allclose(Kb @ V[:, :kb], prep.U[b] * prep.d[b][None, :],
                           atol=1e-10 * prep.d[b][0])
        # the completion spans the numerical null space
        assert np.linalg.norm(Kb @ V[:, kb:]) < 1e-6 * prep.d[b][0]
        w = np.arange(1, V.shape[0] + 1)
        assert np.all(w @ V[:, :kb] > 0)


def test_width_factor_invariance(orc):
    """Eq. (Itrafo): sampling (K W, A) or (K, W A) gives <W A> = W <A>."""
    beta = 10.0
    tau = workloads.imaginary_times(11, beta)
    x, w = workloads.uniform_midpoint_grid(-3.0, 3.0, 6)
    w = w * np.array([0.5, 1.0, 2.0, 1.5, 0.7, 1.2])
    Kraw = workloads.fermionic_kernel(tau, x, beta)
    A = workloads.gaussian_mixture(x, (1.0,), (0.0,), (1.0,))
    sig = 0.02
    G = Kraw @ (A * w) + sig * np.random.default_rng(12).standard_normal(11)
    pa = _problem(Kraw * w[None, :], G, sig, [0, 3, 6])
    pf = _problem(Kraw, G, sig, [0, 3, 6])
    ra = orc.run(orc.prepare(pa), chains=32, burnin=200, sweeps=6000, groups=32)
    rf = orc.run(orc.prepare(pf), chains=32, burnin=200, sweeps=6000, groups=32, seed=4321)
    z = np.abs(rf.mean - w * ra.mean) / np.sqrt(rf.stderr ** 2 + (w * ra.stderr) ** 2)
    assert np.max(z) < 4.5, z


def test_cross_moment_equals_minus_K_cov(orc):
    """r~ is affine in A, so Cov(r~, A) = -K~ Cov(A, A) exactly for the sample moments."""
    p = workloads.small_problem(M=21, N=12, nblocks=2, sigma=1e-2)
    prep = orc.prepare(p)
    res = orc.run(prep, chains=1, burnin=50, sweeps=3000, refresh_every=16, groups=8,
                  want_cross=True, traj_chain=0)
    A = res.traj_A[50:]
    mA = A.mean(0)
    covAA = (A - mA).T @ (A - mA) / len(A)
    ref = -prep.Kt @ covAA
    assert np.max(np.abs(res.cov_rA - ref)) < 1e-8 * np.max(np.abs(ref))


def test_vjp_against_common_random_number_differences(orc):
    """v . (<A>(G + h u) - <A>(G - h u)) / 2h  ==  (J^T v) . u  (same random numbers)."""
    p = workloads.small_problem(M=21, N=10, nblocks=2, sigma=2e-2, seed=31)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(p.N)
    u = rng.standard_normal(p.M)
    u /= np.linalg.norm(u)
    kw = dict(chains=64, burnin=300, sweeps=3000, groups=32, seed=2024)
    base = orc.run(orc.prepare(p), want_cross=True, **kw)
    jv = orc.vjp(base, v)
    h = 1e-3 * p.sigma[0]
    outs = []
    for sgn in (+1, -1):
        q = workloads.Problem(K=p.K, G=p.G + sgn * h * u, sigma=p.sigma, block_start=p.block_start)
        outs.append(orc.run(orc.prepare(q), **kw).mean @ v)
    fd = (outs[0] - outs[1]) / (2 * h)
    assert abs(fd - jv @ u) < 0.1 * max(abs(fd), np.linalg.norm(jv) * 0.1), (fd, jv @ u)


def test_unbounded_zero_mode_is_reported(orc):
    # a null-space direction with all-positive entries makes the posterior improper
    K = np.array([[1.0, -1.0]])
    p = _problem(K, [0.0], 1.0, [0, 2])
    res = orc.run(orc.prepare(p), chains=1, sweeps=2, groups=1)
    assert res.status == -4


# --------------------------------------------------------------------------------------
# the paper's own test case (Sec. III) and its efficiency comparison (Fig. 3)
# --------------------------------------------------------------------------------------

def test_conductivity_workload_sum_rule_and_kernel():
    """Pi(i omega_0) is the sum rule (2/pi) int sigma (Eq. (optcond) at omega_m = 0): the
    generator's fine-grid data against adaptive quadrature of Eq. (model); the kernel's first
    row is (2/pi) times the grid weights."""
    p = workloads.optical_conductivity(40, 4, sigma_rel=0.0)
    total, _ = integrate.quad(lambda x: workloads.conductivity_model(np.array([x]))[0], 0.0, np.inf,
                              limit=400)
    assert abs(p.G[0] - 2.0 / math.pi * total) < 1e-7 * p.G[0]
    wm1 = 2.0 * math.pi / 15.0
    f = lambda x: (2.0 / math.pi) * x * x / (wm1 * wm1 + x * x) * workloads.conductivity_model(np.array([x]))[0]
    v1, _ = integrate.quad(f, 0.0, np.inf, limit=400)
    assert abs(p.G[1] - v1) < 1e-7 * p.G[1]
    assert np.allclose(p.K[0], 2.0 / math.pi * 0.1, rtol=1e-15)
    assert np.all(np.diff(p.G) < 0)


def _median_step(orc, n, nblocks, sweeps=2500, skip=500):
    p = workloads.optical_conductivity(n, nblocks)
    prep = orc.prepare(p)
    r = orc.run(prep, chains=1, burnin=0, sweeps=sweeps, seed=5, groups=1, traj_chain=0,
                init=orc.nnls_start(prep), threads=1)
    A = r.traj_A
    d = np.linalg.norm(np.diff(A, axis=0), axis=1) / np.linalg.norm(A[:-1], axis=1)
    return float(np.median(d[skip:]))


def test_step_sizes_order_as_in_fig3(orc):
    """Fig. 3 / Sec. IV.D, on the optical-conductivity test case with accurate data: with the
    small cutoff (40 points) modes and blocked modes take comparable steps and components
    exceedingly small ones; with the large cutoff (120 points, the tail on the grid) the steps of
    modes sampling collapse, below those of components, while blocked modes keep moving.
    Delta_i = |f(i+1) - f(i)| / |f(i)| per sweep, median over one chain's sweeps; blocked modes
    here use one fixed partition of 4 blocks."""
    c40, m40, b40 = (_median_step(orc, 40, nb) for nb in (40, 1, 4))
    c120, m120, b120 = (_median_step(orc, 120, nb) for nb in (120, 1, 4))
    assert c40 < 0.2 * m40 and c40 < 0.2 * b40
    assert 0.3 < m40 / b40 < 3.0
    assert m120 < c120 < 0.2 * b120
    assert m120 < 0.01 * b120


def test_hierarchy_steps_as_in_fig3(orc):
    """Fig. 3 with the paper's own blocked modes, a random level of the Fig. 2 hierarchy per
    sweep: large steps on both grids, far above components (40 points) and modes (120
    points); the sweeps on the top level (modes of the full grid) and the bottom level
    (components) take the small steps the paper remarks on."""
    for n, small in ((40, 0.0075), (120, 0.0092)):
        p = workloads.optical_conductivity(n, 1)
        p.levels = orc.hierarchy(n)
        prep = orc.prepare(p)
        r = orc.run(prep, chains=1, burnin=0, sweeps=2500, seed=5, groups=1, traj_chain=0,
                    init=orc.nnls_start(prep), threads=1)
        A = r.traj_A
        d = np.linalg.norm(np.diff(A, axis=0), axis=1) / np.linalg.norm(A[:-1], axis=1)
        lv = np.array([orc.sweep_level(5, 0, s, len(prep.levels)) for s in range(1, 2500)])
        med = float(np.median(d[500:]))
        assert med > 10 * small, (n, med)
        lv = lv[500:]                     # d[i]: the move of sweep i + 1
        mid = np.median(d[500:][(lv > 0) & (lv < len(prep.levels) - 1)])
        ends = np.median(d[500:][(lv == 0) | (lv == len(prep.levels) - 1)])
        assert ends < 0.5 * mid, (n, ends, mid)


# --------------------------------------------------------------------------------------
# gamma-prior weights (Sec. V.C): prod_n A_n^(w_n - 1) exp(-chi^2 / 2), Eq. (compat)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("w", [0.5, 2.5])
def test_gamma_prior_one_point_against_quadrature(orc, w):
    """N = 1: density f^(w-1) exp(-(f - mu)^2 / 2 s^2) on f > 0, mean by quadrature."""
    rng = np.random.default_rng(13)
    k = rng.uniform(0.5, 1.5, 7)
    s = 1.0 / np.linalg.norm(k)
    for mu_over_s in [-1.0, 0.5, 3.0]:
        mu = mu_over_s * s
        p = _problem(k[:, None], k * mu, 1.0, [0, 1])
        p.prior_shape = np.array([w])
        res = orc.run(orc.prepare(p), chains=16, burnin=50, sweeps=20000, groups=16)
        dens = lambda f, j: f ** (w - 1 + j) * math.exp(-0.5 * ((f - mu) / s) ** 2)
        up = max(mu, 0) + 12 * s
        Z = integrate.quad(lambda f: dens(f, 0), 0, up, points=[s * 1e-3, s], limit=400)[0]
        ref = integrate.quad(lambda f: dens(f, 1), 0, up, points=[s * 1e-3, s], limit=400)[0] / Z
        assert _within(res.mean, res.stderr, ref) < 4.5, (w, mu_over_s, res.mean, ref)
        assert 0 < res.n_rejected < 20000 * 16


@pytest.mark.parametrize("w", [0.5, 2.0])
def test_gamma_prior_sum_rule_closed_form(orc, w):
    """K = 1^T, g = 1: S = sum A has density S^(N w - 1) exp(-(S - 1)^2 / 2 sigma^2) and
    A / S ~ Dirichlet(w, ..., w), so <A_n> = E[S] / N and <A_n^2> = E[S^2] (w + 1) / (N (N w + 1))."""
    N, sig = 8, 0.3
    ws = lambda S, j: S ** (N * w - 1 + j) * math.exp(-0.5 * ((S - 1.0) / sig) ** 2)
    Z = integrate.quad(lambda S: ws(S, 0), 0, 10, points=[1e-3, 1.0], limit=400)[0]
    ES = integrate.quad(lambda S: ws(S, 1), 0, 10, limit=400)[0] / Z
    ES2 = integrate.quad(lambda S: ws(S, 2), 0, 10, limit=400)[0] / Z
    EA = ES / N
    EA2 = ES2 * (w + 1) / (N * (N * w + 1))
    p = _problem(np.ones((1, N)), [1.0], sig, [0, 4, 8])
    p.prior_shape = np.full(N, w)
    res = orc.run(orc.prepare(p), chains=16, burnin=500, sweeps=40000, groups=16)
    assert _within(res.mean, res.stderr, EA) < 4.5, (res.mean, EA)
    assert np.allclose(res.post_sd, math.sqrt(EA2 - EA * EA), rtol=0.04), (res.post_sd, math.sqrt(EA2 - EA * EA))


def test_gamma_prior_halved_grid_reproduces_the_flat_coarse_grid(orc):
    """Eq. (genconsistency) / Eq. (compat): each interval of a 3-point grid split in two halves
    of the same kernel value (columns K_j / 2) and sampled with shape w = 1/2 per half gives,
    for the pair averages, the flat-prior average of the coarse grid (two gamma(1/2) weights
    convolve to the flat one), exactly up to Monte Carlo error."""
    beta = 10.0
    tau = workloads.imaginary_times(11, beta)
    x = np.array([-1.5, 0.0, 1.5])
    Kc = workloads.fermionic_kernel(tau, x, beta)
    sig = 0.05
    G = Kc @ np.array([0.3, 0.05, 0.2]) + sig * np.random.default_rng(9).standard_normal(11)
    coarse = orc.run(orc.prepare(_problem(Kc, G, sig, [0, 3])), chains=32, burnin=200,
                     sweeps=20000, groups=32)
    Kf = np.repeat(Kc / 2.0, 2, axis=1)
    pf = _problem(Kf, G, sig, [0, 6])
    pf.prior_shape = np.full(6, 0.5)
    fine = orc.run(orc.prepare(pf), chains=32, burnin=200, sweeps=20000, groups=32)
    pair = fine.group_means.reshape(32, 3, 2).mean(axis=2)
    pm, pse = pair.mean(0), pair.std(0, ddof=1) / math.sqrt(32)
    z = np.abs(pm - coarse.mean) / np.sqrt(pse ** 2 + coarse.stderr ** 2)
    assert np.max(z) < 4.5, (pm, coarse.mean, z)
    # the flat prior on the fine grid gives a different answer (the grid dependence of Sec. V)
    pflat = _problem(Kf, G, sig, [0, 6])
    flat = orc.run(orc.prepare(pflat), chains=32, burnin=200, sweeps=20000, groups=32)
    fp = flat.group_means.reshape(32, 3, 2).mean(axis=2)
    zf = np.abs(fp.mean(0) - coarse.mean) / np.sqrt((fp.std(0, ddof=1) / math.sqrt(32)) ** 2 + coarse.stderr ** 2)
    assert np.max(zf) > 6, (fp.mean(0), coarse.mean, zf)


# --------------------------------------------------------------------------------------
# a linear constraint c . A = F (Sec. IV.E): moves restricted to the complement of c
# --------------------------------------------------------------------------------------

def _flat_likelihood_problem(N, bstart, c, F):
    rng = np.random.default_rng(2)
    K = rng.uniform(0.1, 1.0, (3, N))
    p = _problem(K, K @ np.ones(N), 1e7, bstart)   # sigma 1e7: chi^2 is flat on the scale of F
    p.constraint_c = np.asarray(c, np.float64)
    p.constraint_value = float(F)
    return p


@pytest.mark.parametrize("levels", [False, True])
def test_constraint_flat_likelihood_is_uniform_on_the_simplex(orc, levels):
    """With a flat likelihood, A >= 0 and c . A = F make B_n = c_n A_n / F uniform on the
    standard simplex: <A_n> = F / (N c_n), Var A_n = F^2 (N - 1) / (N^2 (N + 1) c_n^2)."""
    N, F = 6, 2.0
    c = np.array([1.0, 0.5, 2.0, 1.0, 1.5, 0.8])
    p = _flat_likelihood_problem(N, [0, N], c, F)
    if levels:
        p.levels = orc.hierarchy(N)
    prep = orc.prepare(p)
    assert list(prep.nm)[:1] == [N - 1]
    res = orc.run(prep, chains=16, burnin=200, sweeps=20000, groups=16, traj_chain=3)
    ref = F / (N * c)
    assert _within(res.mean, res.stderr, ref) < 4.5, (res.mean, ref)
    sd = F * math.sqrt((N - 1) / (N * N * (N + 1))) / c
    assert np.allclose(res.post_sd, sd, rtol=0.04), (res.post_sd, sd)
    # every state of the trajectory keeps the constraint
    assert np.max(np.abs(res.traj_A @ c - F)) < 1e-12 * F
    assert np.min(res.traj_A) >= 0.0


def test_constraint_two_point_grid_against_quadrature(orc):
    """Two points with A_1 + A_2 = F: the posterior lives on the segment t = A_1 in [0, F]."""
    beta = 10.0
    tau = workloads.imaginary_times(11, beta)
    x = np.array([-1.0, 0.5])
    K = workloads.fermionic_kernel(tau, x, beta)
    sig = 0.05
    G = K @ np.array([0.3, 0.2]) + sig * np.random.default_rng(8).standard_normal(11)
    F = 0.5
    p = _problem(K, G, sig, [0, 2])
    p.constraint_c = np.ones(2)
    p.constraint_value = F
    res = orc.run(orc.prepare(p), chains=16, burnin=100, sweeps=20000, groups=16)
    Kt, gt = K / sig, G / sig
    w = lambda t: math.exp(-0.5 * np.sum((gt - Kt[:, 0] * t - Kt[:, 1] * (F - t)) ** 2))
    lw = [math.log(w(t) + 1e-300) for t in np.linspace(0, F, 201)]
    shift = max(lw)
    Z = integrate.quad(lambda t: w(t) * math.exp(-shift), 0, F, epsabs=0, epsrel=1e-12, limit=200)[0]
    m1 = integrate.quad(lambda t: t * w(t) * math.exp(-shift), 0, F, epsabs=0, epsrel=1e-12, limit=200)[0] / Z
    ref = np.array([m1, F - m1])
    assert _within(res.mean, res.stderr, ref) < 4.5, (res.mean, ref)


def test_data_noise_is_standard_normal(orc):
    """The start's data noise (Box-Muller on Philox words) against the normal distribution."""
    xi = orc.data_noise(77, 2, 20000)
    assert abs(xi.mean()) < 4.5 / math.sqrt(20000)
    assert abs(xi.var() - 1.0) < 4.5 * math.sqrt(2.0 / 20000)
    assert stats.kstest(xi, "norm").pvalue > 1e-4
    assert not np.array_equal(xi[:100], orc.data_noise(77, 3, 100))


def test_correlated_bounds_cover_the_oracle_against_oracle_spread():
    """The pass bounds for correlated spectra sit above what independent oracle runs give
    against the stored references (tests/golden/calibrate_correlated.py, oracle only)."""
    import json
    import os
    from parity_criteria import CORRELATED
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "correlated_calibration.json")
    cal = json.load(open(here))
    assert cal["replicas"] >= 12 and len(cal["datasets"]) == 3
    assert cal["max_of_max_z"] < CORRELATED["zmax"]
    assert cal["max_frac3"] < CORRELATED["frac"]
    assert cal["max_mean_z2"] < CORRELATED["mean_z2"]


@pytest.mark.parametrize("M,N,nblocks,k", [(224, 256, 2, 20), (416, 300, 3, 27)])
def test_rank_limited_blocks_have_the_stated_rank(orc, M, N, nblocks, k):
    """The rank-limited input generator (used at the eight-lane sampler's limits) gives blocks of
    numerical rank k exactly: k singular values well above the rank threshold max(M, N_b) eps d_1
    of Sec. IV.B-C's data-mode cut and the rest at rounding level, so the oracle's data-mode count
    is k on every block."""
    p = workloads.rank_limited(M, N, nblocks, k, seed=2)
    prep = orc.prepare(p)
    assert list(prep.kb) == [k] * nblocks
    for b in range(nblocks):
        Kb = prep.Kt[:, int(p.block_start[b]):int(p.block_start[b + 1])]
        s = np.linalg.svd(Kb, compute_uv=False)
        thr = max(Kb.shape) * np.finfo(float).eps * s[0]
        assert s[k - 1] > 1e6 * thr and s[k] < 0.1 * thr
