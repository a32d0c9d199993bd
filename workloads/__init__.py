"""Seeded synthetic problem generators shared by the oracle, the tests and the bench.

This module only *builds inputs*: an imaginary-time kernel matrix on a real-frequency
grid, a model spectrum, and noisy data drawn from it.  It contains none of the
arithmetic of the average spectrum method itself (no whitening, no decomposition,
no sampling), so that the CPU oracle and the GPU library can both consume its
output without sharing any of the method's code.

Physics conventions (Ghanem & Koch, arXiv:1912.01379):
  * fermionic imaginary-time kernel, Sec. II: K(tau, w) = exp(-tau w) / (1 + exp(-beta w));
    the overall -1/(2 pi) factor of the paper is dropped, so the spectra are
    non-negative and normalised to one;
  * piecewise-constant discretisation with Riemann weights w_n = 1 / (N rho(x_n)),
    Sec. V.B, Eq. (Riemann): the weights are folded into the kernel columns, so the
    sampled variable is the spectrum A(w_n) itself (the paper shows in Eq. (Itrafo)
    that folding them into the model instead gives the same average);
  * grid points x_n = P^{-1}(z_n) on the mid-points z_n = (n - 1/2)/N, Sec. V.B.

Every generator is deterministic in its seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

BASE_SEED = 1912013790


# --------------------------------------------------------------------------------------
# kernels and grids
# --------------------------------------------------------------------------------------

def fermionic_kernel(tau: np.ndarray, omega: np.ndarray, beta: float) -> np.ndarray:
    """exp(-tau w)/(1+exp(-beta w)) evaluated without overflow (M x N, float64).

    For w < 0 numerator and denominator are multiplied by exp(beta w), giving
    exp((beta - tau) w)/(1 + exp(beta w)); both forms are the same function.
    """
    t = np.asarray(tau, dtype=np.float64)[:, None]
    w = np.asarray(omega, dtype=np.float64)[None, :]
    pos = w >= 0
    out = np.empty((t.shape[0], w.shape[1]), dtype=np.float64)
    wp = np.where(pos, w, 0.0)
    wn = np.where(pos, 0.0, w)
    kp = np.exp(-t * wp) / (1.0 + np.exp(-beta * wp))
    kn = np.exp((beta - t) * wn) / (1.0 + np.exp(beta * wn))
    out[:] = np.where(pos, kp, kn)
    return out


def uniform_midpoint_grid(lo: float, hi: float, n: int):
    """Uniform grid w_n = lo + (n - 1/2) dw with constant weights dw."""
    dw = (hi - lo) / n
    x = lo + (np.arange(n, dtype=np.float64) + 0.5) * dw
    return x, np.full(n, dw)


def lorentzian_grid(n: int, gamma: float = 2.0, cutoff: float = 10.0):
    """Grid with Lorentzian density on [-cutoff, cutoff] (Sec. V.B table, truncated).

    CDF P(x) = (atan(x/g) + atan(c/g)) / (2 atan(c/g)); x_n = P^{-1}(z_n);
    weight w_n = 1/(N rho(x_n)) with rho = P'.
    """
    z = (np.arange(n, dtype=np.float64) + 0.5) / n
    th = math.atan(cutoff / gamma)
    x = gamma * np.tan((2.0 * z - 1.0) * th)
    rho = (1.0 / (2.0 * th)) * (1.0 / gamma) / (1.0 + (x / gamma) ** 2)
    return x, 1.0 / (n * rho)


def imaginary_times(m: int, beta: float) -> np.ndarray:
    """m points uniform on [0, beta], both ends included."""
    return np.linspace(0.0, beta, m)


def gaussian_mixture(x, weights, centres, sds):
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for a, c, s in zip(weights, centres, sds):
        out += a * np.exp(-0.5 * ((x - c) / s) ** 2) / (s * math.sqrt(2.0 * math.pi))
    return out


def ar1_noise(rng: np.random.Generator, m: int, sigma: float, length: float) -> np.ndarray:
    """Gaussian noise with covariance sigma^2 exp(-|i-j|/length), drawn as an AR(1) process."""
    rho = math.exp(-1.0 / length)
    e = rng.standard_normal(m)
    out = np.empty(m)
    out[0] = sigma * e[0]
    s = math.sqrt(1.0 - rho * rho)
    for i in range(1, m):
        out[i] = rho * out[i - 1] + sigma * s * e[i]
    return out


def exp_covariance(m: int, sigma: float, length: float) -> np.ndarray:
    idx = np.arange(m, dtype=np.float64)
    return sigma * sigma * np.exp(-np.abs(idx[:, None] - idx[None, :]) / length)


def equal_blocks(n: int, nblocks: int) -> np.ndarray:
    """Block offsets s_0 = 0 < ... < s_B = n splitting n points into nearly equal blocks."""
    return np.array([(b * n) // nblocks for b in range(nblocks + 1)], dtype=np.int64)


# --------------------------------------------------------------------------------------
# problem container
# --------------------------------------------------------------------------------------

@dataclass
class Problem:
    """One analytic-continuation problem: G = K A + noise, A >= 0."""
    K: np.ndarray                      # M x N (weights folded in)
    G: np.ndarray                      # M
    sigma: Optional[np.ndarray] = None  # M (iid noise) or None
    cov: Optional[np.ndarray] = None    # M x M or None
    omega: Optional[np.ndarray] = None  # N grid points
    weights: Optional[np.ndarray] = None
    block_start: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    k: Optional[np.ndarray] = None      # requested data modes per block (None -> numerical rank)
    A_true: Optional[np.ndarray] = None
    name: str = ""
    prior_shape: Optional[np.ndarray] = None   # N gamma-prior shapes w_n (Eq. (compat));
                                        # None: the flat prior (w = 1)
    constraint_c: Optional[np.ndarray] = None  # N: a linear constraint c . A = F (Sec. IV.E)
    constraint_value: float = 0.0       # F
    levels: Optional[list] = None       # a hierarchy of partitions (each B_l+1 offsets), used
                                        # instead of block_start when given; k then covers the
                                        # blocks of all levels in order

    def partitions(self) -> list:
        if self.levels is not None:
            return [np.asarray(ls, np.int64) for ls in self.levels]
        return [np.asarray(self.block_start, np.int64)]

    @property
    def M(self) -> int:
        return int(self.K.shape[0])

    @property
    def N(self) -> int:
        return int(self.K.shape[1])

    @property
    def B(self) -> int:
        return int(sum(len(ls) - 1 for ls in self.partitions()))


def _finish(K, A_true, rng, sigma=None, cov_len=None, **kw) -> Problem:
    g_exact = K @ A_true
    M = K.shape[0]
    if cov_len is None:
        s = np.full(M, float(sigma))
        G = g_exact + s * rng.standard_normal(M)
        return Problem(K=K, G=G, sigma=s, A_true=A_true, **kw)
    G = g_exact + ar1_noise(rng, M, float(sigma), float(cov_len))
    return Problem(K=K, G=G, cov=exp_covariance(M, float(sigma), float(cov_len)),
                   A_true=A_true, **kw)


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------

SINGLE_SPECTRUM = dict(weights=(0.30, 0.25, 0.25, 0.20), centres=(-3.0, -0.8, 2.5, 0.3),
                     sds=(0.8, 0.4, 1.0, 0.05))


def plain_one_chain(seed: int = BASE_SEED + 1) -> Problem:
    """Plain modes sampling: beta=10, 41 times, 100 uniform points on [-5,5], one block."""
    beta = 10.0
    tau = imaginary_times(41, beta)
    x, w = uniform_midpoint_grid(-5.0, 5.0, 100)
    a = gaussian_mixture(x, (0.4, 0.6), (-1.5, 2.0), (0.4, 0.8))
    a = a / np.sum(a * w)
    K = fermionic_kernel(tau, x, beta) * w[None, :]
    rng = np.random.default_rng(seed)
    return _finish(K, a, rng, sigma=1e-3, omega=x, weights=w,
                   block_start=equal_blocks(100, 1), k=None, name="plain-one-chain")


def single_continuation(seed: int = BASE_SEED + 2) -> Problem:
    """Single continuation, blocked modes: beta=20, 201 times, 800 Lorentzian points, 8 blocks."""
    beta = 20.0
    tau = imaginary_times(201, beta)
    x, w = lorentzian_grid(800, 2.0, 10.0)
    a = gaussian_mixture(x, **SINGLE_SPECTRUM)
    a = a / np.sum(a * w)
    K = fermionic_kernel(tau, x, beta) * w[None, :]
    rng = np.random.default_rng(seed)
    return _finish(K, a, rng, sigma=1e-4, omega=x, weights=w,
                   block_start=equal_blocks(800, 8), k=np.full(8, 20, np.int32),
                   name="single-continuation")


def batched_dataset(index: int, base_seed: int = BASE_SEED + 3) -> Problem:
    """One of the 256 uneven continuations of the batched workload."""
    rng = np.random.default_rng(base_seed * 1000 + index)
    M = int(rng.integers(51, 202))
    N = int(rng.integers(200, 1001))
    beta = float(rng.choice([10.0, 20.0, 40.0]))
    ng = int(rng.integers(2, 5))
    centres = rng.uniform(-6.0, 6.0, ng)
    sds = rng.uniform(0.2, 1.5, ng)
    wts = rng.dirichlet(np.ones(ng))
    sigma = 10.0 ** rng.uniform(-5.0, -3.0)
    tau = imaginary_times(M, beta)
    x, w = lorentzian_grid(N, 2.0, 10.0)
    a = gaussian_mixture(x, wts, centres, sds)
    a = a / np.sum(a * w)
    K = fermionic_kernel(tau, x, beta) * w[None, :]
    B = max(1, int(round(N / 100.0)))
    bs = equal_blocks(N, B)
    k = np.array([min(20, int(bs[b + 1] - bs[b])) for b in range(B)], np.int32)
    return _finish(K, a, rng, sigma=sigma, omega=x, weights=w, block_start=bs, k=k,
                   name=f"batched-{index}")


def batched_datasets(n: int = 256) -> list:
    return [batched_dataset(i) for i in range(n)]


def differentiation_cotangent(N: int, seed: int = BASE_SEED + 4) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(N)


def gaussian_limit_problem(omega=(-3.0, -1.0, 1.0, 3.0), sigma: float = 0.1, level: float = 2.0,
                           seed: int = BASE_SEED + 40) -> Problem:
    """Few-point problem on the cfg-2 kernel where positivity is practically inactive."""
    beta = 20.0
    tau = imaginary_times(201, beta)
    x = np.asarray(omega, dtype=np.float64)
    K = fermionic_kernel(tau, x, beta)
    a = np.full(len(x), level)
    rng = np.random.default_rng(seed)
    return _finish(K, a, rng, sigma=sigma, omega=x, weights=np.ones(len(x)),
                   block_start=equal_blocks(len(x), 1), k=None, name="gauss-limit")


def large_workload(seed: int = BASE_SEED + 5) -> Problem:
    """Large: beta=50, 401 times, 4000 Lorentzian points, 32 blocks, correlated noise."""
    beta = 50.0
    tau = imaginary_times(401, beta)
    x, w = lorentzian_grid(4000, 2.0, 10.0)
    a = gaussian_mixture(x, **SINGLE_SPECTRUM)
    a = a / np.sum(a * w)
    K = fermionic_kernel(tau, x, beta) * w[None, :]
    rng = np.random.default_rng(seed)
    return _finish(K, a, rng, sigma=1e-4, cov_len=5.0, omega=x, weights=w,
                   block_start=equal_blocks(4000, 32), k=np.full(32, 30, np.int32),
                   name="large")


# --------------------------------------------------------------------------------------
# the paper's own test case (Sec. III): the optical conductivity from bosonic Matsubara data
# --------------------------------------------------------------------------------------

def conductivity_model(omega: np.ndarray, model: int = 1) -> np.ndarray:
    """sigma(omega) of Eq. (model): a Drude peak (weight 0.3, width 0.3 for model 1, 0.6 for
    model 2) and two peaks of weight 0.2 and width 1.2 at +-3, cut off by 1/(1 + (w/4)^6)."""
    ge, w0, w1, g1, e1 = 4.0, 0.3, 0.2, 1.2, 3.0
    g0 = 0.3 if model == 1 else 0.6
    peaks = (w0 / (1.0 + (omega / g0) ** 2) + w1 / (1.0 + ((omega + e1) / g1) ** 2)
             + w1 / (1.0 + ((omega - e1) / g1) ** 2))
    return peaks / (1.0 + (omega / ge) ** 6)


def bosonic_kernel(omega_m: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """K(i omega_m, omega) = (2/pi) omega^2 / (omega_m^2 + omega^2) of Eq. (optcond)."""
    w2 = omega[None, :] ** 2
    return (2.0 / np.pi) * w2 / (omega_m[:, None] ** 2 + w2)


def optical_conductivity(n_omega: int = 40, nblocks: int = 4, model: int = 1,
                         sigma_rel: float = 1e-3, beta: float = 15.0, n_matsubara: int = 60,
                         seed: int = BASE_SEED + 6, step: float = 0.1, grid=None) -> Problem:
    """The test case of Sec. III and Fig. 3: Pi(i omega_m) of Eq. (optcond) at the first 60
    bosonic Matsubara frequencies (beta = 15) from sigma(omega) of Eq. (model), with relative
    Gaussian noise of standard deviation sigma_rel; the grid is omega_n = 0.1 (n - 1/2),
    n = 1..n_omega (40: small cutoff, 120: large), split into nblocks equal blocks (1: modes
    sampling, n_omega: components sampling).  The data come from the continuous integral
    (a fine mid-point rule up to omega = 400), not from the grid, so grids of another spacing
    (`step`) see the same data."""
    wm = 2.0 * np.pi * np.arange(n_matsubara) / beta
    if grid is None:
        x = step * (np.arange(1, n_omega + 1) - 0.5)
        w = np.full(n_omega, step)
    else:   # (points, weights) of another grid on [0, inf)
        x, w = (np.asarray(a, np.float64) for a in grid)
        n_omega = len(x)
    K = bosonic_kernel(wm, x) * w[None, :]
    xf = (np.arange(400000) + 0.5) * 1e-3
    pi_exact = bosonic_kernel(wm, xf) @ (conductivity_model(xf, model) * 1e-3)
    rng = np.random.default_rng(seed)
    sig = sigma_rel * np.abs(pi_exact)
    G = pi_exact + sig * rng.standard_normal(n_matsubara)
    return Problem(K=K, G=G, sigma=sig, omega=x, weights=w, block_start=equal_blocks(n_omega, nblocks),
                   k=None, A_true=conductivity_model(x, model), name=f"optcond-{n_omega}-{nblocks}")


def small_problem(M: int = 41, N: int = 24, nblocks: int = 2, sigma: float = 1e-3,
                  beta: float = 10.0, seed: int = BASE_SEED + 7, k=None) -> Problem:
    """A small version of the cfg-1 problem used by parity tests (several blocks)."""
    tau = imaginary_times(M, beta)
    x, w = uniform_midpoint_grid(-5.0, 5.0, N)
    a = gaussian_mixture(x, (0.4, 0.6), (-1.5, 2.0), (0.4, 0.8))
    a = a / np.sum(a * w)
    K = fermionic_kernel(tau, x, beta) * w[None, :]
    rng = np.random.default_rng(seed)
    return _finish(K, a, rng, sigma=sigma, omega=x, weights=w,
                   block_start=equal_blocks(N, nblocks),
                   k=None if k is None else np.asarray(k, np.int32), name="small")


def rank_limited(M: int, N: int, nblocks: int, rank: int, seed: int = 13, sigma: float = 0.05) -> Problem:
    """Blocks of exactly the given numerical rank (each block's columns a random product of an
    M x rank and a rank x N_b Gaussian matrix), with that many data modes per block: the
    block kernels' remaining modes lie in their null spaces up to rounding, as in the
    fermionic kernel past its numerical rank, while the number of data modes is fixed by
    the input instead of by a singular-value decay."""
    rng = np.random.default_rng(seed)
    starts = equal_blocks(N, nblocks)
    K = np.zeros((M, N))
    for b in range(nblocks):
        lo, hi = int(starts[b]), int(starts[b + 1])
        K[:, lo:hi] = rng.standard_normal((M, rank)) @ rng.standard_normal((rank, hi - lo)) / math.sqrt(M * rank)
    a = 0.5 + rng.random(N)
    return _finish(K, a, rng, sigma=sigma, omega=np.arange(N, dtype=np.float64), weights=np.ones(N),
                   block_start=starts, k=np.full(nblocks, rank, np.int32), name="rank-limited")


def random_wellconditioned(M: int = 40, N: int = 24, nblocks: int = 2, seed: int = 11,
                           level: float = 1.0, sigma: float = 0.05) -> Problem:
    """Dense positive-and-negative kernel with well separated singular values.

    Used where two independent decompositions must agree to rounding: every block
    has distinct, well separated singular values and (for N_b <= M) no null space.
    """
    rng = np.random.default_rng(seed)
    K = rng.standard_normal((M, N)) / math.sqrt(M)
    a = level * (0.5 + rng.random(N))
    return _finish(K, a, rng, sigma=sigma, omega=np.arange(N, dtype=np.float64),
                   weights=np.ones(N), block_start=equal_blocks(N, nblocks), k=None,
                   name="wellcond")
