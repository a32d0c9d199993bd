"""Grids on [0, inf) from the table of Sec. V.B and the default model they imply (Sec. VI).

A grid of N points with density rho(x) = dz/dx puts x_n = x(z_n) at the mid-points
z_n = (n - 1/2) / N and weights w_n = 1 / (N rho(x_n)) (Eq. (Riemann)); the kernel columns carry
the weights.  Sampling on such a grid makes rho act as a default model (Sec. V.C); Sec. VI writes
the default optical conductivity as sigma_def = pi Pi(0) rho / 2, whose Matsubara data are

    Pi_def(omega_m) = Pi(0) (1 - int_0^inf rho(w) / (1 + (w / omega_m)^2) dw),

and picks the grid parameter that brings Pi_def closest to the data (Fig. 9).  Host code only.
"""
from __future__ import annotations

import math

import numpy as np

FAMILIES = ("gaussian", "exponential", "lorentzian", "uniform")


def density(family: str, par: float, x):
    """rho(x) of the grid family with parameter alpha, beta, gamma or the cutoff omega_c."""
    x = np.asarray(x, np.float64)
    if family == "gaussian":
        return np.exp(-x * x / (2.0 * par * par)) / (math.sqrt(2.0 * math.pi) * par / 2.0)
    if family == "exponential":
        return np.exp(-x / par) / par
    if family == "lorentzian":
        return (2.0 / (math.pi * par)) / (1.0 + (x / par) ** 2)
    if family == "uniform":
        return np.where((x >= 0.0) & (x <= par), 1.0 / par, 0.0)
    raise ValueError(family)


def points(family: str, par: float, z):
    """x(z), the inverse of the grid's distribution function."""
    from scipy import special
    z = np.asarray(z, np.float64)
    if family == "gaussian":
        return math.sqrt(2.0) * par * special.erfinv(z)
    if family == "exponential":
        return -par * np.log1p(-z)
    if family == "lorentzian":
        return par * np.tan(math.pi * z / 2.0)
    if family == "uniform":
        return par * z
    raise ValueError(family)


def grid(family: str, par: float, n: int):
    """(x_n, w_n) of an n-point grid (Eq. (Riemann))."""
    z = (np.arange(n, dtype=np.float64) + 0.5) / n
    x = points(family, par, z)
    return x, 1.0 / (n * density(family, par, x))


def default_model_data(family: str, par: float, pi0: float, omega_m) -> np.ndarray:
    """Pi_def(omega_m) of the default model sigma_def = pi Pi(0) rho / 2 (Sec. VI)."""
    from scipy import integrate
    out = []
    for wm in np.asarray(omega_m, np.float64):
        if wm == 0.0:
            out.append(pi0)
            continue
        f = lambda w: float(density(family, par, w)) / (1.0 + (w / wm) ** 2)
        upper = par if family == "uniform" else np.inf
        val = integrate.quad(f, 0.0, upper, limit=400, epsabs=1e-13, epsrel=1e-11)[0]
        out.append(pi0 * (1.0 - val))
    return np.asarray(out)


def fit_default_model(family: str, pi, omega_m, bounds=(0.1, 20.0)):
    """The grid parameter minimising sum_m (Pi(omega_m) - Pi_def(omega_m))^2 (Fig. 9), and
    that sum."""
    from scipy import optimize
    pi = np.asarray(pi, np.float64)
    sse = lambda par: float(np.sum((pi - default_model_data(family, par, pi[0], omega_m)) ** 2))
    r = optimize.minimize_scalar(sse, bounds=bounds, method="bounded", options={"xatol": 1e-5})
    return float(r.x), float(r.fun)
