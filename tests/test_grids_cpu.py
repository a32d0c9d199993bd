"""Host code of the package: the grid families of Sec. V.B and the default-model fit of
Sec. VI (Fig. 9), against closed forms, quadrature and the values the paper reads off Fig. 9."""
import math

import numpy as np
from scipy import integrate

import workloads


# --------------------------------------------------------------------------------------
# grids of Sec. V.B and the default-model fit of Sec. VI (Fig. 9): host code of the package
# --------------------------------------------------------------------------------------

def test_grid_families_integrate_and_default_models_have_closed_forms():
    """Riemann sums on each family integrate a smooth function; the Lorentzian and uniform
    default models have closed forms omega_m / (gamma + omega_m) and
    (omega_m / omega_c) atan(omega_c / omega_m) for the integral."""
    from paper_1912_01379_amd import grids
    f = lambda x: np.exp(-x) * (1.0 + np.sin(x))
    exact = integrate.quad(f, 0, np.inf)[0]
    for fam, par in (("gaussian", 3.0), ("exponential", 1.5), ("lorentzian", 1.0)):
        x, w = grids.grid(fam, par, 4000)
        assert abs(np.sum(w * f(x)) - exact) < 2e-3 * exact, fam
    x, w = grids.grid("uniform", 30.0, 4000)
    assert abs(np.sum(w * f(x)) - exact) < 1e-3 * exact
    wm = np.array([0.0, 0.4, 1.3, 7.0])
    for g in (0.7, 2.5):
        ref = np.r_[1.0, 1.0 - wm[1:] / (g + wm[1:])]
        assert np.allclose(grids.default_model_data("lorentzian", g, 1.0, wm), ref, rtol=1e-9)
    c = 3.7
    ref = np.r_[1.0, 1.0 - wm[1:] / c * np.arctan(c / wm[1:])]
    assert np.allclose(grids.default_model_data("uniform", c, 1.0, wm), ref, rtol=1e-9)


def test_default_model_fit_reproduces_fig9():
    """Fig. 9 on the paper's own test case (model 2): the best Gaussian width is 2.4 and the
    best uniform cutoff 3.7, as the paper reads them off; the Lorentzian of width 2.5 fits far
    worse than the best Gaussian."""
    import json, os
    from paper_1912_01379_amd import grids
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fig9_default_model.json")))
    p = workloads.optical_conductivity(40, 1, model=2)
    wm = 2.0 * np.pi * np.arange(len(p.G)) / 15.0
    a, sse_g = grids.fit_default_model("gaussian", p.G, wm, (0.5, 10.0))
    c, sse_u = grids.fit_default_model("uniform", p.G, wm, (1.0, 20.0))
    assert abs(a - gold["gaussian_alpha"]) < 0.1, a
    assert abs(c - gold["uniform_cutoff"]) < 0.15, c
    sse_l = float(np.sum((p.G - grids.default_model_data("lorentzian", gold["lorentzian_gamma_off"], p.G[0], wm)) ** 2))
    assert sse_l > 100 * sse_g, (sse_l, sse_g)
