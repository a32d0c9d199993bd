"""Plain FP64 CPU oracle of blocked modes sampling (Ghanem & Koch, arXiv:1912.01379).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark are the only users.  The product (the GPU library and its binding) never
imports this package, and this package never imports the product.

Steps, in the paper's order:
  1. whitening, Sec. IV after Eq. (chi2): C^-1 = T^T T, g~ = T g, K~ = T K;
  2. per-block SVD K~_b = U_b D_b V_b^T, Sec. IV.B/IV.C, with d := 0 beyond the
     numerical rank (the paper's zero modes);
  3. the random walk over blocked modes (C core, `core.c`), optionally with the gamma-prior
     weights prod_n A_n^(w_n - 1) of Sec. V.C (Eq. (compat)) through an acceptance test per move;
  4. averages of Eq. (MCint), their error bars, and the sensitivity of the average to
     the data, d<f>/dg = -Cov(f, r~) T, which follows from differentiating the
     posterior of Eq. (PI) (the normaliser depends on g).

Readings where the paper leaves a choice open (shared by the GPU library by definition,
not by code):
  * numerical rank: d_i > max(M, N_b) * eps * d_1; the number of data modes of a block is
    min(requested, rank);
  * sign of a data mode: sum_n (n+1) V_ni > 0;
  * zero-mode basis: the last N_b - k columns of the Householder product that
    triangularises the data-mode columns (reflector x -> beta e_1, beta = -sign(x_1)|x|,
    sign(0) = +1);
  * start vector: the best constant fit c* = (K~ 1).g~ / |K~ 1|^2 (1 if c* <= 0);
  * error bars: standard error of the mean over G independent chain groups (or G batches
    of sweeps when there are fewer chains than groups).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_SRC = os.path.join(_HERE, "core.c")
_lock = threading.Lock()
_lib = None

EPS = np.finfo(np.float64).eps
GL_NODES = 20
_gl_keep = []


def build(force: bool = False) -> str:
    """Compile the C core with gcc (plain -O2, IEEE arithmetic, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("B", ctypes.c_int64),
                ("Kt", ctypes.c_void_p), ("gt", ctypes.c_void_p), ("bn0", ctypes.c_void_p),
                ("bnb", ctypes.c_void_p), ("L", ctypes.c_int64), ("lfirst", ctypes.c_void_p),
                ("lcount", ctypes.c_void_p), ("kb", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("U", ctypes.c_void_p), ("V", ctypes.c_void_p), ("shape_m1", ctypes.c_void_p),
                ("bnm", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_int64), ("burnin", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("problem_index", ctypes.c_int64),
                ("refresh_every", ctypes.c_int64), ("groups", ctypes.c_int64),
                ("want_cross", ctypes.c_int64), ("threads", ctypes.c_int64),
                ("traj_chain", ctypes.c_int64), ("init", ctypes.c_void_p), ("vjp_v", ctypes.c_void_p)]


class _Out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("sumA", "sumA2", "count", "sumR", "sumRA", "final_A", "final_r", "final_chi2",
                 "traj_A", "traj_chi2", "drift_max", "n_frozen", "n_clamped", "status",
                 "n_rejected", "gRv", "gR", "gAv")]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            L.orc_mass.restype = ctypes.c_double
            L.orc_mass.argtypes = [ctypes.c_double] * 3
            L.orc_set_quadrature.restype = None
            L.orc_set_quadrature.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
            L.orc_tn_draw.restype = ctypes.c_double
            L.orc_tn_draw.argtypes = [ctypes.c_double] * 5
            L.orc_mills.restype = ctypes.c_double
            L.orc_mills.argtypes = [ctypes.c_double]
            L.orc_move_uniform.restype = ctypes.c_double
            L.orc_move_uniform.argtypes = [ctypes.c_uint64] + [ctypes.c_int64] * 5
            L.orc_sweep_level.restype = ctypes.c_int64
            L.orc_sweep_level.argtypes = [ctypes.c_uint64] + [ctypes.c_int64] * 3
            L.orc_philox.restype = None
            L.orc_philox.argtypes = [ctypes.c_void_p] * 3
            L.orc_run.restype = ctypes.c_int
            L.orc_run.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Options),
                                  ctypes.POINTER(_Out)]
            # the truncated-normal masses over short stretches: 20-point Gauss-Legendre
            x, w = np.polynomial.legendre.leggauss(GL_NODES)
            _gl_keep[:] = [np.ascontiguousarray(x), np.ascontiguousarray(w)]
            L.orc_set_quadrature(GL_NODES, _gl_keep[0].ctypes.data, _gl_keep[1].ctypes.data)
            _lib = L
    return _lib


# --------------------------------------------------------------------------------------
# scalar helpers exposed for the pins
# --------------------------------------------------------------------------------------

def mass(r0: float, t1: float, t2: float) -> float:
    """int_{t1}^{t2} exp(-tau (2 r0 + tau) / 2) dtau: the normal mass of [r0 + t1, r0 + t2]
    divided by the density at r0 (the truncated normal's distribution function is a ratio
    of two of these)."""
    return lib().orc_mass(float(r0), float(t1), float(t2))


def tn_draw(c: float, d: float, lo: float, hi: float, u: float) -> float:
    """The u-quantile of N(c/d, 1/d^2) restricted to [lo, hi] (Sec. IV.B), by bisection."""
    return lib().orc_tn_draw(float(c), float(d), float(lo), float(hi), float(u))


def mills(x: float) -> float:
    return lib().orc_mills(float(x))


def move_uniform(seed, problem, chain, sweep, block, mode) -> float:
    return lib().orc_move_uniform(int(seed) & 0xFFFFFFFFFFFFFFFF, problem, chain, sweep, block, mode)


def sweep_level(seed, problem, sweep, levels) -> int:
    """The hierarchy level sampled in a sweep (shared by all chains of the problem)."""
    return int(lib().orc_sweep_level(int(seed) & 0xFFFFFFFFFFFFFFFF, problem, sweep, levels))


def philox(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


# --------------------------------------------------------------------------------------
# setup: whitening and block factors
# --------------------------------------------------------------------------------------

@dataclass
class Prepared:
    Kt: np.ndarray            # M x N
    gt: np.ndarray            # M
    levels: list              # partitions of the hierarchy, each B_l+1 offsets
    kb: np.ndarray            # B (int32), blocks of all levels in order
    d: list                   # per block: singular values of the data modes
    U: list                   # per block: M x kb
    V: list                   # per block: Nb x Nb (columns = modes, data first)
    dall: list                # per block: all singular values (min(M, Nb))
    Tt: object                # callable y -> T^T y
    init: np.ndarray          # N
    shape: Optional[np.ndarray] = None   # N gamma-prior shapes w_n (Eq. (compat)), or flat
    cvec: Optional[np.ndarray] = None    # N: linear constraint c . A = cval (Sec. IV.E), or None
    cval: float = 0.0
    nm: Optional[np.ndarray] = None      # B: modes per block (N_b, or N_b - 1 under the constraint)

    @property
    def M(self):
        return int(self.Kt.shape[0])

    @property
    def N(self):
        return int(self.Kt.shape[1])

    @property
    def B(self):
        return int(sum(len(ls) - 1 for ls in self.levels))

    @property
    def bstart(self):
        """The offsets of a single partition."""
        if len(self.levels) != 1:
            raise ValueError("a hierarchy has one partition per level")
        return self.levels[0]

    @property
    def blocks(self):
        """(first grid point, size) of every block, level after level."""
        return [(int(ls[b]), int(ls[b + 1] - ls[b])) for ls in self.levels for b in range(len(ls) - 1)]


def whiten(K, G, sigma=None, cov=None):
    """C^-1 = T^T T; returns K~ = T K, g~ = T g and y -> T^T y."""
    if cov is None:
        s = np.asarray(sigma, dtype=np.float64)
        Kt = K / s[:, None]
        gt = G / s
        return Kt, gt, (lambda y: np.asarray(y) / s)
    L = np.linalg.cholesky(np.asarray(cov, dtype=np.float64))   # C = L L^T, T = L^-1
    Kt = np.linalg.solve(L, K)
    gt = np.linalg.solve(L, G)
    return Kt, gt, (lambda y: np.linalg.solve(L.T, np.asarray(y)))


def householder_complete(Vd: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the complement of the (orthonormal) columns of Vd.

    Householder reflections H_0..H_{k-1} triangularise Vd; the completion is
    Q e_j, j = k..nb-1, with Q = H_0 H_1 ... H_{k-1}.
    """
    nb, k = Vd.shape
    X = np.array(Vd, dtype=np.float64, copy=True)
    refl = []
    for j in range(k):
        x = X[j:, j]
        alpha = x[0]
        norm = np.sqrt(np.dot(x, x))
        beta = -norm if alpha >= 0.0 else norm
        v = x.copy()
        v[0] = alpha - beta
        vv = np.dot(v, v)
        if vv > 0.0:
            X[j:, j:] -= np.outer(v, (2.0 / vv) * (v @ X[j:, j:]))
        refl.append((v, vv))
    Z = np.zeros((nb, nb - k))
    for col in range(k, nb):
        e = np.zeros(nb)
        e[col] = 1.0
        for j in reversed(range(k)):
            v, vv = refl[j]
            if vv > 0.0:
                e[j:] -= v * (2.0 / vv * np.dot(v, e[j:]))
        Z[:, col - k] = e
    return Z


def block_factors(Kb: np.ndarray, k_req: Optional[int]):
    """SVD of one whitened block with the rank cut, sign rule and zero-mode completion."""
    M, nb = Kb.shape
    Uf, sv, Vt = np.linalg.svd(Kb, full_matrices=False)
    r = min(M, nb)
    sv = sv[:r]
    thr = max(M, nb) * EPS * (sv[0] if r > 0 else 0.0)
    rank = int(np.sum(sv > thr)) if r > 0 and sv[0] > 0 else 0
    k = rank if k_req is None else min(int(k_req), rank)
    Vd = Vt[:k, :].T.copy()
    Ud = Uf[:, :k].copy()
    w = np.arange(1, nb + 1, dtype=np.float64)
    for i in range(k):
        if np.dot(w, Vd[:, i]) < 0.0:
            Vd[:, i] = -Vd[:, i]
            Ud[:, i] = -Ud[:, i]
    Z = householder_complete(Vd)
    V = np.concatenate([Vd, Z], axis=1)
    return sv[:k].copy(), Ud, V, sv.copy()


def data_noise(seed: int, problem: int, M: int) -> np.ndarray:
    """Standard normal noise for the whitened data (Sec. IV.D suggests the NNLS fit of noised
    data as the start): Box-Muller, xi_m = sqrt(-2 ln u1) cos(2 pi u2), with u1 and u2 the
    uniforms of words (w0, w1) and (w2, w3) of Philox on counter (2^32 - 2, m, 0, 5)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = [seed & 0xFFFFFFFF, ((seed >> 32) ^ int(problem)) & 0xFFFFFFFF]

    def u01(a, b):
        return ((int(a) >> 6) * 2 ** 26 + (int(b) >> 6) + 0.5) * 2.0 ** -52

    out = np.empty(M)
    for m in range(M):
        w = philox([0xFFFFFFFE, m, 0, 5], key)
        out[m] = np.sqrt(-2.0 * np.log(u01(w[0], w[1]))) * np.cos(2.0 * np.pi * u01(w[2], w[3]))
    return out


def nnls_start(prep: Prepared, blend: float = 0.01, noise_seed=None, problem: int = 0) -> np.ndarray:
    """Start model from the non-negative least-squares fit, Sec. IV.D (start from NNLS).

    The NNLS solution of K~ f = g~ (Lawson-Hanson, scipy) has exact zeros, which would
    leave most zero modes with an empty interval; it is therefore blended with the best
    constant fit: f0 = (1 - blend) f_NNLS + blend c*.  With noise_seed, both are taken of the
    noised data g~ + xi (data_noise).
    """
    from scipy.optimize import nnls
    g = prep.gt if noise_seed is None else prep.gt + data_noise(noise_seed, problem, prep.M)
    x, _ = nnls(prep.Kt, g, maxiter=50 * prep.N)
    one = prep.Kt @ np.ones(prep.N)
    cstar = float(np.dot(one, g) / np.dot(one, one))
    if not (cstar > 0.0 and np.isfinite(cstar)):
        cstar = 1.0
    return (1.0 - blend) * x + blend * cstar


def hierarchy(N: int, max_block: int = 0) -> list:
    """The hierarchy of partitions of Fig. 2 (Sec. IV.C), top level first.

    Level l splits the grid into intervals of width w = N / 2^l (one block at l = 0, two
    halves at l = 1); on the even levels l >= 2 the intervals are shifted by w / 2, so that
    the end blocks have half the width and the centre of the grid is not a boundary.  The
    boundaries are floor(N (2j + s) / 2^(l+1)), s = 1 on shifted levels.  The blocked
    levels run while w >= 2; the last level is the single grid points (components).
    Levels with a block longer than max_block (> 0) are left out.
    """
    N = int(N)
    out = []
    lvl = 0
    while N >= 2 ** (lvl + 1):           # w = N / 2^l >= 2
        shift = 1 if lvl >= 2 and lvl % 2 == 0 else 0
        inner = [N * (2 * j + shift) // 2 ** (lvl + 1) for j in range(2 ** lvl + 1)]
        out.append(np.asarray([0] + [c for c in inner if 0 < c < N] + [N], np.int64))
        lvl += 1
    out.append(np.arange(N + 1, dtype=np.int64))
    if max_block > 0:
        out = [ls for ls in out if int(np.max(np.diff(ls))) <= max_block]
    return out


def constraint_basis(cb: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the part of a block orthogonal to its share c_b of a linear
    constraint (Sec. IV.E): the Householder reflector H = I - 2 v v^T / v.v with H c_b =
    beta e_1 (beta = -sign(c_b[0]) |c_b|, sign(0) = +1) has H e_1 parallel to c_b, so its other
    columns span the complement.  A block where c_b = 0 keeps the identity."""
    nb = len(cb)
    if not np.any(cb != 0.0):
        return np.eye(nb)
    x = np.asarray(cb, np.float64)
    alpha = x[0]
    norm = np.sqrt(np.dot(x, x))
    beta = -norm if alpha >= 0.0 else norm
    v = x.copy()
    v[0] = alpha - beta
    H = np.eye(nb) - np.outer(v, v) * (2.0 / np.dot(v, v))
    return H[:, 1:]


def prepare(problem, k=None) -> Prepared:
    """Whitening + block factors + start vector for one workloads.Problem."""
    Kt, gt, Tt = whiten(problem.K, problem.G, problem.sigma, problem.cov)
    levels = problem.partitions()
    spans = [(int(ls[b]), int(ls[b + 1])) for ls in levels for b in range(len(ls) - 1)]
    kreq = k if k is not None else problem.k
    cvec = getattr(problem, "constraint_c", None)
    cvec = None if cvec is None else np.asarray(cvec, np.float64)
    ds, Us, Vs, dall = [], [], [], []
    kb, nm = [], []
    for b, (s0, s1) in enumerate(spans):
        Kb = Kt[:, s0:s1]
        kr = None if kreq is None else int(np.asarray(kreq)[b])
        if cvec is None:
            d, U, V, sv = block_factors(Kb, kr)
        else:
            # modes of the block restricted to the complement of its constraint share: the
            # factors of K~_b Q_b, mapped back, V = Q_b V'
            Q = constraint_basis(cvec[s0:s1])
            if Q.shape[1] == 0:
                d, U, V, sv = np.zeros(0), np.zeros((Kt.shape[0], 0)), np.zeros((s1 - s0, 0)), np.zeros(0)
            else:
                d, U, Vr, sv = block_factors(Kb @ Q, kr)
                V = Q @ Vr
        ds.append(d); Us.append(U); Vs.append(V); dall.append(sv)
        kb.append(len(d))
        nm.append(V.shape[1])
    one = Kt @ np.ones(Kt.shape[1])
    cstar = float(np.dot(one, gt) / np.dot(one, one))
    if not (cstar > 0.0 and np.isfinite(cstar)):
        cstar = 1.0
    init = np.full(Kt.shape[1], cstar)
    return Prepared(Kt=np.ascontiguousarray(Kt), gt=np.ascontiguousarray(gt), levels=levels,
                    kb=np.asarray(kb, dtype=np.int32), d=ds, U=Us, V=Vs, dall=dall, Tt=Tt,
                    init=init, shape=None if getattr(problem, "prior_shape", None) is None
                    else np.asarray(problem.prior_shape, np.float64),
                    cvec=cvec, cval=float(getattr(problem, "constraint_value", 0.0)),
                    nm=np.asarray(nm, np.int64))


# --------------------------------------------------------------------------------------
# running the chains
# --------------------------------------------------------------------------------------

@dataclass
class Result:
    mean: np.ndarray
    stderr: np.ndarray
    post_sd: np.ndarray
    ess: np.ndarray
    group_means: np.ndarray
    final_A: np.ndarray
    final_r: np.ndarray
    final_chi2: np.ndarray
    traj_A: Optional[np.ndarray]
    traj_chi2: Optional[np.ndarray]
    drift_max: float
    n_frozen: int
    n_clamped: int
    status: int
    n_rejected: int
    cov_rA: Optional[np.ndarray]   # M x N sample Cov(r~, A)
    mean_r: Optional[np.ndarray]
    prep: Prepared
    vjp: Optional[np.ndarray] = None       # M: J^T v for the run's vjp_v (pooled covariance)
    vjp_se: Optional[np.ndarray] = None    # M: its standard error over the chain groups
    vjp_groups: Optional[np.ndarray] = None   # G x M: J^T v of each group's own covariance


def run(prep: Prepared, chains=1, burnin=0, sweeps=100, seed=1234, problem_index=0,
        refresh_every=64, groups=32, want_cross=False, threads=None, traj_chain=-1,
        init=None, vjp_v=None) -> Result:
    L = lib()
    M, N, B = prep.M, prep.N, prep.B
    if threads is None:
        threads = os.cpu_count() or 1
    d_all = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64) for x in prep.d]) if sum(prep.kb) else np.zeros(1))
    U_all = np.ascontiguousarray(np.concatenate([np.asarray(u, np.float64).ravel() for u in prep.U]) if sum(prep.kb) else np.zeros(1))
    V_all = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64).ravel() for v in prep.V]))
    bn0 = np.ascontiguousarray([b[0] for b in prep.blocks], dtype=np.int64)
    bnb = np.ascontiguousarray([b[1] for b in prep.blocks], dtype=np.int64)
    lcount = np.ascontiguousarray([len(ls) - 1 for ls in prep.levels], dtype=np.int64)
    lfirst = np.ascontiguousarray(np.concatenate([[0], np.cumsum(lcount)[:-1]]), dtype=np.int64)
    kb = np.ascontiguousarray(prep.kb, dtype=np.int32)
    start = np.asarray(prep.init if init is None else np.asarray(init, np.float64), np.float64)
    if prep.cvec is not None:
        # the start moved onto c . A = F: scaled by F / (c . A) when that is positive (which
        # keeps it non-negative), else projected along c; it must stay non-negative
        c = prep.cvec
        cs = float(np.dot(c, start))
        if cs != 0.0 and prep.cval / cs > 0.0:
            start = start * (prep.cval / cs)
        else:
            start = start + c * ((prep.cval - cs) / np.dot(c, c))
        if np.min(start) < 0.0:
            raise ValueError("the start moved onto the constraint has a negative component")
    start = np.ascontiguousarray(start)
    bnm = np.ascontiguousarray(prep.nm if prep.nm is not None else [b[1] for b in prep.blocks], dtype=np.int64)
    G = int(groups)
    total = burnin + sweeps
    bufs = dict(
        sumA=np.zeros(G * N), sumA2=np.zeros(G * N), count=np.zeros(G, np.int64),
        sumR=np.zeros(M) if want_cross else None, sumRA=np.zeros(M * N) if want_cross else None,
        final_A=np.zeros(chains * N), final_r=np.zeros(chains * M), final_chi2=np.zeros(chains),
        traj_A=np.zeros(total * N) if traj_chain >= 0 else None,
        traj_chi2=np.zeros(total) if traj_chain >= 0 else None,
        drift_max=np.zeros(1), n_frozen=np.zeros(1, np.int64), n_clamped=np.zeros(1, np.int64),
        status=np.zeros(1, np.int32), n_rejected=np.zeros(1, np.int64),
        gRv=np.zeros(G * M) if vjp_v is not None else None,
        gR=np.zeros(G * M) if vjp_v is not None else None,
        gAv=np.zeros(G) if vjp_v is not None else None)
    vv = None if vjp_v is None else np.ascontiguousarray(np.asarray(vjp_v, np.float64))
    shape_m1 = None if prep.shape is None else np.ascontiguousarray(np.asarray(prep.shape, np.float64) - 1.0)
    p = _Problem(M=M, N=N, B=B, Kt=prep.Kt.ctypes.data, gt=prep.gt.ctypes.data,
                 bn0=bn0.ctypes.data, bnb=bnb.ctypes.data, L=len(prep.levels),
                 lfirst=lfirst.ctypes.data, lcount=lcount.ctypes.data, kb=kb.ctypes.data, d=d_all.ctypes.data,
                 U=U_all.ctypes.data, V=V_all.ctypes.data,
                 shape_m1=None if shape_m1 is None else shape_m1.ctypes.data, bnm=bnm.ctypes.data)
    o = _Options(chains=chains, burnin=burnin, sweeps=sweeps, seed=int(seed) & 0xFFFFFFFFFFFFFFFF,
                 problem_index=problem_index, refresh_every=refresh_every, groups=G,
                 want_cross=1 if want_cross else 0, threads=int(threads), traj_chain=traj_chain,
                 init=start.ctypes.data, vjp_v=None if vv is None else vv.ctypes.data)
    out = _Out(**{k: (v.ctypes.data if v is not None else None) for k, v in bufs.items()})
    L.orc_run(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out))
    sumA = bufs["sumA"].reshape(G, N)
    sumA2 = bufs["sumA2"].reshape(G, N)
    cnt = bufs["count"].astype(np.float64)
    tot = float(cnt.sum())
    mean = sumA.sum(0) / tot if tot > 0 else np.zeros(N)
    with np.errstate(invalid="ignore", divide="ignore"):
        gm = sumA / cnt[:, None]
    ok = cnt > 0
    if ok.sum() >= 2:
        se = np.std(gm[ok], axis=0, ddof=1) / np.sqrt(ok.sum())
    else:
        se = np.full(N, np.nan)
    var = np.maximum(sumA2.sum(0) / tot - mean * mean, 0.0) if tot > 0 else np.zeros(N)
    with np.errstate(invalid="ignore", divide="ignore"):
        ess = var / (se * se)
    cov_rA = mean_r = None
    if want_cross and tot > 0:
        mean_r = bufs["sumR"] / tot
        cov_rA = bufs["sumRA"].reshape(M, N) / tot - np.outer(mean_r, mean)
    vjp_p = vjp_g = vjp_se = None
    if vv is not None and tot > 0:
        # J^T v = -T^T Cov(r~, A) v (Sec. II, Eq. (PI) differentiated in the data): per group
        # from the group's own moments, pooled from all samples; the error bar is the
        # standard deviation of the group values over sqrt(G)
        gRv = bufs["gRv"].reshape(G, M)
        gR = bufs["gR"].reshape(G, M)
        gAv = bufs["gAv"]
        yp = gRv.sum(0) / tot - (gR.sum(0) / tot) * (gAv.sum() / tot)
        vjp_p = -np.asarray(prep.Tt(yp))
        rows = []
        for g in range(G):
            if cnt[g] > 0:
                yg = gRv[g] / cnt[g] - (gR[g] / cnt[g]) * (gAv[g] / cnt[g])
                rows.append(-np.asarray(prep.Tt(yg)))
        vjp_g = np.array(rows)
        vjp_se = np.std(vjp_g, axis=0, ddof=1) / np.sqrt(len(rows)) if len(rows) >= 2 else None
    return Result(mean=mean, stderr=se, post_sd=np.sqrt(var), ess=ess, group_means=gm,
                  vjp=vjp_p, vjp_se=vjp_se, vjp_groups=vjp_g,
                  final_A=bufs["final_A"].reshape(chains, N),
                  final_r=bufs["final_r"].reshape(chains, M), final_chi2=bufs["final_chi2"],
                  traj_A=None if bufs["traj_A"] is None else bufs["traj_A"].reshape(total, N),
                  traj_chi2=bufs["traj_chi2"], drift_max=float(bufs["drift_max"][0]),
                  n_frozen=int(bufs["n_frozen"][0]), n_clamped=int(bufs["n_clamped"][0]),
                  status=int(bufs["status"][0]), n_rejected=int(bufs["n_rejected"][0]),
                  cov_rA=cov_rA, mean_r=mean_r, prep=prep)


def vjp(res: Result, v: np.ndarray) -> np.ndarray:
    """J^T v with J = d<A>/dg = -Cov(A, r~) T, i.e. J^T v = -T^T (Cov(r~, A) v)."""
    if res.cov_rA is None:
        raise ValueError("run(..., want_cross=True) is required for the VJP")
    return -res.prep.Tt(res.cov_rA @ np.asarray(v, dtype=np.float64))
