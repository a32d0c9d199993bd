"""Python binding of libasm, the MI355X blocked-modes sampler for the average spectrum
method (Ghanem & Koch, arXiv:1912.01379).

Argument marshalling only: every step of the computation runs in the HIP library behind
the C ABI of include/asm.h.  PyTorch provides device memory and the stream.  Importing
this module loads libasm.so and raises if it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasm.so")

ASM_OK, ASM_EINVAL, ASM_EDOMAIN, ASM_ESTATE, ASM_EUNBOUNDED, ASM_EHIP, ASM_ENOMEM = 0, -1, -2, -3, -4, -5, -6
ASM_FP64, ASM_FP32 = 0, 1
ASM_START_FLAT, ASM_START_NNLS, ASM_START_NNLS_NOISED = 0, 1, 2

EXPORTED = ["asm_plan_create", "asm_plan_run", "asm_plan_vjp", "asm_plan_vjp_noalloc", "asm_plan_group_means",
            "asm_plan_advance",
            "asm_plan_state",
            "asm_plan_factors", "asm_plan_whitened", "asm_plan_destroy", "asm_tn_draw",
            "asm_uniforms", "asm_hierarchy", "asm_last_error", "asm_version"]


class AsmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libasm error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_void_p),
                ("G", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("cov", ctypes.c_void_p),
                ("B", ctypes.c_int64), ("block_start", ctypes.c_void_p), ("k", ctypes.c_void_p),
                ("init", ctypes.c_void_p), ("levels", ctypes.c_int64), ("level_blocks", ctypes.c_void_p),
                ("prior_shape", ctypes.c_void_p), ("constraint_c", ctypes.c_void_p),
                ("constraint_value", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_int64), ("burnin", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("refresh_every", ctypes.c_int32), ("want_vjp", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("lanes_per_chain", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("start", ctypes.c_int32), ("roles", ctypes.c_int32),
                ("chains_per_workgroup", ctypes.c_int32), ("u_rows", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("setup_ms", ctypes.c_double), ("sample_ms", ctypes.c_double),
                ("finalize_ms", ctypes.c_double), ("mode_moves", ctypes.c_double),
                ("data_moves", ctypes.c_double), ("chi2_drift_max", ctypes.c_double),
                ("clamped", ctypes.c_int64), ("frozen", ctypes.c_int64),
                ("lanes_per_chain", ctypes.c_int32), ("chains_per_block", ctypes.c_int32),
                ("sampler_ms", ctypes.c_double), ("sampler_launches", ctypes.c_int64),
                ("sampler_sweeps", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("roles", ctypes.c_int64), ("rejected", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1912_01379_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.asm_last_error.restype = ctypes.c_char_p
    L.asm_version.restype = ctypes.c_int
    L.asm_plan_create.argtypes = [ctypes.POINTER(_Problem), i64, ctypes.POINTER(_Options), vp,
                                  ctypes.POINTER(vp)]
    L.asm_plan_run.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Stats)]
    L.asm_plan_vjp.argtypes = [vp, vp, vp, vp]
    L.asm_plan_vjp_noalloc.argtypes = [vp, vp, vp, vp]
    L.asm_plan_group_means.argtypes = [vp, vp, vp, vp]
    L.asm_plan_advance.argtypes = [vp, i64]
    L.asm_plan_state.argtypes = [vp, i64, vp, vp, vp]
    L.asm_plan_factors.argtypes = [vp, i64, i64, ctypes.POINTER(i32), vp, vp, vp]
    L.asm_plan_whitened.argtypes = [vp, i64, vp, vp]
    L.asm_plan_destroy.argtypes = [vp]
    L.asm_tn_draw.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, vp]
    L.asm_uniforms.argtypes = [ctypes.c_uint64, i64, i64, i64, i64, i64, i64, vp, vp]
    L.asm_hierarchy.argtypes = [i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp]
    for name in EXPORTED:
        if name not in ("asm_last_error", "asm_version"):
            getattr(L, name).restype = ctypes.c_int
    return L


_lib = _load()


def lib():
    return _lib


def _check(rc: int):
    if rc != ASM_OK:
        raise AsmError(rc, _lib.asm_last_error().decode())


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev(x, device) -> Optional[torch.Tensor]:
    if x is None:
        return None
    t = torch.as_tensor(np.asarray(x) if not torch.is_tensor(x) else x, dtype=torch.float64)
    return t.to(device).contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


@dataclass
class RunResult:
    mean: torch.Tensor
    stderr: torch.Tensor
    post_sd: torch.Tensor
    stats: dict

    def split(self, sizes: Sequence[int]):
        return (torch.split(self.mean, list(sizes)), torch.split(self.stderr, list(sizes)),
                torch.split(self.post_sd, list(sizes)))


class Plan:
    """A set of continuation problems with their chains, living on one GPU.

    problems: sequence of objects with K (M x N), G (M), sigma (M) or cov (M x M),
    block_start (B+1) or levels (a list of such partitions: a hierarchy, see hierarchy()),
    optional k (B, over the blocks of all levels), init (N), prior_shape (N gamma-prior
    shapes) and constraint_c / constraint_value (a linear constraint c . A = F); numpy arrays
    or tensors.
    """

    def __init__(self, problems, chains=256, burnin=100, sweeps=1000, seed=1234, precision="fp32",
                 refresh_every=64, want_vjp=False, groups=32, lanes_per_chain=0, use_graph=False,
                 start="flat", roles=0, chains_per_workgroup=0, u_rows="auto", device="cuda:0"):
        self.device = torch.device(device)
        if isinstance(precision, str):
            precision = ASM_FP32 if precision.lower() == "fp32" else ASM_FP64
        self._keep = []
        probs = (_Problem * len(problems))()
        self.M, self.N = [], []
        for i, p in enumerate(problems):
            K = _dev(p.K, self.device)
            G = _dev(p.G, self.device)
            sig = _dev(getattr(p, "sigma", None), self.device)
            cov = _dev(getattr(p, "cov", None), self.device)
            if cov is not None:
                sig = None
            init = _dev(getattr(p, "init", None), self.device)
            shape = _dev(getattr(p, "prior_shape", None), self.device)
            cvec = _dev(getattr(p, "constraint_c", None), self.device)
            lv = getattr(p, "levels", None)
            parts = [np.asarray(x, dtype=np.int64) for x in lv] if lv is not None else \
                [np.asarray(p.block_start, dtype=np.int64)]
            bs = np.ascontiguousarray(np.concatenate(parts))
            lb = np.ascontiguousarray([len(x) - 1 for x in parts], dtype=np.int64)
            kk = getattr(p, "k", None)
            kk = None if kk is None else np.ascontiguousarray(np.asarray(kk, dtype=np.int32))
            self._keep += [K, G, sig, cov, init, shape, cvec, bs, lb, kk]
            M, N = int(K.shape[0]), int(K.shape[1])
            self.M.append(M)
            self.N.append(N)
            probs[i] = _Problem(M=M, N=N, K=_ptr(K), G=_ptr(G), sigma=_ptr(sig), cov=_ptr(cov),
                                B=int(lb.sum()), block_start=bs.ctypes.data,
                                k=None if kk is None else kk.ctypes.data, init=_ptr(init),
                                levels=len(parts), level_blocks=lb.ctypes.data if len(parts) > 1 else None,
                                prior_shape=_ptr(shape), constraint_c=_ptr(cvec),
                                constraint_value=float(getattr(p, "constraint_value", 0.0) or 0.0))
        self.options = _Options(chains=int(chains), burnin=int(burnin), sweeps=int(sweeps),
                                seed=int(seed) & 0xFFFFFFFFFFFFFFFF, precision=int(precision),
                                refresh_every=int(refresh_every), want_vjp=int(bool(want_vjp)),
                                groups=int(groups), lanes_per_chain=int(lanes_per_chain),
                                use_graph=int(bool(use_graph)),
                                start={"nnls": ASM_START_NNLS, "nnls_noised": ASM_START_NNLS_NOISED}.get(
                                    start, ASM_START_FLAT),
                                roles=int(roles), chains_per_workgroup=int(chains_per_workgroup),
                                u_rows={"auto": 0, "global": 1}[u_rows])
        self.chains = int(chains)
        self.handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_create(probs, len(problems), ctypes.byref(self.options),
                                        _stream(self.device), ctypes.byref(self.handle)))
        self.last = None

    def close(self):
        if self.handle:
            _lib.asm_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self) -> RunResult:
        tot = sum(self.N)
        mean = torch.empty(tot, dtype=torch.float64, device=self.device)
        se = torch.empty_like(mean)
        sd = torch.empty_like(mean)
        st = Stats()
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_run(self.handle, mean.data_ptr(), se.data_ptr(), sd.data_ptr(),
                                     ctypes.byref(st)))
        self.last = RunResult(mean, se, sd, st.as_dict())
        return self.last

    def vjp(self, v, stderr: bool = False):
        """J^T v of the last run (float64, sum M); with stderr=True also its standard error over
        the chain groups."""
        v = _dev(v, self.device)
        out = torch.empty(sum(self.M), dtype=torch.float64, device=self.device)
        se = torch.empty_like(out) if stderr else None
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_vjp(self.handle, v.data_ptr(), out.data_ptr(), _ptr(se)))
        return (out, se) if stderr else out

    def vjp_noalloc(self, v, out, se=None):
        """J^T v of the last run into the caller's float64 device tensors out (and se, its
        standard error, if given), without any device allocation (asm_plan_vjp_noalloc); the
        work is enqueued on the plan's stream and not waited for."""
        for t in (v, out) + (() if se is None else (se,)):
            if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_contiguous() and t.is_cuda):
                raise TypeError("v, out and se must be contiguous float64 tensors on the plan's device")
        if v.numel() != sum(self.N) or out.numel() != sum(self.M) or (se is not None and se.numel() != out.numel()):
            raise ValueError("v has sum N entries, out and se sum M")
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_vjp_noalloc(self.handle, v.data_ptr(), out.data_ptr(), _ptr(se)))
        return out

    def group_means(self) -> torch.Tensor:
        """The last run's average of each chain group: (groups, sum N)."""
        tot = sum(self.N)
        m = torch.empty(tot, dtype=torch.float64, device=self.device)
        se = torch.empty_like(m)
        g = torch.empty((self.options.groups or 32, tot), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_group_means(self.handle, m.data_ptr(), se.data_ptr(), g.data_ptr()))
        return g

    def advance(self, sweeps: int):
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_advance(self.handle, int(sweeps)))

    def state(self, problem: int = 0):
        M, N, C = self.M[problem], self.N[problem], self.chains
        A = torch.empty((C, N), dtype=torch.float64, device=self.device)
        r = torch.empty((C, M), dtype=torch.float64, device=self.device)
        chi2 = torch.empty(C, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_state(self.handle, problem, A.data_ptr(), r.data_ptr(),
                                       chi2.data_ptr()))
        return A, r, chi2

    def factors(self, problem: int, block: int, nb: int):
        M = self.M[problem]
        kb = ctypes.c_int32()
        V = torch.empty((nb, nb), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_factors(self.handle, problem, block, ctypes.byref(kb), None, None,
                                         V.data_ptr()))
        k = kb.value
        d = torch.empty(max(k, 1), dtype=torch.float64, device=self.device)
        U = torch.empty((M, max(k, 1)), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_factors(self.handle, problem, block, ctypes.byref(kb),
                                         d.data_ptr(), U.data_ptr(), None))
        return k, d[:k], U[:, :k], V

    def whitened(self, problem: int = 0):
        M, N = self.M[problem], self.N[problem]
        Kt = torch.empty((M, N), dtype=torch.float64, device=self.device)
        gt = torch.empty(M, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(_lib.asm_plan_whitened(self.handle, problem, Kt.data_ptr(), gt.data_ptr()))
        return Kt, gt


def hierarchy(N: int, max_block: int = 0) -> list:
    """The library's hierarchy of partitions (Fig. 2) for N grid points: a list of block
    offset arrays, top level (one block) first, single points last (asm_hierarchy)."""
    nl, ns = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.asm_hierarchy(int(N), int(max_block), ctypes.byref(nl), ctypes.byref(ns), None, None))
    lb = np.zeros(max(64, nl.value), np.int64)
    st = np.zeros(ns.value, np.int64)
    _check(_lib.asm_hierarchy(int(N), int(max_block), ctypes.byref(nl), ctypes.byref(ns),
                              lb.ctypes.data, st.ctypes.data))
    out, at = [], 0
    for b in lb[:nl.value]:
        out.append(st[at:at + int(b) + 1].copy())
        at += int(b) + 1
    return out


def tn_draw(c, d, lo, hi, u, precision="fp64", device="cuda:0"):
    """Device truncated-normal draws (test entry point of the move primitive)."""
    dev = torch.device(device)
    ts = [_dev(x, dev) for x in (c, d, lo, hi, u)]
    out = torch.empty_like(ts[0])
    prec = ASM_FP64 if precision == "fp64" else ASM_FP32
    with torch.cuda.device(dev):
        _check(_lib.asm_tn_draw(*[t.data_ptr() for t in ts], out.data_ptr(), out.numel(), prec,
                                _stream(dev)))
    return out


def uniforms(seed, problem, chain, sweep0, nsweeps, nblocks, nmodes, device="cuda:0"):
    dev = torch.device(device)
    out = torch.empty((nsweeps, nblocks, nmodes), dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        _check(_lib.asm_uniforms(int(seed) & 0xFFFFFFFFFFFFFFFF, problem, chain, sweep0, nsweeps,
                                 nblocks, nmodes, out.data_ptr(), _stream(dev)))
    return out


class AverageSpectrum(torch.autograd.Function):
    """(<A>, its standard error) as functions of the data G, with a backward pass through the
    on-device covariance estimator (asm_plan_vjp).

    forward(G, plan_factory) builds a plan with plan_factory(G) (it must pass want_vjp=True),
    runs it, and returns the average spectrum and its error bars (the error bars carry no
    gradient).  backward(grad_mean, grad_stderr) returns J^T grad_mean and releases the plan.
    """

    @staticmethod
    def forward(ctx, G, plan_factory):
        plan = plan_factory(G.detach())
        res = plan.run()
        ctx.plan = plan
        ctx.mark_non_differentiable(res.stderr)
        return res.mean.clone(), res.stderr.clone()

    @staticmethod
    def backward(ctx, grad_mean, grad_stderr):
        plan = ctx.plan
        g = plan.vjp(grad_mean.detach().to(torch.float64).contiguous())
        plan.close()
        ctx.plan = None
        return g, None
