"""Python binding of librbffmm: plans, products, solves.

Torch provides device memory and the stream; every step of the computation runs in the
HIP library (include/rbf_fmm.h).  Nothing here computes a result.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_KERNELS = {"gaussian": L.RBF_GAUSSIAN, "multiquadric": L.RBF_MULTIQUADRIC,
            "inverse_multiquadric": L.RBF_INVERSE_MULTIQUADRIC, "wendland": L.RBF_WENDLAND,
            "thin_plate": L.RBF_THIN_PLATE, "r5": L.RBF_R5, "gaussian_bandlimited": L.RBF_GAUSSIAN_BANDLIMITED}
_PCS = {"none": L.RBF_PC_NONE, "block_jacobi": L.RBF_PC_BLOCK_JACOBI, "learned": L.RBF_PC_LEARNED}


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return L.RBF_F32
    if t.dtype == torch.float64:
        return L.RBF_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensor must live on the HIP device")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _opts(n_max=0, max_level=0, min_level=0, coarse_level=-1, coarse_radius=-1, nodes=0, band=0.0,
          m2l_schedule=0, exact=0, band_transfer=0):
    return L.RbfOpts(n_max, max_level, min_level, coarse_level, coarse_radius, nodes, band, m2l_schedule,
                     1 if exact else 0, int(band_transfer))


def _opts_dict(o: "L.RbfOpts") -> dict:
    return {"n_max": o.n_max, "max_level": o.max_level, "min_level": o.min_level, "coarse_level": o.coarse_level,
            "coarse_radius": o.coarse_radius, "nodes": o.nodes, "band": o.band, "m2l_schedule": o.m2l_schedule,
            "exact": o.exact, "band_transfer": o.band_transfer}


def autotune(points: torch.Tensor, kernel: str = "gaussian", shape: float = 0.05, tol: float = 1e-6,
             reps: int = 3, stream: Optional[torch.cuda.Stream] = None, **base) -> tuple:
    """Measure candidate configurations (rbf_fmm_autotune); returns (opts dict, ms per product)."""
    lib = L.load()
    stream = stream if stream is not None else torch.cuda.current_stream(points.device)
    b = _opts(**base)
    best = L.RbfOpts()
    ms = ctypes.c_double()
    L.check(lib.rbf_fmm_autotune(_ptr(points), points.shape[0], points.shape[1], _dtype_code(points),
                                 _KERNELS[kernel], float(shape), float(tol), ctypes.byref(b), reps,
                                 ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best), ctypes.byref(ms)))
    return _opts_dict(best), ms.value


class BatchPlan:
    """Many independent problems (concatenated points, per-problem shapes) in one batched
    product per call (rbf_fmm_plan_batch / rbf_fmm_matvec_batch)."""

    def __init__(self, points: torch.Tensor, offsets, shapes, kernel: str = "gaussian", tol: float = 1e-4,
                 autotune: bool = False, stream: Optional[torch.cuda.Stream] = None, **opts):
        lib = L.load()
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.shapes = np.ascontiguousarray(shapes, dtype=np.float64)
        self.nprob = len(self.shapes)
        if self.offsets.shape != (self.nprob + 1,) or self.offsets[-1] != points.shape[0]:
            raise ValueError("offsets must have nprob + 1 entries ending at the number of points")
        self.n, self.d = points.shape
        self.dtype, self.device = points.dtype, points.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(points.device)
        o = _opts(**opts) if opts else None
        h = ctypes.c_void_p()
        L.check(lib.rbf_fmm_plan_batch(_ptr(points), self.offsets.ctypes.data, self.nprob, self.d,
                                       _dtype_code(points), _KERNELS[kernel], self.shapes.ctypes.data, float(tol),
                                       ctypes.byref(o) if o is not None else None, 1 if autotune else 0,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def matvec(self, lam: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if lam.shape != (self.n,) or lam.dtype != self.dtype:
            raise ValueError("lambda must be the concatenated vector of all problems")
        if out is None:
            out = torch.empty_like(lam)
        L.check(L.load().rbf_fmm_matvec_batch(self._h, _ptr(lam), _ptr(out)))
        return out

    def solve(self, f: torch.Tensor, lam: Optional[torch.Tensor] = None, rtol: float = 1e-8, restart: int = 50,
              max_iters: int = 1000, time_limit_s: float = 0.0, precond: str = "none"):
        """Restarted GMRES for every problem (rbf_interp_solve_batch), precond "none" or
        "block_jacobi"; returns (lambda, [info per problem])."""
        if f.shape != (self.n,) or f.dtype != self.dtype:
            raise ValueError("f must be the concatenated right-hand side of all problems")
        pk = {"none": L.RBF_PC_NONE, "block_jacobi": L.RBF_PC_BLOCK_JACOBI}[precond]
        zero = lam is None
        if lam is None:
            lam = torch.zeros_like(f)
        o = L.RbfSolveOpts(restart, max_iters, pk, 1 if zero else 0, 1, float(time_limit_s))
        infos = (L.RbfSolveInfo * self.nprob)()
        code = L.load().rbf_interp_solve_batch(self._h, _ptr(f), _ptr(lam), float(rtol), ctypes.byref(o), infos)
        L.check(code, allow=(L.RBF_OK, L.RBF_ENOCONV))
        out = [{"iters": i.iters, "restarts": i.restarts, "converged": bool(i.converged), "true_res": i.true_res,
                "seconds": i.seconds, "history": list(i.history[:i.nhistory]),
                "history_s": list(i.history_s[:i.nhistory])} for i in infos]
        return lam, out

    def set_graph(self, on: bool):
        L.check(L.load().rbf_fmm_batch_set_graph(self._h, 1 if on else 0))

    def info(self) -> dict:
        inf = L.RbfBatchInfo()
        nm = np.empty(self.nprob, np.int32)
        nd = np.empty(self.nprob, np.int32)
        L.check(L.load().rbf_fmm_batch_info(self._h, ctypes.byref(inf), nm.ctypes.data, nd.ctypes.data))
        out = {name: getattr(inf, name) for name, _ in L.RbfBatchInfo._fields_}
        out["n_max"], out["nodes"] = nm, nd
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.load().rbf_fmm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FmmPlan:
    """Plan for u = A lambda with A_ij = Phi(x_i - x_j) on a fixed point set."""

    def __init__(self, points: torch.Tensor, kernel: str = "gaussian", shape: float = 0.05,
                 tol: float = 1e-6, n_max: int = 0, max_level: int = 0, min_level: int = 0,
                 coarse_level: int = -1, coarse_radius: int = -1, nodes: int = 0, band: float = 0.0,
                 m2l_schedule: int = 0, exact: bool = False, band_transfer: int = 0,
                 stream: Optional[torch.cuda.Stream] = None):
        lib = L.load()
        if points.dim() != 2:
            raise ValueError("points must be (n, d)")
        self.n, self.d = points.shape
        self.dtype = points.dtype
        self.device = points.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(points.device)
        opts = _opts(n_max, max_level, min_level, coarse_level, coarse_radius, nodes, band, m2l_schedule, exact,
                     band_transfer)
        h = ctypes.c_void_p()
        L.check(lib.rbf_fmm_plan(_ptr(points), self.n, self.d, _dtype_code(points), _KERNELS[kernel],
                                 float(shape), float(tol), ctypes.byref(opts),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.kernel, self.shape, self.tol = kernel, shape, tol

    # -- products --------------------------------------------------------------------
    def _check_vec(self, v: torch.Tensor):
        if v.shape != (self.n,) or v.dtype != self.dtype or v.device != self.device:
            raise ValueError(f"expected a ({self.n},) {self.dtype} vector on {self.device}")

    def matvec(self, lam: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_vec(lam)
        if out is None:
            out = torch.empty_like(lam)
        self._check_vec(out)
        L.check(L.load().rbf_fmm_matvec(self._h, _ptr(lam), _ptr(out)))
        return out

    def direct(self, lam: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_vec(lam)
        if out is None:
            out = torch.empty_like(lam)
        self._check_vec(out)
        L.check(L.load().rbf_direct_matvec(self._h, _ptr(lam), _ptr(out)))
        return out

    def solve(self, f: torch.Tensor, lam: Optional[torch.Tensor] = None, rtol: float = 1e-8,
              restart: int = 50, max_iters: int = 1000, precond: str = "none", fallback: bool = True,
              time_limit_s: float = 0.0):
        self._check_vec(f)
        zero = lam is None
        if lam is None:
            lam = torch.zeros_like(f)
        self._check_vec(lam)
        o = L.RbfSolveOpts(restart, max_iters, _PCS[precond], 1 if zero else 0, 1 if fallback else 0,
                           float(time_limit_s))
        info = L.RbfSolveInfo()
        code = L.load().rbf_interp_solve(self._h, _ptr(f), _ptr(lam), float(rtol), ctypes.byref(o),
                                         ctypes.byref(info))
        L.check(code, allow=(L.RBF_OK, L.RBF_ENOCONV))
        return lam, {"iters": info.iters, "restarts": info.restarts, "converged": bool(info.converged),
                     "fallback_used": int(info.fallback_used), "true_res": info.true_res,
                     "seconds": info.seconds, "history": list(info.history[:info.nhistory]),
                "history_s": list(info.history_s[:info.nhistory])}

    def poly_terms(self) -> int:
        """Number of polynomial terms of solve_poly (rbf_poly_terms)."""
        return L.check_count(L.load().rbf_poly_terms(self._h))

    def solve_poly(self, f: torch.Tensor, lam: Optional[torch.Tensor] = None, coeffs: Optional[torch.Tensor] = None,
                   rtol: float = 1e-8, restart: int = 50, max_iters: int = 1000, time_limit_s: float = 0.0):
        """Interpolation with the kernel's polynomial terms (rbf_interp_solve_poly); returns
        (lambda, coeffs, info)."""
        self._check_vec(f)
        q = self.poly_terms()
        zero = lam is None
        if lam is None:
            lam = torch.zeros_like(f)
        self._check_vec(lam)
        if coeffs is None:
            coeffs = torch.zeros(max(q, 1), dtype=f.dtype, device=f.device)
        if coeffs.dtype != f.dtype or coeffs.device != f.device or coeffs.numel() < q:
            raise ValueError(f"coeffs must hold {q} entries of the plan's dtype on its device")
        o = L.RbfSolveOpts(restart, max_iters, L.RBF_PC_NONE, 1 if zero else 0, 0, float(time_limit_s))
        info = L.RbfSolveInfo()
        code = L.load().rbf_interp_solve_poly(self._h, _ptr(f), _ptr(lam), _ptr(coeffs), float(rtol),
                                              ctypes.byref(o), ctypes.byref(info))
        L.check(code, allow=(L.RBF_OK, L.RBF_ENOCONV))
        return lam, coeffs[:q], {"iters": info.iters, "restarts": info.restarts, "converged": bool(info.converged),
                                 "true_res": info.true_res, "seconds": info.seconds,
                                 "history": list(info.history[:info.nhistory]),
                                 "history_s": list(info.history_s[:info.nhistory])}

    # -- introspection ---------------------------------------------------------------
    def info(self) -> dict:
        inf = L.RbfPlanInfo()
        L.check(L.load().rbf_fmm_plan_info(self._h, ctypes.byref(inf)))
        out = {name: getattr(inf, name) for name, _ in L.RbfPlanInfo._fields_}
        out["lo"] = list(inf.lo)[: self.d]
        return out

    def bands(self) -> list:
        """Scale bands of a banded plan (rbf_fmm_band_info), one dict per band, the top last."""
        out = []
        for j in range(self.info()["nbands"]):
            b = L.RbfBandInfo()
            L.check(L.load().rbf_fmm_band_info(self._h, j, ctypes.byref(b)))
            out.append({name: getattr(b, name) for name, _ in L.RbfBandInfo._fields_ if name != "reserved"})
        return out

    def tree(self) -> dict:
        inf = self.info()
        nl, nn = inf["nleaves"], inf["nnear"]
        perm = np.empty(self.n, np.int64)
        lb = np.empty(nl + 1, np.int32)
        lv = np.empty(nl, np.int32)
        pf = np.empty(nl, np.uint64)
        npt = np.empty(nl + 1, np.int32)
        nid = np.empty(max(nn, 1), np.int32)
        L.check(L.load().rbf_fmm_tree_export(self._h, perm.ctypes.data, lb.ctypes.data, lv.ctypes.data,
                                             pf.ctypes.data, npt.ctypes.data, nid.ctypes.data))
        return {"perm": perm, "leaf_begin": lb, "leaf_level": lv, "leaf_prefix": pf, "near_ptr": npt,
                "near_idx": nid[:nn]}

    def set_profiling(self, on: bool = True):
        L.check(L.load().rbf_fmm_set_profiling(self._h, 1 if on else 0))

    def phase_times(self) -> dict:
        ms = (ctypes.c_double * L.RBF_NPHASES)()
        calls = ctypes.c_int64()
        L.check(L.load().rbf_fmm_phase_times(self._h, ms, ctypes.byref(calls)))
        return {"calls": calls.value, **{L.PHASES[k]: ms[k] for k in range(L.RBF_NPHASES)}}

    def close(self):
        if getattr(self, "_h", None):
            L.load().rbf_fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EvalPlan(FmmPlan):
    """Plan for u_t = sum_j lambda_j Phi(y_t - x_j) at targets y other than the sources x
    (rbf_fmm_plan_eval); the plan's points are the sources followed by the targets."""

    def __init__(self, sources: torch.Tensor, targets: torch.Tensor, kernel: str = "gaussian",
                 shape: float = 0.05, tol: float = 1e-6, n_max: int = 0, max_level: int = 0,
                 min_level: int = 0, coarse_level: int = -1, coarse_radius: int = -1, nodes: int = 0,
                 band: float = 0.0, m2l_schedule: int = 0, exact: bool = False, band_transfer: int = 0,
                 stream: Optional[torch.cuda.Stream] = None):
        lib = L.load()
        if sources.dim() != 2 or targets.dim() != 2 or targets.shape[1] != sources.shape[1]:
            raise ValueError("sources (n, d) and targets (m, d) must share d")
        if targets.dtype != sources.dtype or targets.device != sources.device:
            raise ValueError("sources and targets must share dtype and device")
        self.n_src, self.d = sources.shape
        self.m = targets.shape[0]
        self.n = self.n_src + self.m
        self.dtype = sources.dtype
        self.device = sources.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(sources.device)
        opts = _opts(n_max, max_level, min_level, coarse_level, coarse_radius, nodes, band, m2l_schedule, exact,
                     band_transfer)
        h = ctypes.c_void_p()
        tp = _ptr(targets) if self.m > 0 else None
        L.check(lib.rbf_fmm_plan_eval(_ptr(sources), self.n_src, tp, self.m, self.d, _dtype_code(sources),
                                      _KERNELS[kernel], float(shape), float(tol), ctypes.byref(opts),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.kernel, self.shape, self.tol = kernel, shape, tol

    def _check(self, v: torch.Tensor, k: int):
        if v.shape != (k,) or v.dtype != self.dtype or v.device != self.device:
            raise ValueError(f"expected a ({k},) {self.dtype} vector on {self.device}")

    def eval(self, lam: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """u at the targets for weights lam at the sources (rbf_fmm_eval)."""
        self._check(lam, self.n_src)
        if out is None:
            out = torch.empty(self.m, dtype=self.dtype, device=self.device)
        self._check(out, self.m)
        L.check(L.load().rbf_fmm_eval(self._h, _ptr(lam), out.data_ptr() if self.m > 0 else None))
        return out

    def direct(self, lam: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The exact sum at the targets (rbf_direct_eval)."""
        self._check(lam, self.n_src)
        if out is None:
            out = torch.empty(self.m, dtype=self.dtype, device=self.device)
        self._check(out, self.m)
        L.check(L.load().rbf_direct_eval(self._h, _ptr(lam), out.data_ptr() if self.m > 0 else None))
        return out
