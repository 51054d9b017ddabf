"""Python binding of the preconditioner and network entry points (argument marshalling only).

Every computation runs in librbffmm (include/rbf_fmm.h): the block factorisation and
applies, the network's inference and training kernels, the training-pair builder and the
solves that harvest pairs.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .fmm import FmmPlan, _ptr

NPARAMS = L.RBF_MLP_NPARAMS
BLOCK = L.RBF_PC_BLOCK
_PREC = {"bf16": L.RBF_MLP_BF16, "f32": L.RBF_MLP_F32}
_KINDS = {"block_jacobi": L.RBF_PC_BLOCK_JACOBI, "learned": L.RBF_PC_LEARNED}


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f32(t: torch.Tensor, shape=None) -> int:
    if t.dtype != torch.float32:
        raise TypeError("expected a float32 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return _ptr(t)


class Mlp:
    """The 64-256-256-256-64 ReLU network of the learned preconditioner (rbf_mlp_*)."""

    def __init__(self, params: Optional[np.ndarray] = None, seed: int = 0, _handle=None):
        lib = L.load()
        if _handle is not None:
            self._h = _handle
            return
        h = ctypes.c_void_p()
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.shape != (NPARAMS,):
                raise ValueError(f"params must have {NPARAMS} values")
            L.check(lib.rbf_mlp_create(p.ctypes.data, seed, ctypes.byref(h)))
        else:
            L.check(lib.rbf_mlp_create(None, seed, ctypes.byref(h)))
        self._h = h

    @classmethod
    def load(cls, path: str) -> "Mlp":
        h = ctypes.c_void_p()
        L.check(L.load().rbf_mlp_load(str(path).encode(), ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path: str):
        L.check(L.load().rbf_mlp_save(self._h, str(path).encode()))

    def params(self) -> np.ndarray:
        out = np.empty(NPARAMS, np.float32)
        L.check(L.load().rbf_mlp_get_params(self._h, out.ctypes.data))
        return out

    def forward(self, x: torch.Tensor, precision: str = "bf16", out: Optional[torch.Tensor] = None) -> torch.Tensor:
        rows = x.shape[0]
        if out is None:
            out = torch.empty((rows, BLOCK), dtype=torch.float32, device=x.device)
        L.check(L.load().rbf_mlp_forward(self._h, _f32(x, (rows, BLOCK)), rows, _f32(out, (rows, BLOCK)),
                                         _PREC[precision], _stream(x.device)))
        return out

    def forward_static(self, x: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """FP32 forward through rbf_mlp_forward_static (no allocation inside the library;
        at most RBF_MLP_STATIC_MAX_ROWS rows; `out` is preallocated by the caller)."""
        rows = x.shape[0]
        L.check(L.load().rbf_mlp_forward_static(self._h, _f32(x, (rows, BLOCK)), rows, _f32(out, (rows, BLOCK)),
                                                _stream(x.device)))
        return out

    def loss_grad(self, x: torch.Tensor, t: torch.Tensor, w: torch.Tensor):
        rows = x.shape[0]
        g = np.empty(NPARAMS, np.float32)
        loss = ctypes.c_double()
        L.check(L.load().rbf_mlp_loss_grad(self._h, _f32(x, (rows, BLOCK)), _f32(t, (rows, BLOCK)),
                                           _f32(w, (rows,)), rows, ctypes.byref(loss), g.ctypes.data,
                                           _stream(x.device)))
        return loss.value, g

    def train(self, x: torch.Tensor, t: torch.Tensor, w: torch.Tensor, epochs: int = 100, batch: int = 512,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, val_frac: float = 0.1,
              patience: int = 0, seed: int = 0) -> dict:
        rows = x.shape[0]
        o = L.RbfTrainOpts(epochs, batch, patience, 0, lr, beta1, beta2, eps, val_frac, seed)
        inf = L.RbfTrainInfo()
        L.check(L.load().rbf_mlp_train(self._h, _f32(x, (rows, BLOCK)), _f32(t, (rows, BLOCK)), _f32(w, (rows,)),
                                       rows, ctypes.byref(o), _stream(x.device), ctypes.byref(inf)))
        k = inf.nhist
        return {"epochs_run": inf.epochs_run, "best_epoch": inf.best_epoch, "init_val_loss": inf.init_val_loss,
                "best_val_loss": inf.best_val_loss, "final_train_loss": inf.final_train_loss,
                "seconds": inf.seconds, "train_loss": list(inf.train_loss[:k]), "val_loss": list(inf.val_loss[:k])}

    def close(self):
        if getattr(self, "_h", None):
            L.load().rbf_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nblocks(plan: FmmPlan) -> int:
    return (plan.n + BLOCK - 1) // BLOCK


def block_jacobi(plan: FmmPlan, reg: float = -1.0):
    """Build the block-Jacobi inverses of (A_bb + reg I); reg < 0 picks the default (1e-2)."""
    L.check(L.load().rbf_pc_block_jacobi(plan._h, float(reg)))


def learned_features(plan: FmmPlan, reg: float = -1.0):
    """Build the inverses that form the learned map's features; reg < 0 picks the default (1e-6)."""
    L.check(L.load().rbf_pc_learned_features(plan._h, float(reg)))


def set_learned(plan: FmmPlan, mlp: Optional[Mlp]):
    L.check(L.load().rbf_pc_set_learned(plan._h, mlp._h if mlp is not None else None))
    plan._mlp_ref = mlp   # keep the network alive while the plan may use it


def apply(plan: FmmPlan, kind: str, v: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    if v.dtype != torch.float64 or v.shape != (plan.n,):
        raise ValueError("v must be a float64 vector of the plan's length")
    if out is None:
        out = torch.empty_like(v)
    L.check(L.load().rbf_pc_apply(plan._h, _KINDS[kind], _ptr(v), _ptr(out)))
    return out


def pairs(plan: FmmPlan, r: torch.Tensor, e: torch.Tensor):
    nb = nblocks(plan)
    dev = r.device
    x = torch.empty((nb, BLOCK), dtype=torch.float32, device=dev)
    t = torch.empty_like(x)
    w = torch.empty(nb, dtype=torch.float32, device=dev)
    for v in (r, e):
        if v.dtype != torch.float64 or v.shape != (plan.n,):
            raise ValueError("r and e must be float64 vectors of the plan's length")
    L.check(L.load().rbf_pc_pairs(plan._h, _ptr(r), _ptr(e), _ptr(x), _ptr(t), _ptr(w)))
    return x, t, w


def harvest(plan: FmmPlan, f: torch.Tensor, caps=(0, 1, 2, 5, 10, 20, 50, 100, 200), rtol: float = 1e-10,
            max_iters: int = 1000, precond: str = "none"):
    """Training rows from solves of A lambda = f (rbf_pc_harvest); precond 'none' or 'block_jacobi'."""
    nb = nblocks(plan)
    c = np.ascontiguousarray(caps, dtype=np.int32)
    dev = f.device
    x = torch.empty((len(c) * nb, BLOCK), dtype=torch.float32, device=dev)
    t = torch.empty_like(x)
    w = torch.empty(len(c) * nb, dtype=torch.float32, device=dev)
    plan._check_vec(f)
    kind = {"none": L.RBF_PC_NONE, "block_jacobi": L.RBF_PC_BLOCK_JACOBI}[precond]
    L.check(L.load().rbf_pc_harvest(plan._h, _ptr(f), float(rtol), int(max_iters), kind, c.ctypes.data, len(c),
                                    _ptr(x), _ptr(t), _ptr(w)))
    return x, t, w


def train_file(plans, fs, path: str, caps=None, rtol: float = 1e-10, max_iters: int = 1000, seed: int = 0,
               epochs: int = 100, batch: int = 512, lr: float = 1e-3, val_frac: float = 0.1, patience: int = 0,
               shuffle_seed: int = 0) -> dict:
    """The whole training in one library call (rbf_pc_train): rows harvested from solves of every
    plan with its right-hand side, a network from `seed` trained on them, written to `path`."""
    if len(plans) != len(fs) or not plans:
        raise ValueError("one right-hand side per plan")
    for p_, f_ in zip(plans, fs):
        p_._check_vec(f_)
    hp = (ctypes.c_void_p * len(plans))(*[p_._h.value for p_ in plans])
    hf = (ctypes.c_void_p * len(fs))(*[f_.data_ptr() for f_ in fs])
    c = None if caps is None else np.ascontiguousarray(caps, dtype=np.int32)
    o = L.RbfTrainOpts(epochs, batch, patience, 0, lr, 0.9, 0.999, 1e-8, val_frac, shuffle_seed)
    inf = L.RbfTrainInfo()
    L.check(L.load().rbf_pc_train(hp, hf, len(plans), float(rtol), int(max_iters),
                                  None if c is None else c.ctypes.data, 0 if c is None else len(c), int(seed),
                                  ctypes.byref(o), str(path).encode(), ctypes.byref(inf)))
    k = inf.nhist
    return {"epochs_run": inf.epochs_run, "best_epoch": inf.best_epoch, "init_val_loss": inf.init_val_loss,
            "best_val_loss": inf.best_val_loss, "seconds": inf.seconds, "val_loss": list(inf.val_loss[:k])}


def load_into(plan: FmmPlan, path: str) -> Mlp:
    """Load a weight file and attach it to the plan (rbf_pc_load); returns the network, which the
    plan keeps alive."""
    h = ctypes.c_void_p()
    L.check(L.load().rbf_pc_load(plan._h, str(path).encode(), ctypes.byref(h)))
    m = Mlp(_handle=h)
    plan._mlp_ref = m
    return m
