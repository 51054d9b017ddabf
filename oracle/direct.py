"""Oracle A: the direct O(N^2) sum of eq. (1) (section 1), FP64.  Test infrastructure only.

``direct_sum`` runs plain C loops (``oracle/csrc/direct_sum.c``, gcc -O2 -fopenmp, no
fast-math) and ``direct_sum_numpy`` the same definition in chunked numpy; a pin test
checks the two against each other and against a dense matrix built with
scipy.spatial.distance.cdist.  Targets may be a subset of the sources (the large
workloads evaluate a seeded subset of targets against all sources).

Pinned by: dense-matrix comparison, symmetry of the matrix, translation and rotation
invariance, permutation equivariance, N=1 and one-hot cases (tests/test_oracle_direct.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .rbf import GAUSSIAN, INVERSE_MULTIQUADRIC, MULTIQUADRIC, R5, THIN_PLATE, WENDLAND, phi_of_r2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "direct_sum.c")
_OUT = os.path.join(_HERE, "_build", "liboracle_direct.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, IEEE arithmetic)."""
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_direct_sum.restype = None
        lib.oracle_direct_sum.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def direct_sum(points, lam, kernel: str, shape: float, targets=None) -> np.ndarray:
    """u_i = sum_j lam_j Phi(y_i - x_j) over all sources j (eq. 1); y = targets or the sources."""
    src = np.ascontiguousarray(points, dtype=np.float64)
    n, d = src.shape
    lam64 = np.ascontiguousarray(lam, dtype=np.float64)
    tgt = src if targets is None else np.ascontiguousarray(targets, dtype=np.float64)
    nt = tgt.shape[0]
    out = np.zeros(nt)
    kid = {GAUSSIAN: 0, MULTIQUADRIC: 1, INVERSE_MULTIQUADRIC: 2, WENDLAND: 3, THIN_PLATE: 4, R5: 5}[kernel]
    _load().oracle_direct_sum(src.ctypes.data, n, d, lam64.ctypes.data, tgt.ctypes.data, nt,
                              kid, float(shape), out.ctypes.data)
    return out


def direct_sum_numpy(points, lam, kernel: str, shape: float, targets=None, chunk: int = 256):
    """Same definition as ``direct_sum`` in numpy, chunked over targets."""
    src = np.asarray(points, dtype=np.float64)
    lam64 = np.asarray(lam, dtype=np.float64)
    tgt = src if targets is None else np.asarray(targets, dtype=np.float64)
    out = np.empty(tgt.shape[0])
    for a in range(0, tgt.shape[0], chunk):
        y = tgt[a:a + chunk]
        r2 = ((y[:, None, :] - src[None, :, :]) ** 2).sum(-1)
        out[a:a + chunk] = phi_of_r2(kernel, r2, shape) @ lam64
    return out


def rel_l2(approx, exact) -> float:
    """Relative 2-norm error ||approx - exact|| / ||exact||."""
    a = np.asarray(approx, dtype=np.float64)
    e = np.asarray(exact, dtype=np.float64)
    return float(np.linalg.norm(a - e) / np.linalg.norm(e))
