"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and arranges them into arrays.  It holds
none of the method's arithmetic (no kernels, no quadrature, no tree), so that the
CPU oracle and the HIP path can both take their inputs from here without sharing
any code that computes a result.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64), which gives the
same stream on every platform, and draws in the fixed order documented on each
function.  The workloads follow the problem statement of the paper (centres X,
coefficients lambda, values f; section 1, eq. 1) with the shapes and
distributions of the five benchmark workloads:

* ``c1``: 2-D, N=4096 uniform in [0,1]^2, Gaussian shape 0.05, f = sin(2 pi x1) cos(2 pi x2).
* ``c2``: 3-D, N=2^20 float32, half uniform in [0,1]^3, half from 32 isotropic Gaussian
  blobs (standard deviation 0.01, centres uniform in [0,1]^3).
* ``c3``: 512 independent 3-D problems, N log-uniform in [2000, 200000], Gaussian shape
  log-uniform in [0.01, 0.1], f a random sum of 8 Fourier modes.
* ``c4``: 5-D, N=2^18 uniform in [0,1]^5.
* ``c5``: 3-D, N=2^21 mixed as ``c2``, f a sum of 16 Gaussian bumps of width 0.1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

__all__ = [
    "uniform_points", "mixed_points", "jittered_grid", "normal_weights", "Problem",
    "c1", "c2", "c3", "c4", "c5", "small_mixed", "fourier_modes_rhs", "bumps_rhs",
]


def uniform_points(n: int, d: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n points i.i.d. uniform in [0,1]^d, row-major (n, d).  One draw: ``rng.random((n, d))``."""
    rng = np.random.default_rng(seed)
    return rng.random((n, d)).astype(dtype)


def mixed_points(n: int, d: int, seed: int, nblobs: int = 32, blob_sd: float = 0.01,
                 dtype=np.float64) -> np.ndarray:
    """Half uniform, half Gaussian blobs.

    Draw order: (1) ``rng.random((n - n//2, d))`` uniform part; (2) ``rng.random((nblobs, d))``
    blob centres; (3) ``rng.standard_normal((n//2, d))`` offsets, scaled by ``blob_sd``; blob k
    takes the k-th consecutive slice of ``n//2 // nblobs`` offsets (the last blob takes the
    remainder).  Rows are uniform part first, then blobs in order.
    """
    rng = np.random.default_rng(seed)
    nu = n - n // 2
    nb = n // 2
    u = rng.random((nu, d))
    centres = rng.random((nblobs, d))
    offs = rng.standard_normal((nb, d)) * blob_sd
    per = nb // nblobs
    owner = np.minimum(np.arange(nb) // max(per, 1), nblobs - 1)
    b = centres[owner] + offs
    return np.concatenate([u, b], axis=0).astype(dtype)


def jittered_grid(side: int, d: int, seed: int, jitter: float = 0.25, dtype=np.float64) -> np.ndarray:
    """side^d points: cell centres of a regular grid on [0,1]^d, each moved by a uniform offset
    of at most jitter * spacing per coordinate (one draw: ``rng.random((side**d, d))``).
    Quasi-uniform: the separation stays above (1 - 2 jitter) * spacing."""
    rng = np.random.default_rng(seed)
    h = 1.0 / side
    g = np.stack(np.meshgrid(*([np.arange(side)] * d), indexing="ij"), -1).reshape(-1, d)
    off = (rng.random((side ** d, d)) * 2.0 - 1.0) * jitter * h
    return ((g + 0.5) * h + off).astype(dtype)


def normal_weights(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Coefficients lambda ~ N(0,1): ``default_rng(seed).standard_normal(n)``."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def fourier_modes_rhs(x: np.ndarray, seed: int, nmodes: int = 8, kmax: int = 3) -> np.ndarray:
    """f(x) = sum_k a_k cos(2 pi kappa_k . x + phi_k); draw order a (normal), kappa (integers in
    [-kmax, kmax]^d), phi (uniform [0, 2 pi))."""
    rng = np.random.default_rng(seed)
    d = x.shape[1]
    a = rng.standard_normal(nmodes)
    kap = rng.integers(-kmax, kmax + 1, size=(nmodes, d))
    ph = rng.random(nmodes) * 2.0 * math.pi
    xx = x.astype(np.float64)
    return (a[None, :] * np.cos(2.0 * math.pi * xx @ kap.T.astype(np.float64) + ph[None, :])).sum(1)


def bumps_rhs(x: np.ndarray, seed: int, nbumps: int = 16, width: float = 0.1) -> np.ndarray:
    """f(x) = sum_k a_k exp(-|x - c_k|^2 / (2 width^2)); draw order a (normal), c (uniform)."""
    rng = np.random.default_rng(seed)
    d = x.shape[1]
    a = rng.standard_normal(nbumps)
    c = rng.random((nbumps, d))
    xx = x.astype(np.float64)
    out = np.zeros(x.shape[0])
    for k in range(nbumps):
        out += a[k] * np.exp(-((xx - c[k]) ** 2).sum(1) / (2.0 * width * width))
    return out


@dataclass
class Problem:
    name: str
    points: np.ndarray          # (n, d)
    lam: np.ndarray             # (n,)
    f: Optional[np.ndarray]     # (n,) right-hand side for the interpolation solve
    kernel: str                 # "gaussian" or "multiquadric"
    shape: float                # Gaussian s in exp(-r^2/(2 s^2)), or multiquadric c
    tol: float


def c1() -> Problem:
    """2-D N=4096 uniform, Gaussian s=0.05, seed 1 (points then lambda from one stream)."""
    rng = np.random.default_rng(1)
    x = rng.random((4096, 2))
    lam = rng.standard_normal(4096)
    f = np.sin(2 * math.pi * x[:, 0]) * np.cos(2 * math.pi * x[:, 1])
    return Problem("c1_2d_gauss_n4096", x, lam, f, "gaussian", 0.05, 1e-6)


def c2(kernel: str = "gaussian", n: int = 1 << 20, seed: int = 2) -> Problem:
    """3-D mixed uniform/blob float32 points; Gaussian s=0.03 or multiquadric c=0.02."""
    x = mixed_points(n, 3, seed, 32, 0.01, dtype=np.float32)
    lam = normal_weights(n, seed + 1000, dtype=np.float32)
    shape = 0.03 if kernel == "gaussian" else 0.02
    return Problem(f"c2_3d_mixed_{kernel}_n{n}", x, lam, None, kernel, shape, 1e-6)


def small_mixed(n: int, d: int, seed: int, kernel: str = "gaussian", shape: float = 0.03,
                nblobs: int = 4, dtype=np.float64) -> Problem:
    """Scaled-down mixed workload for parity tests."""
    x = mixed_points(n, d, seed, nblobs, 0.01, dtype=dtype)
    lam = normal_weights(n, seed + 1000, dtype=dtype)
    return Problem(f"mixed_d{d}_n{n}_s{seed}", x, lam, None, kernel, shape, 1e-6)


def c3(nprob: int = 512, seed: int = 3) -> List[Problem]:
    """Batched problems.  Draw order from ``default_rng(seed)``: N_p (log-uniform), then s_p
    (log-uniform), each as one vector of length nprob; then per problem p the points come from
    ``default_rng(seed * 100000 + p)`` and lambda from ``default_rng(seed * 100000 + p + 50000)``."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(2e3), math.log(2e5), nprob))).astype(np.int64)
    ss = np.exp(rng.uniform(math.log(0.01), math.log(0.1), nprob))
    out = []
    for p in range(nprob):
        x = uniform_points(int(ns[p]), 3, seed * 100000 + p, dtype=np.float32)
        lam = normal_weights(int(ns[p]), seed * 100000 + p + 50000, dtype=np.float32)
        f = fourier_modes_rhs(x, seed * 100000 + p + 70000)
        out.append(Problem(f"c3_p{p}", x, lam, f, "gaussian", float(ss[p]), 1e-4))
    return out


def c4(n: int = 1 << 18, seed: int = 4) -> Problem:
    """5-D uniform, Gaussian s=0.2."""
    x = uniform_points(n, 5, seed, dtype=np.float32)
    lam = normal_weights(n, seed + 1000, dtype=np.float32)
    return Problem(f"c4_5d_gauss_n{n}", x, lam, None, "gaussian", 0.2, 1e-5)


def c5(n: int = 1 << 21, seed: int = 5, kernel: str = "multiquadric") -> Problem:
    """3-D mixed (as c2), f = 16 Gaussian bumps of width 0.1."""
    x = mixed_points(n, 3, seed, 32, 0.01, dtype=np.float32)
    lam = normal_weights(n, seed + 1000, dtype=np.float32)
    f = bumps_rhs(x, seed + 2000)
    shape = 0.02 if kernel == "multiquadric" else 0.03
    return Problem(f"c5_3d_mixed_{kernel}_n{n}", x, lam, f, kernel, shape, 1e-6)
