"""Polynomial augmentation of the interpolation system (oracle, FP64).  Test infrastructure only.

The paper's kernels include conditionally positive definite ones: the multiquadric (order 1)
and, in its Fourier-transform table (section 3), the thin-plate spline r^2 log r (order 2) and
r^5 (order 3).  For a kernel of order m the interpolant carries a polynomial of degree m - 1,
    u(x) = sum_j lambda_j Phi(x - x_j) + sum_k c_k p_k(t(x)),
with the side conditions sum_j lambda_j p_k(t(x_j)) = 0, i.e. the square system
    [A  P] [lambda]   [f]
    [P' 0] [c     ] = [0].
(The paper does not treat this; it is the textbook construction for such kernels.)  The
positive definite kernels (Gaussian, inverse multiquadric, Wendland) carry no polynomial.

Basis: monomials of t = (x - lo) / ext, where lo is the componentwise minimum of the points and
ext the largest side of their bounding box (the tree's root cube): degree 0 is [1], degree 1
appends t_1 .. t_d, degree 2 appends t_a t_b for a <= b in row-major order.

Pinned by (tests/test_oracle_poly.py): polynomial reproduction (a right-hand side that is a
polynomial of the degree gives lambda = 0 and its own coefficients), the side conditions
P' lambda = 0, the interpolation conditions, and the term counts 1, 1 + d, 1 + d + d(d+1)/2.
"""
from __future__ import annotations

import numpy as np

from . import rbf
from .tree import root_cube

DEGREE = {rbf.GAUSSIAN: -1, rbf.INVERSE_MULTIQUADRIC: -1, rbf.WENDLAND: -1, rbf.MULTIQUADRIC: 0,
          rbf.THIN_PLATE: 1, rbf.R5: 2}


def nterms(d: int, degree: int) -> int:
    if degree < 0:
        return 0
    return 1 + (d if degree >= 1 else 0) + (d * (d + 1) // 2 if degree >= 2 else 0)


def monomials(t, degree: int) -> np.ndarray:
    """(n, q) matrix of the basis at the normalised points t (n, d)."""
    t = np.asarray(t, dtype=np.float64)
    n, d = t.shape
    cols = []
    if degree >= 0:
        cols.append(np.ones(n))
    if degree >= 1:
        cols += [t[:, a] for a in range(d)]
    if degree >= 2:
        cols += [t[:, a] * t[:, b] for a in range(d) for b in range(a, d)]
    return np.stack(cols, axis=1) if cols else np.zeros((n, 0))


def basis(points, degree: int) -> np.ndarray:
    lo, ext = root_cube(points)
    return monomials((np.asarray(points, dtype=np.float64) - lo) / ext, degree)


def augmented_matrix(points, kernel: str, shape: float) -> np.ndarray:
    x = np.asarray(points, dtype=np.float64)
    r2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    A = rbf.phi_of_r2(kernel, r2, shape)
    P = basis(x, DEGREE[kernel])
    q = P.shape[1]
    return np.block([[A, P], [P.T, np.zeros((q, q))]])


def augmented_solve(points, kernel: str, shape: float, f):
    """(lambda, c) of the augmented system, by a dense FP64 solve."""
    M = augmented_matrix(points, kernel, shape)
    n = np.asarray(points).shape[0]
    rhs = np.concatenate([np.asarray(f, dtype=np.float64), np.zeros(M.shape[0] - n)])
    sol = np.linalg.solve(M, rhs)
    return sol[:n], sol[n:]
