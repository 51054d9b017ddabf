"""Radial kernels and their Fourier transforms (oracle, FP64).  Test infrastructure only.

* Gaussian: the paper lists exp(-c r^2) (Tab. "Global functions", section 2.2); the
  workloads use the shape form exp(-r^2 / (2 s^2)), i.e. c = 1/(2 s^2).
* Multiquadric: sqrt(r^2 + c^2) and inverse multiquadric 1/sqrt(r^2 + c^2) (same table).
* Wendland's compactly supported function (1 - e r)_+^3 (3 e r + 1) (section 5, the third
  kernel of the numerical examples, with the scaled support radius 1/e of its figure).
* The piecewise smooth kernels of the Fourier-transform table: the thin-plate spline r^2 log r
  (0 at r = 0) and r^5.  Both are scale-free (the shape argument is ignored).
* Fourier transform convention: eq. (5), Phi_hat(w) = int Phi(x) exp(-i w.x) dx, inverse
  with (2 pi)^-d (eq. 6).  Under this convention the Gaussian transforms to
  (2 pi s^2)^(d/2) exp(-s^2 |w|^2 / 2).  (The paper's Fourier-transform table prints the
  unitary (2 pi)^(-d/2) convention; eq. 5 is taken as the definition.)
* The quadrature coefficient of eq. (28)/(29) is C(xi) = (2 pi)^-d Phi_hat(xi).

Pins: ``tests/test_oracle_rbf.py`` checks the transform by numerical integration
(scipy.integrate.quad) and the kernels at closed-form points; the multiquadric
evaluator and its second derivative reproduce the left column of the paper's
Table "RMS errors" (tests/golden/tab_rms_left.txt).  The inverse multiquadric is pinned
to the paper's Fourier-transform table (a Bessel-K transform, by numerical integration) and
Wendland's function to its expanded polynomial, its C^2 joint at the support radius and
the sign of its radial Fourier transform by dimension (positive in 1-D, negative somewhere in
2-D and 3-D: the function is Wendland's phi_{1,1}, positive definite in one dimension only).  The thin-plate spline and r^5
are pinned by finite-difference Laplacians (4 log r + 4 in 2-D, 30 r^3 in 3-D).
"""
from __future__ import annotations

import math

import numpy as np

GAUSSIAN = "gaussian"
MULTIQUADRIC = "multiquadric"
INVERSE_MULTIQUADRIC = "inverse_multiquadric"
WENDLAND = "wendland"
THIN_PLATE = "thin_plate"
R5 = "r5"


def phi_of_r2(kernel: str, r2, shape: float):
    """Phi as a function of the squared distance r^2 (eq. 7: Phi(x - x_j) = phi(|x - x_j|))."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kernel == GAUSSIAN:
        return np.exp(-r2 / (2.0 * shape * shape))
    if kernel == MULTIQUADRIC:
        return np.sqrt(r2 + shape * shape)
    if kernel == INVERSE_MULTIQUADRIC:
        return 1.0 / np.sqrt(r2 + shape * shape)
    if kernel == WENDLAND:
        er = shape * np.sqrt(r2)
        return np.maximum(1.0 - er, 0.0) ** 3 * (3.0 * er + 1.0)
    if kernel == THIN_PLATE:
        # r^2 log r = r^2 log(r^2) / 2, continued by 0 at r = 0
        safe = np.where(r2 > 0.0, r2, 1.0)
        return np.where(r2 > 0.0, 0.5 * r2 * np.log(safe), 0.0)
    if kernel == R5:
        return r2 * r2 * np.sqrt(r2)
    raise ValueError(kernel)


def phi0(kernel: str, shape: float) -> float:
    """Phi(0): the diagonal entry of the RBF matrix (eq. 54, A^diagonal)."""
    if kernel == MULTIQUADRIC:
        return float(shape)
    if kernel == INVERSE_MULTIQUADRIC:
        return 1.0 / float(shape)
    if kernel in (THIN_PLATE, R5):
        return 0.0
    return 1.0


def gaussian_ft(xi, s: float, d: int):
    """Phi_hat(xi) of exp(-|x|^2/(2 s^2)) in the convention of eq. (5); xi has shape (..., d)."""
    xi = np.asarray(xi, dtype=np.float64)
    k2 = (xi * xi).sum(-1)
    return (2.0 * math.pi * s * s) ** (d / 2.0) * np.exp(-0.5 * s * s * k2)


def gaussian_c1(xi, s: float):
    """One-dimensional factor of C(xi) = (2 pi)^-d Phi_hat(xi) for the Gaussian.

    The Gaussian transform is a product over coordinates, so C(xi) = prod_k c1(xi_k) with
    c1(t) = (2 pi)^-1 * sqrt(2 pi) s exp(-s^2 t^2 / 2) = s / sqrt(2 pi) * exp(-s^2 t^2 / 2).
    """
    xi = np.asarray(xi, dtype=np.float64)
    return s / math.sqrt(2.0 * math.pi) * np.exp(-0.5 * s * s * xi * xi)


def gaussian_C(xi, s: float, d: int):
    """C(xi) = (2 pi)^-d Phi_hat(xi) (eq. 28/29) for the Gaussian."""
    return (2.0 * math.pi) ** (-d) * gaussian_ft(xi, s, d)
