"""Pins of the oracle's kernels and Fourier convention (CPU only)."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import rbf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_kernel_closed_form_points():
    assert rbf.phi_of_r2("gaussian", 0.0, 0.05) == 1.0
    # exp(-r^2/(2 s^2)) at r = s is e^-1/2
    assert abs(rbf.phi_of_r2("gaussian", 0.05 ** 2, 0.05) - math.exp(-0.5)) < 1e-15
    assert abs(rbf.phi_of_r2("multiquadric", 9.0, 4.0) - 5.0) < 1e-15
    assert rbf.phi0("multiquadric", 0.02) == 0.02


@pytest.mark.parametrize("xi", [0.0, 3.0, 17.5, 60.0])
def test_gaussian_transform_by_quadrature(xi):
    """eq. (5) convention: int exp(-x^2/(2 s^2)) exp(-i xi x) dx, integrated numerically."""
    s = 0.05
    re = integrate.quad(lambda x: math.exp(-x * x / (2 * s * s)) * math.cos(xi * x), -1, 1,
                        limit=400, epsabs=1e-14)[0]
    assert abs(rbf.gaussian_ft(np.array([xi]), s, 1) - re) < 1e-12
    # C = (2 pi)^-1 Phi_hat in 1-D equals the one-dimensional factor c1
    assert abs(rbf.gaussian_C(np.array([xi]), s, 1) - rbf.gaussian_c1(xi, s)) < 1e-15


def test_gaussian_transform_separable_3d():
    s = 0.2
    xi = np.array([1.0, -2.0, 0.5])
    c = rbf.gaussian_C(xi, s, 3)
    assert abs(c - np.prod(rbf.gaussian_c1(xi, s))) < 1e-15


def test_inverse_transform_recovers_kernel():
    """eq. (6): (2 pi)^-1 int Phi_hat(w) e^{i w x} dw = Phi(x)."""
    s = 0.1
    for x in [0.0, 0.07, 0.2]:
        val = integrate.quad(lambda w: rbf.gaussian_ft(np.array([w]), s, 1) * math.cos(w * x),
                             -200, 200, limit=400)[0] / (2 * math.pi)
        assert abs(val - math.exp(-x * x / (2 * s * s))) < 1e-10


def test_tab_rms_left_column():
    """Multiquadric collocation of the paper's 1-D model problem reproduces its RMS table."""
    rows = [l.split() for l in open(os.path.join(GOLD, "tab_rms_left.txt")) if l.strip() and l[0] != "#"]
    for n_s, rms_s, tol_s in rows:
        n = int(n_s)
        x = np.linspace(0.0, 1.0, n)
        r2 = (x[:, None] - x[None, :]) ** 2
        phi = rbf.phi_of_r2("multiquadric", r2, 1.0)
        d2 = 1.0 / (r2 + 1.0) ** 1.5          # second derivative of sqrt(t^2 + 1)
        a = -d2 + math.pi ** 2 * phi
        a[0], a[-1] = phi[0], phi[-1]
        rhs = 2 * math.pi ** 2 * np.sin(math.pi * x)
        rhs[0] = rhs[-1] = 0.0
        lam = np.linalg.solve(a, rhs)
        rms = math.sqrt(np.mean((phi @ lam - np.sin(math.pi * x)) ** 2))
        assert abs(rms / float(rms_s) - 1.0) < float(tol_s), (n, rms, rms_s)
