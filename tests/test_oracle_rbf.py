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


def test_inverse_multiquadric_closed_form_points():
    assert rbf.phi_of_r2("inverse_multiquadric", 0.0, 0.25) == 4.0
    # 1/sqrt(r^2 + c^2) at r = sqrt(3) c is 1/(2c)
    assert abs(rbf.phi_of_r2("inverse_multiquadric", 3.0 * 0.3 ** 2, 0.3) - 1.0 / 0.6) < 1e-14
    assert rbf.phi0("inverse_multiquadric", 0.25) == 4.0
    r2 = np.linspace(0.0, 4.0, 41)
    prod = rbf.phi_of_r2("inverse_multiquadric", r2, 0.7) * rbf.phi_of_r2("multiquadric", r2, 0.7)
    assert np.max(np.abs(prod - 1.0)) < 4e-16


@pytest.mark.parametrize("xi", [0.25, 1.0, 3.0, 8.0])
def test_inverse_multiquadric_transform_table(xi):
    """The paper's Fourier-transform table (unitary convention) gives 1/sqrt(1 + r^2) in one
    dimension the transform sqrt(2/pi) K_0(|xi|).  The cosine integral of the oracle's kernel
    over the half line (QAWF) times 2 / sqrt(2 pi) must equal it; K_0 comes from scipy.special."""
    from scipy.special import k0
    half = integrate.quad(lambda x: float(rbf.phi_of_r2("inverse_multiquadric", x * x, 1.0)), 0.0, np.inf,
                          weight="cos", wvar=xi, limlst=200)[0]
    assert abs(2.0 * half / math.sqrt(2.0 * math.pi) - math.sqrt(2.0 / math.pi) * k0(xi)) < 1e-9


def test_wendland_polynomial_and_support():
    """(1 - e r)_+^3 (3 e r + 1) = 1 - 6 x^2 + 8 x^3 - 3 x^4 for x = e r < 1, and 0 beyond."""
    e = 2.5
    r = np.linspace(0.0, 0.6, 601)
    x = e * r
    val = rbf.phi_of_r2("wendland", r * r, e)
    poly = np.where(x < 1.0, 1.0 - 6.0 * x ** 2 + 8.0 * x ** 3 - 3.0 * x ** 4, 0.0)
    # the expanded form adds terms as large as 8 x^3: a few ulps of 8 is its own rounding
    assert np.max(np.abs(val - poly)) < 4e-15
    assert rbf.phi0("wendland", e) == 1.0
    assert rbf.phi_of_r2("wendland", (1.0 / e) ** 2, e) == 0.0
    assert np.all(val[x >= 1.0] == 0.0) and np.all(val[x < 1.0] > 0.0)


def test_wendland_c2_joint():
    """At the support radius the value and the first two derivatives vanish from the inside:
    phi(1/e - h) = (e h)^3 (4 - 3 e h), so phi / h^3 tends to 4 e^3."""
    e = 3.0
    for h in [1e-2, 1e-3]:
        r = 1.0 / e - h
        v = float(rbf.phi_of_r2("wendland", r * r, e))
        assert abs(v / h ** 3 - e ** 3 * (4.0 - 3.0 * e * h)) < 1e-6 * e ** 3


def _radial_transform(f, d, w):
    """d-dimensional Fourier transform of a radial function supported in [0, 1] at |xi| = w:
    2 int f(r) cos(w r) dr (d = 1), 2 pi int f(r) r J0(w r) dr (d = 2),
    4 pi / w int f(r) r sin(w r) dr (d = 3)."""
    from scipy.integrate import quad
    from scipy.special import j0
    if d == 1:
        g = lambda r: 2.0 * f(r) * math.cos(w * r)
    elif d == 2:
        g = lambda r: 2.0 * math.pi * f(r) * r * j0(w * r)
    else:
        g = lambda r: 4.0 * math.pi * f(r) * r * math.sin(w * r) / w
    return quad(g, 0.0, 1.0, limit=400, epsabs=1e-14, epsrel=1e-12)[0]


def test_wendland_transform_sign_by_dimension():
    """(1 - r)_+^3 (3 r + 1) is Wendland's phi_{1,1}: positive definite in one dimension only.
    Its radial Fourier transform is positive in 1-D but dips below zero in 2-D and 3-D, while
    (1 - r)_+^4 (4 r + 1) (phi_{3,1}, positive definite up to three dimensions) stays
    non-negative in 3-D.  So kernel matrices of the paper's Wendland function in 2-D and 3-D
    may be indefinite (the block preconditioner factors with pivoting)."""
    phi = lambda r: float(rbf.phi_of_r2("wendland", r * r, 1.0))
    phi31 = lambda r: (1.0 - r) ** 4 * (4.0 * r + 1.0)
    ws = np.linspace(0.5, 40.0, 160)
    t1 = np.array([_radial_transform(phi, 1, w) for w in ws])
    t2 = np.array([_radial_transform(phi, 2, w) for w in ws])
    t3 = np.array([_radial_transform(phi, 3, w) for w in ws])
    t3b = np.array([_radial_transform(phi31, 3, w) for w in ws])
    assert t1.min() > 0.0
    assert t2.min() < -1e-7 * t2.max()
    assert t3.min() < -1e-6 * t3.max()
    assert t3b.min() > -1e-12 * t3b.max()


def laplacian_fd(f, p, h):
    """Second-order central-difference Laplacian of f at the point p."""
    p = np.asarray(p, dtype=np.float64)
    acc = 0.0
    for k in range(p.shape[0]):
        e = np.zeros_like(p)
        e[k] = h
        acc += (f(p + e) - 2.0 * f(p) + f(p - e)) / (h * h)
    return acc


@pytest.mark.parametrize("p", [[0.3, 0.4], [1.5, -0.2], [0.05, 0.02]])
def test_thin_plate_laplacian_2d(p):
    """r^2 log r in the plane has the Laplacian 4 log r + 4 away from the origin (it is the
    biharmonic fundamental solution up to a constant)."""
    f = lambda q: float(rbf.phi_of_r2("thin_plate", float(np.dot(q, q)), 1.0))
    r = math.hypot(*p)
    h = 1e-4 * r
    assert abs(laplacian_fd(f, p, h) - (4.0 * math.log(r) + 4.0)) < 1e-4 * (1.0 + abs(4.0 * math.log(r)))


@pytest.mark.parametrize("p", [[0.3, 0.4, 0.1], [1.0, -2.0, 0.5]])
def test_r5_laplacian_3d(p):
    """Delta r^k = k (k + d - 2) r^(k-2): r^5 in 3-D has the Laplacian 30 r^3."""
    f = lambda q: float(rbf.phi_of_r2("r5", float(np.dot(q, q)), 1.0))
    r = math.sqrt(sum(t * t for t in p))
    h = 1e-4 * r
    assert abs(laplacian_fd(f, p, h) - 30.0 * r ** 3) < 1e-5 * 30.0 * r ** 3 + 1e-9


def test_piecewise_smooth_closed_form_points():
    assert rbf.phi_of_r2("thin_plate", 0.0, 1.0) == 0.0
    assert rbf.phi_of_r2("thin_plate", 1.0, 1.0) == 0.0
    assert abs(rbf.phi_of_r2("thin_plate", math.e ** 2, 1.0) - math.e ** 2) < 1e-14
    assert rbf.phi_of_r2("r5", 4.0, 1.0) == 32.0
    assert rbf.phi0("thin_plate", 1.0) == 0.0 and rbf.phi0("r5", 1.0) == 0.0


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
