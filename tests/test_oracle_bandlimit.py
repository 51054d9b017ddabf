"""Pins of the band-limited kernel and its quadrature (CPU only)."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erfc

from oracle import bandlimit
from oracle.rbf import gaussian_c1


@pytest.mark.parametrize("t", [0.0, 0.013, 0.05, 0.11, 0.4])
def test_closed_form_against_integral(t):
    s, sig = 0.05, 90.0
    num = integrate.quad(lambda x: gaussian_c1(x, s) * math.cos(x * t), -sig, sig, limit=500,
                         epsabs=1e-15)[0]
    assert abs(bandlimit.phi_sigma_1d_gauss(np.array(t), s, sig) - num) < 1e-13


@pytest.mark.parametrize("ssig", [3.0, 4.2, 5.15, 5.5])
def test_band_limit_error_is_erfc_at_origin(ssig):
    s = 0.03
    sig = ssig / s
    t = np.linspace(-0.3, 0.3, 6001)
    dev = np.abs(bandlimit.phi_sigma_1d_gauss(t, s, sig) - np.exp(-t * t / (2 * s * s)))
    assert abs(dev.max() - erfc(ssig / math.sqrt(2))) < 1e-12 * max(1.0, dev.max()) + 1e-17
    assert np.argmax(dev) == 3000


@pytest.mark.parametrize("mn", [24, 31, 46])
def test_poisson_periodisation(mn):
    """Trapezoid quadrature kernel == periodised closed form (images (-1)^{n(Mn-1)})."""
    s, sig = 0.05, 5.15 / 0.05
    L = bandlimit.period(sig, mn)
    t = np.linspace(-1.5 * L, 1.5 * L, 601)
    q = bandlimit.phi_q_1d_gauss(t, s, sig, mn)
    # The image series of a box-truncated spectrum converges like 1/N under symmetric
    # truncation; one Richardson step removes that term.
    p1 = bandlimit.phi_q_poisson_1d_gauss(t, s, sig, mn, nimg=200)
    p2 = bandlimit.phi_q_poisson_1d_gauss(t, s, sig, mn, nimg=400)
    p = 2.0 * p2 - p1
    assert np.max(np.abs(q - p)) < 1e-11


def test_trapezoid_equals_real_part_of_left_endpoint_rule():
    s, sig, mn = 0.03, 170.0, 24
    t = np.linspace(-0.5, 0.5, 777)
    trap = bandlimit.phi_q_1d_gauss(t, s, sig, mn)
    left = bandlimit.phi_q_leftpoint_1d_gauss(t, s, sig, mn - 1)
    assert np.max(np.abs(trap - left.real)) < 1e-14


def test_quadrature_kernel_separable_and_close():
    s = 0.05
    sig = 5.15 / s
    mn = 30
    r = np.array([[0.01, -0.02, 0.03], [0.2, 0.1, -0.05]])
    q = bandlimit.phi_q_gauss(r, s, sig, mn)
    direct = np.prod(bandlimit.phi_q_1d_gauss(r, s, sig, mn), axis=-1)
    assert np.max(np.abs(q - direct)) < 1e-15
    exact = np.exp(-(r * r).sum(-1) / (2 * s * s))
    assert np.max(np.abs(q - exact)) < 3 * erfc(5.15 / math.sqrt(2))


def test_weights_sum_to_kernel_at_origin():
    s, sig, mn = 0.05, 5.15 / 0.05, 40
    xi, w = bandlimit.nodes_weights(sig, mn)
    assert abs(xi[0] + sig) < 1e-12 and abs(xi[-1] - sig) < 1e-12
    assert abs((w * gaussian_c1(xi, s)).sum() - bandlimit.phi_q_1d_gauss(np.array(0.0), s, sig, mn)) < 1e-15
    assert abs((w * gaussian_c1(xi, s)).sum() - 1.0) < 2 * erfc(5.15 / math.sqrt(2))


# ---- the band-limited Gaussian as a basis (section 3, eq. 16 with the box of eq. 28) ----

@pytest.mark.parametrize("r", [(0.05, -0.12), (0.21, 0.3), (0.0, 0.4)])
def test_box_kernel_against_2d_integral(r):
    """Phi_sigma(r) = int over the box [-sigma, sigma]^2 of C(xi) e^{i xi.r}, integrated as a 2-D
    integral (no factorisation assumed): pins the product over the axes and the box cut-off."""
    s, sig = 0.1, 25.0
    a = s / math.sqrt(2 * math.pi)

    def f(x2, x1):
        return a * a * math.exp(-0.5 * s * s * (x1 * x1 + x2 * x2)) * math.cos(x1 * r[0] + x2 * r[1])

    num = integrate.dblquad(f, -sig, sig, -sig, sig, epsabs=1e-13, epsrel=1e-12)[0]
    assert abs(bandlimit.phi_sigma_gauss(np.array(r), s, sig) - num) < 1e-11


def _sinc(z):
    return np.sinc(z / np.pi)   # sin(z) / z


@pytest.mark.parametrize("d,jitter", [(1, 0.1), (1, 0.25), (2, 0.1)])
def test_phi_sigma_smallest_eigenvalue_bound(d, jitter):
    """Section 3.1: sum_jk l_j l_k Phi_sigma(x_j - x_k) >= inf_box C * sum_jk l_j l_k
    prod_a int (1 - |xi_a|/sigma) e^{i xi_a (x_ja - x_ka)} dxi_a, and the Fejer integrals are
    sigma sinc^2(sigma t / 2); diagonal dominance then bounds the smallest eigenvalue below by
    sigma^d C(sigma, .., sigma) (1 - max_j sum_{k != j} prod_a sinc^2(sigma (x_ja - x_ka) / 2)).
    Checked on jittered grids with sigma = 2 pi / spacing (the theorem's choice)."""
    rng = np.random.default_rng(5 + d)
    s, h = 0.07, 0.1
    side = 30 if d == 1 else 7
    g = np.stack(np.meshgrid(*([np.arange(side) * h] * d), indexing="ij"), -1).reshape(-1, d)
    x = g + jitter * h * rng.uniform(-1, 1, g.shape)
    sig = 2 * math.pi / h
    diff = x[:, None, :] - x[None, :, :]
    A = bandlimit.phi_sigma_gauss(diff, s, sig)
    fejer = np.prod(_sinc(0.5 * sig * diff) ** 2, axis=-1)
    np.fill_diagonal(fejer, 0.0)
    factor = 1.0 - fejer.sum(1).max()
    assert factor > 0.3
    bound = (sig * gaussian_c1(np.array(sig), s)) ** d * factor
    lmin = np.linalg.eigvalsh(A).min()
    assert lmin >= bound * (1 - 1e-9)
    assert np.allclose(A, A.T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("ssig", [2.5, 4.0, 9.0])
def test_phi_sigma_sum_approaches_gaussian(ssig):
    """|phi_sigma - Gaussian| <= erfc(s sigma / sqrt 2) per axis and both are at most 1, so the
    sums differ by at most d erfc(s sigma / sqrt 2) sum |lam| (against the C oracle's Gaussian
    sum).  A single weight at its own point attains 1 - erf(s sigma / sqrt 2)^d, within 2% of
    the bound at s sigma = 2.5."""
    from oracle import direct
    rng = np.random.default_rng(11)
    s, d = 0.05, 3
    x = rng.random((400, d))
    lam = rng.standard_normal(400)
    u_bl = bandlimit.direct_sum_phi_sigma(x, lam, s, ssig / s)
    u_g = direct.direct_sum(x, lam, "gaussian", s)
    bound = d * erfc(ssig / math.sqrt(2)) * np.abs(lam).sum()
    dev = np.abs(u_bl - u_g).max()
    assert dev <= bound + 1e-13 * np.abs(lam).sum()
    if ssig == 2.5:
        one = np.zeros(400)
        one[0] = 1.0
        at0 = abs(bandlimit.direct_sum_phi_sigma(x, one, s, ssig / s, targets=x[:1])[0] - 1.0)
        e = erfc(ssig / math.sqrt(2))
        assert abs(at0 - (1.0 - (1.0 - e) ** d)) < 1e-14
        assert at0 >= 0.98 * d * e
