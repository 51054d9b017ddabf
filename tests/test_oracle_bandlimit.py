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
