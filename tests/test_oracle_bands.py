"""Pins of oracle/bands.py: the scale bands of the multiquadric kernels against numerical
integration of their Gaussian superpositions and against the kernels themselves, and the
sample-based translation factor (eq. "M2Loperator") against the analytic Gaussian factor,
exact reproduction at lattice points and the transform of a Gaussian mixture."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import bands as B
from oracle import rbf

C_MQ = 0.02
KERNELS = [B.MQ, B.IMQ]


def _kernel_b(kernel, b):
    return b if kernel == B.MQ else 1.0 / b


@pytest.mark.parametrize("kernel", KERNELS)
def test_closed_forms_equal_the_integrals(kernel):
    """Band, residual and top closed forms = numerical s-integrals of the superposition."""
    for b in (0.02, 0.05, 0.3, 1.7):
        for lo, hi in ((0.01, 0.014), (0.05, 0.1), (0.7, 1.4)):
            num, _ = quad(lambda s: B.density(kernel, s, b), lo, hi, epsabs=0, epsrel=1e-13)
            assert B.band(kernel, b, lo, hi) == pytest.approx(num, rel=1e-10, abs=1e-15)
        s0 = 0.01
        num, _ = quad(lambda s: B.density(kernel, s, b), 0.0, s0, epsabs=0, epsrel=1e-13, limit=200)
        assert B.residual(kernel, b, s0) == pytest.approx(num, rel=1e-9, abs=1e-15)
        st = 2.0
        if kernel == B.IMQ:
            num, _ = quad(lambda s: B.density(kernel, s, b), st, np.inf, epsabs=0, epsrel=1e-13)
            assert B.top(kernel, b, st) == pytest.approx(num, rel=1e-10)
        else:
            # top = the kernel minus every narrower width (their density integrated from 0)
            num, _ = quad(lambda s: B.density(kernel, s, b), 0.0, st, epsabs=0, epsrel=1e-13, limit=200)
            assert B.top(kernel, b, st) == pytest.approx(b - num, rel=1e-10)


@pytest.mark.parametrize("kernel", KERNELS)
def test_bands_add_up_to_the_kernel(kernel):
    """residual + bands + top = the kernel, with the kernel from oracle.rbf (independent)."""
    s0, st = 0.0107, 2.07
    edges = [s0]
    while edges[-1] * math.sqrt(2) < st:
        edges.append(edges[-1] * math.sqrt(2))
    edges.append(st)
    r = np.concatenate([[0.0], np.geomspace(1e-4, 3.0, 200)])
    b = np.sqrt(r * r + C_MQ ** 2)
    tot = B.residual(kernel, b, s0) + B.top(kernel, b, st)
    for lo, hi in zip(edges[:-1], edges[1:]):
        tot = tot + B.band(kernel, b, lo, hi)
    ref = rbf.phi_of_r2(kernel, r * r, C_MQ)
    np.testing.assert_allclose(tot, ref, rtol=1e-13, atol=1e-15)


def test_bands_decay_and_residual_is_short_range():
    """A band is below 1e-12 of its value at 0 from 8 widths s_hi on; the residual is
    below 1e-9 of s0 from 6 sqrt(2) s0 on (the near zone of the product)."""
    for kernel in KERNELS:
        lo, hi = 0.02, 0.02 * math.sqrt(2)
        b0 = B.band(kernel, C_MQ, lo, hi)
        assert abs(B.band(kernel, 8 * hi, lo, hi)) < 1e-12 * abs(b0)
        s0 = 0.01
        x = 6 * math.sqrt(2) * s0
        assert abs(B.residual(kernel, x, s0)) < 1e-9 * (s0 if kernel == B.MQ else 1 / s0)


def test_sample_c_of_a_gaussian_is_the_analytic_c():
    """For K = exp(-|r|^2 / 2 s^2) the sample-based C equals (2 pi)^-d Phi_hat (eq. 28) up to
    the aliasing of the tails: sigma s = 6.5, half period > 6.5 s."""
    s, d = 0.3, 2
    sigma = 6.5 / s
    mn = 34
    C = B.sample_c(lambda r: np.exp(-np.sum(r * r, axis=-1) / (2 * s * s)), sigma, mn, d)
    xi, _ = B.trapezoid(sigma, mn)
    X = np.stack(np.meshgrid(xi, xi, indexing="ij"), -1)
    ana = np.prod(rbf.gaussian_c1(X, s), axis=-1)
    assert np.abs(C - ana).max() <= 1e-9 * ana.max()


def test_sample_c_reproduces_the_samples_at_lattice_points():
    """The quadrature kernel built from sampled C is the trigonometric interpolant: it equals
    K at every lattice point of the period, for a smooth K and for a kinked one."""
    rng = np.random.default_rng(5)
    for d, mn in ((2, 12), (3, 8)):
        sigma = 3.0
        h, q = B.sample_points(sigma, mn)
        for kfun in (B.radial(lambda b: B.band(B.MQ, b, 0.1, 0.14), C_MQ),
                     lambda r: np.sqrt(np.sum(np.asarray(r) ** 2, axis=-1)),   # |r|: kinked
                     lambda r: np.cos(np.asarray(r)[..., 0]) + np.asarray(r)[..., -1] ** 2):
            C = B.sample_c(kfun, sigma, mn, d)
            pts = rng.choice(q, size=(40, d)) * h
            np.testing.assert_allclose(B.quad_kernel(C, sigma, mn, pts), kfun(pts), rtol=0, atol=1e-11)


def test_sample_c_of_a_band_is_its_transform():
    """Sampled C of a multiquadric band = the transform of its Gaussian superposition,
    C(xi) = -sqrt(2/pi) int e^{-c^2/2s^2} (s^2 / 2 pi)^{d/2} e^{-s^2 |xi|^2 / 2} ds."""
    d, lo, hi = 2, 0.05, 0.05 * math.sqrt(2)
    sigma = 6.5 / lo
    mn = 38
    C = B.sample_c(B.radial(lambda b: B.band(B.MQ, b, lo, hi), C_MQ), sigma, mn, d)
    xi, _ = B.trapezoid(sigma, mn)
    worst, scale = 0.0, 0.0
    for i in (0, 5, 11, 19, 26, 37):
        for j in (3, 19, 30):
            k2 = xi[i] ** 2 + xi[j] ** 2
            f = lambda s: -B.SQ2PI * math.exp(-C_MQ ** 2 / (2 * s * s)) * (s * s / (2 * math.pi)) ** (d / 2) \
                * math.exp(-s * s * k2 / 2)
            ana, _ = quad(f, lo, hi, epsabs=0, epsrel=1e-12)
            worst = max(worst, abs(C[i, j] - ana))
            scale = max(scale, abs(ana))
    assert worst <= 1e-8 * scale


def test_window_is_flat_inside_and_vanishes_at_the_half_period():
    ext, tau = 1.03, 0.7
    t = np.linspace(-ext, ext, 1001)
    assert np.all(np.abs(B.window(t, ext, tau) - 1) < 1e-8)
    assert B.window(ext + 8 * tau, ext, tau) < 1e-8


def test_windowed_top_is_reproduced_inside_the_cube():
    """The windowed top band's quadrature kernel matches the top band for every difference
    inside the bounding cube (2-D, multiquadric, s_top = 2 ext)."""
    ext, d = 1.0, 2
    st, tau = 2.0, 2.8
    L = 2 * (ext + 8 * tau)
    mn = 40
    sigma = math.pi * (mn - 1) / L
    kfun = lambda r: B.top(B.MQ, np.sqrt(np.sum(r * r, -1) + C_MQ ** 2), st) * \
        np.prod(B.window(r, ext, tau), axis=-1)
    C = B.sample_c(kfun, sigma, mn, d)
    r = np.random.default_rng(3).uniform(-ext, ext, (500, d))
    ref = B.top(B.MQ, np.sqrt(np.sum(r * r, -1) + C_MQ ** 2), st)
    assert np.abs(B.quad_kernel(C, sigma, mn, r) - ref).max() < 1e-6


def test_antiperiodic_fold_reproduces_a_band_wider_than_half_the_period():
    """A band not negligible at L / 2 (4e-6 of its peak) but negligible beyond L - ext: the
    quadrature kernel (even Mn) built from folded samples matches the band on the whole
    bounding cube to 1e-8 of its peak; from plain samples, or from the periodic sum, it
    misses by more than ten times that (item 4 of the module)."""
    d, lo, ext, L = 2, 0.2, 1.0, 2.6
    hi = lo * math.sqrt(2)
    band = B.radial(lambda b: B.band(B.MQ, b, lo, hi), C_MQ)
    peak = abs(band(np.zeros((1, d)))[0])
    assert abs(band(np.array([[L / 2, 0.0]]))[0]) > 1e-6 * peak
    r = np.random.default_rng(8).uniform(-ext, ext, (400, d))
    ref = band(r)
    mn = 34
    sigma = math.pi * (mn - 1) / L
    periodic = lambda x: sum(band(np.asarray(x) + np.array([i, j]) * L)
                             for i in range(-3, 4) for j in range(-3, 4))
    errs = {}
    for name, k in (("fold", B.fold_antiperiodic(band, L, 8 * hi, d)), ("plain", band),
                    ("periodic", periodic)):
        C = B.sample_c(k, sigma, mn, d)
        errs[name] = np.abs(B.quad_kernel(C, sigma, mn, r) - ref).max() / peak
    assert errs["fold"] <= 1e-8
    assert errs["plain"] > 10 * errs["fold"] and errs["periodic"] > 10 * errs["fold"]
