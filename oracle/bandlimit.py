"""Band-limited kernel and its quadrature (oracle, FP64).  Test infrastructure only.

Definitions followed (Zhao & Stoll, sections 3 and 3.2):

* Band-limited kernel (eq. 16, 28): Phi_sigma(r) = int_{[-sigma, sigma]^d} C(xi) e^{i xi.r} dxi
  with C = (2 pi)^-d Phi_hat (eq. 5 convention).  The cut-off is the box of eq. (28), with
  unit gain inside (eq. 13 and the low-rank section; the 1/sigma factor of eq. 14 is not
  applied: it contradicts eq. 13 and the low-rank section, which use unit gain).
* Quadrature (eq. "quadrature", 29): Phi^Q(r) = sum_m w_m C(xi_m) e^{i xi_m.r}.  Reading of
  the node rule: the paper spaces the nodes Delta xi = 2 sigma / M from -sigma; this oracle
  takes the tensor trapezoid rule on Mn equally spaced nodes from -sigma to +sigma
  (spacing h = 2 sigma / (Mn - 1), end weights h/2).  In 1-D its value equals the real
  part of the paper's left-endpoint sum exactly (pinned in the tests).  The sum is real
  because C is even.
* For the Gaussian the integrand factorises over coordinates, so
  Phi_sigma(r) = prod_k phi_sigma(r_k) and Phi^Q(r) = prod_k phi^Q(r_k).

Closed forms used as pins (not used by the split reference itself):

* phi_sigma(t) = e^{-t^2/(2 s^2)} - Re[ e^{-s^2 sigma^2/2 + i sigma t} w((t/s + i s sigma)/sqrt 2) ]
  with w the Faddeeva function; its largest deviation from the Gaussian, at t = 0, is
  erfc(s sigma / sqrt 2).
* Poisson summation: phi^Q(t) = sum_n (-1)^{n (Mn-1)} phi_sigma(t - n L), L = 2 pi / h.

The band-limited Gaussian as a basis of its own (section 3, eq. 16 with the box of eq. 28):
``phi_sigma_gauss`` is Phi_sigma(r) = prod_k phi_sigma(r_k) and ``direct_sum_phi_sigma`` the
sum of eq. (1) with it, u_i = sum_j lam_j Phi_sigma(y_i - x_j), in chunked numpy.  Pinned by
a two-dimensional numerical integral over the box, the smallest-eigenvalue bound of section
3.1, and the Gaussian limit at large s sigma (tests/test_oracle_bandlimit.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import wofz

from .rbf import gaussian_c1


def nodes_weights(sigma: float, mn: int):
    """Trapezoid nodes xi_k = -sigma + k h, k = 0..mn-1, h = 2 sigma/(mn-1); weights h, h/2 at ends."""
    h = 2.0 * sigma / (mn - 1)
    xi = -sigma + h * np.arange(mn, dtype=np.float64)
    w = np.full(mn, h)
    w[0] = w[-1] = 0.5 * h
    return xi, w


def period(sigma: float, mn: int) -> float:
    """Period L = 2 pi / h of the quadrature kernel."""
    return 2.0 * math.pi / (2.0 * sigma / (mn - 1))


def phi_q_1d_gauss(t, s: float, sigma: float, mn: int):
    """One-dimensional quadrature kernel sum_k w_k c1(xi_k) cos(xi_k t) for the Gaussian."""
    xi, w = nodes_weights(sigma, mn)
    wc = w * gaussian_c1(xi, s)
    t = np.asarray(t, dtype=np.float64)
    return np.cos(t[..., None] * xi) @ wc


def phi_q_gauss(r, s: float, sigma: float, mn: int):
    """Phi^Q(r) = prod_k phi^Q(r_k) for the Gaussian; r has shape (..., d)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.ones(r.shape[:-1])
    for k in range(r.shape[-1]):
        out = out * phi_q_1d_gauss(r[..., k], s, sigma, mn)
    return out


def phi_q_leftpoint_1d_gauss(t, s: float, sigma: float, m: int):
    """The paper's printed rule (low-rank section): M nodes xi_m = -sigma + (m-1) 2 sigma/M,
    weights 2 sigma / M, complex sum; returned as a complex array."""
    dx = 2.0 * sigma / m
    xi = -sigma + dx * np.arange(m, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return np.exp(1j * t[..., None] * xi) @ (dx * gaussian_c1(xi, s))


def phi_sigma_1d_gauss(t, s: float, sigma: float):
    """Closed form of int_{-sigma}^{sigma} c1(xi) e^{i xi t} dxi for the Gaussian (Faddeeva)."""
    t = np.asarray(t, dtype=np.float64)
    z = (t / s + 1j * s * sigma) / math.sqrt(2.0)
    tail = np.exp(-0.5 * s * s * sigma * sigma + 1j * sigma * t) * wofz(z)
    return np.exp(-t * t / (2.0 * s * s)) - tail.real


def phi_q_poisson_1d_gauss(t, s: float, sigma: float, mn: int, nimg: int = 8):
    """Periodised closed form sum_{|n|<=nimg} (-1)^{n(mn-1)} phi_sigma(t - n L)."""
    L = period(sigma, mn)
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    for n in range(-nimg, nimg + 1):
        sgn = -1.0 if (n * (mn - 1)) % 2 else 1.0
        out = out + sgn * phi_sigma_1d_gauss(t - n * L, s, sigma)
    return out


def phi_sigma_gauss(r, s: float, sigma: float):
    """Phi_sigma(r) = prod_k phi_sigma(r_k): the Gaussian's transform cut off at the box
    [-sigma, sigma]^d (eq. 28) factorises over the coordinates; r has shape (..., d)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.ones(r.shape[:-1])
    for k in range(r.shape[-1]):
        out = out * phi_sigma_1d_gauss(r[..., k], s, sigma)
    return out


def direct_sum_phi_sigma(points, lam, s: float, sigma: float, targets=None, chunk: int = 256) -> np.ndarray:
    """u_i = sum_j lam_j Phi_sigma(y_i - x_j) over all sources j (eq. 1 with the band-limited
    kernel of eq. 16); y = targets or the sources.  Targets in chunks of ``chunk`` rows."""
    src = np.asarray(points, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    tgt = src if targets is None else np.asarray(targets, dtype=np.float64)
    out = np.empty(tgt.shape[0])
    for a in range(0, tgt.shape[0], chunk):
        diff = tgt[a:a + chunk, None, :] - src[None, :, :]
        out[a:a + chunk] = phi_sigma_gauss(diff, s, sigma) @ lam
    return out
