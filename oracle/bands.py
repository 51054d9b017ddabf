"""Scale bands of the multiquadric kernels and the sample-based translation factor
(oracle, FP64).  Test infrastructure only.

1. Translation factor from kernel samples (section 3.2, eq. "M2Loperator" and the Fourier-
   series form of Phi_hat that precedes it): the paper replaces the transform at a node by a
   Fourier series of the kernel's values on the integer lattice, C(xi_m) = (1/2 pi) sum_q
   Phi(q) e^{-i q xi_m}, with sigma = pi (unit spacing).  In physical units, with samples
   at spacing h = pi / sigma:

       C(xi) = (h / 2 pi)^d  sum_{q in Q^d}  K(q h)  e^{-i h q . xi}.

   Readings (the paper is silent or garbled here):
   * the nodes are the tensor trapezoid rule on Mn points of [-sigma, sigma] (spacing
     2 sigma / (Mn - 1), end weights halved; the reading of ``bandlimit``); the period of
     the quadrature kernel is then L = 2 pi (Mn - 1) / (2 sigma), and one period holds
     Mn - 1 samples per axis, so q runs over the Mn - 1 integers -(Mn-2)/2 .. (Mn-2)/2
     (Mn even; the printed q = -Q..Q would count the period's end twice);
   * K is the function the far field has to reproduce: a band of the kernel (item 2) or
     the windowed top band (item 3), never the raw kernel, whose periodic extension would
     have a kink.
   With these readings the quadrature kernel sum_m w_m C(xi_m) e^{i xi_m . r} is the
   trigonometric interpolant of the periodised samples: it equals K at every lattice
   point r = q h (pinned), and for a Gaussian K it equals the analytic C of eq. (28) up to
   the aliasing of the tails (pinned).

2. Scale bands.  The multiquadric sqrt(r^2 + c^2) and the inverse multiquadric
   1 / sqrt(r^2 + c^2) (Tab. "Global functions") are superpositions of Gaussians of width
   s (b = sqrt(r^2 + c^2)):

       sqrt(b^2)   = sqrt(2/pi) int_0^inf [ e^{-c^2/(2 s^2)} - e^{-b^2/(2 s^2)} ] ds + c,
       1 / b       = sqrt(2/pi) int_0^inf s^-2 e^{-b^2/(2 s^2)} ds.

   Cutting the s axis at s_0 < s_1 < ... < s_J splits the kernel into
     * the residual (s < s_0), a short-range function summed directly over near pairs,
     * bands j (s_j <= s < s_{j+1}), each a smooth Gaussian mixture that decays like a
       Gaussian of width s_{j+1}: its own band limit, period and coarse grid (the per-level
       scaling of section 4.1: band limit proportional to 1/width),
     * the top band (s >= s_J), smooth on the scale s_J but not decaying.
   Closed forms, with G(s; b) = s e^{-b^2/(2 s^2)} - b sqrt(pi/2) erfc(b / (sqrt 2 s)) an
   antiderivative of e^{-b^2/(2 s^2)} in s:
     multiquadric:  band  g = -sqrt(2/pi) [G(s_{j+1}) - G(s_j)]
                    top   T = b erf(b / (sqrt 2 s_J)) + sqrt(2/pi) s_J e^{-b^2/(2 s_J^2)}
                    resid   = b erfc(x) - sqrt(2/pi) s_0 e^{-x^2},  x = b / (sqrt 2 s_0)
     inverse mq.:   band  g = [erf(b / (sqrt 2 s_j)) - erf(b / (sqrt 2 s_{j+1}))] / b
                    top   T = erf(b / (sqrt 2 s_J)) / b
                    resid   = erfc(x) / b
   and kernel = top + sum of bands + residual, exactly (pinned against the numerical
   s-integral of the definitions and against the kernel).  This split is not in the paper:
   it is how this library gives a kernel that grows (or decays like a power) the per-level
   band limits of section 4.1.

3. Window of the top band: K_top(r) = T(r) prod_k w(r_k) with w(t) = erfc((|t| - a)/tau)/2,
   a = ext + 4 tau, which is 1 to within erfc(4)/2 < 1e-8 on |t| <= ext (every coordinate
   difference inside the bounding cube) and falls to below that at |t| = ext + 8 tau, the
   half period.  (The paper does not window; reading: the periodic extension of a growing
   kernel needs it.)

4. Anti-periodic fold (reading).  With Mn even the trapezoid nodes are the odd multiples of
   half the node spacing, so every term e^{i xi_m t} changes sign under t -> t + L: the
   quadrature kernel is anti-periodic with period L along each axis, and it interpolates the
   samples of its own anti-periodic extension.  A band that has not decayed at the half period
   L / 2 but is negligible beyond L - ext is therefore sampled as

       K_fold(r) = sum_{n in Z^d} prod_k (-1)^{n_k} K(r + n L),

   which equals K on the bounding cube (every image term there is at distance >= L - ext) and
   is smooth and anti-periodic, so its trigonometric interpolant converges; sampling K alone
   (a jump at the period's end) or its plain periodic sum (the wrong parity) converges only to
   the size of K at L / 2 (pinned: the folded samples reproduce a band inside the cube, the
   other two do not).

Parity: the closed forms are pinned against numerical integration of the definitions; the
sample-based C against the analytic Gaussian C and against lattice reproduction; bands
against the numerical transform of a Gaussian mixture.  The product built on them is judged
against oracle A (the direct sum), which is the correctness gate.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

SQ2PI = math.sqrt(2.0 / math.pi)
MQ = "multiquadric"
IMQ = "inverse_multiquadric"


def _G(s, b):
    """Antiderivative in s of exp(-b^2 / (2 s^2)) (G(0; b) = 0 for b > 0)."""
    s = np.asarray(s, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return s * np.exp(-b * b / (2.0 * s * s)) - b * math.sqrt(math.pi / 2.0) * erfc(b / (math.sqrt(2.0) * s))


def band(kernel: str, b, s_lo: float, s_hi: float):
    """Band of the kernel between widths s_lo < s_hi as a function of b = sqrt(r^2 + c^2)."""
    b = np.asarray(b, dtype=np.float64)
    if kernel == MQ:
        return -SQ2PI * (_G(s_hi, b) - _G(s_lo, b))
    if kernel == IMQ:
        r2 = math.sqrt(2.0)
        return (erf(b / (r2 * s_lo)) - erf(b / (r2 * s_hi))) / b
    raise ValueError(kernel)


def top(kernel: str, b, s_top: float):
    """Top band (all widths >= s_top) as a function of b."""
    b = np.asarray(b, dtype=np.float64)
    x = b / (math.sqrt(2.0) * s_top)
    if kernel == MQ:
        return b * erf(x) + SQ2PI * s_top * np.exp(-x * x)
    if kernel == IMQ:
        return erf(x) / b
    raise ValueError(kernel)


def residual(kernel: str, b, s0: float):
    """Residual (all widths < s0) as a function of b."""
    b = np.asarray(b, dtype=np.float64)
    x = b / (math.sqrt(2.0) * s0)
    if kernel == MQ:
        return b * erfc(x) - SQ2PI * s0 * np.exp(-x * x)
    if kernel == IMQ:
        return erfc(x) / b
    raise ValueError(kernel)


def density(kernel: str, s, b):
    """Integrand in s of the Gaussian superposition (item 2), for numerical pins."""
    s = np.asarray(s, dtype=np.float64)
    if kernel == MQ:
        return -SQ2PI * np.exp(-b * b / (2.0 * s * s))          # the b-dependent part
    if kernel == IMQ:
        return SQ2PI * np.exp(-b * b / (2.0 * s * s)) / (s * s)
    raise ValueError(kernel)


def window(t, ext: float, tau: float):
    """Window of the top band along one axis (item 3)."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    return 0.5 * erfc((t - (ext + 4.0 * tau)) / tau)


def trapezoid(sigma: float, mn: int):
    """Trapezoid nodes on [-sigma, sigma] (mn points) and their weights."""
    dxi = 2.0 * sigma / (mn - 1)
    xi = -sigma + dxi * np.arange(mn, dtype=np.float64)
    w = np.full(mn, dxi)
    w[0] = w[-1] = 0.5 * dxi
    return xi, w


def sample_points(sigma: float, mn: int):
    """Sample spacing h (one period L = (mn - 1) h) and the integer offsets q of one period (item 1)."""
    if mn % 2:
        raise ValueError("mn must be even")
    h = (2.0 * math.pi / (2.0 * sigma / (mn - 1))) / (mn - 1)
    q = np.arange(-(mn - 2) // 2, (mn - 2) // 2 + 1, dtype=np.float64)
    return h, q


def sample_c(kfun, sigma: float, mn: int, d: int):
    """C on the full tensor grid [mn]^d from samples of kfun(r) (r of shape (..., d)), by the
    plain double sum of eq. "M2Loperator" (every sample times every node)."""
    xi, _ = trapezoid(sigma, mn)
    h, q = sample_points(sigma, mn)
    grids = np.meshgrid(*([q * h] * d), indexing="ij")
    rs = np.stack(grids, axis=-1).reshape(-1, d)            # sample positions
    K = np.asarray(kfun(rs), dtype=np.float64)               # (Q^d,)
    xg = np.stack(np.meshgrid(*([xi] * d), indexing="ij"), axis=-1).reshape(-1, d)
    C = np.empty(xg.shape[0])
    for a0 in range(0, xg.shape[0], 256):
        ph = xg[a0:a0 + 256] @ rs.T                          # xi . (q h)
        C[a0:a0 + 256] = (np.exp(-1j * ph) @ K).real
    C *= (h / (2.0 * math.pi)) ** d
    return C.reshape([mn] * d)


def quad_kernel(C, sigma: float, mn: int, r):
    """sum_m w_m C(xi_m) e^{i xi_m . r} over the full grid (real part), r of shape (n, d)."""
    r = np.asarray(r, dtype=np.float64)
    d = r.shape[1]
    xi, w = trapezoid(sigma, mn)
    W = w
    for _ in range(d - 1):
        W = np.multiply.outer(W, w)
    wc = (W * C).reshape(-1)
    xg = np.stack(np.meshgrid(*([xi] * d), indexing="ij"), axis=-1).reshape(-1, d)
    out = np.empty(r.shape[0])
    for a0 in range(0, r.shape[0], 256):
        out[a0:a0 + 256] = np.cos(r[a0:a0 + 256] @ xg.T) @ wc
    return out


def radial(kfun_b, c: float):
    """Wrap a function of b into a function of the difference vector r."""
    return lambda r: kfun_b(np.sqrt(np.sum(np.asarray(r) ** 2, axis=-1) + c * c))


def fold_antiperiodic(kfun, L: float, reach: float, d: int):
    """K_fold of item 4: the images of kfun within ``reach`` of the origin cell, signed by the
    parity of their lattice offsets."""
    import itertools
    nmax = int(math.ceil(reach / L)) + 1
    offs = [np.array(n, dtype=np.float64) for n in itertools.product(range(-nmax, nmax + 1), repeat=d)]

    def f(r):
        r = np.asarray(r, dtype=np.float64)
        out = np.zeros(r.shape[:-1])
        for n in offs:
            sign = -1.0 if int(np.abs(n).sum()) % 2 else 1.0
            out = out + sign * kfun(r + n * L)
        return out
    return f
