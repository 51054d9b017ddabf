"""Tolerance -> (band limit, nodes, coarse level) rule (oracle).  Test infrastructure only.

The paper leaves the choice of sigma and M open (low-rank section: "in practice one
chooses ...", with sigma = pi for unit-spaced samples).  The library uses the rule
below for the Gaussian exp(-r^2/(2 s^2)); it is written out here independently so that a
test can compare the plan's choice with it.  Each line is an error budget on a relative
scale (tol/4, tol/4 and tol/2, so that together they make up tol):

* band limit: s sigma = t_b with erfc(t_b / sqrt 2) = tol / 4 (the largest deviation of the
  band-limited Gaussian from the Gaussian, at r = 0; see ``bandlimit``);
* pruning radius: box pairs whose gap is at least R_cut = s sqrt(2 ln(4/tol) + 1) are
  dropped (their kernel values are below 0.61 tol / 4);
* aliasing margin: the period L must exceed the largest coordinate distance R_far of a
  kept far pair by s sqrt(2 ln(2/tol)), so that the periodic images of the band-limited
  kernel are below tol / 2 (the part of the tolerance the two budgets above leave);
* coarse level: level l (cell width w = ext / 2^l) with stencil radius r = 1 + floor(R_cut/w)
  keeps every pair closer than R_cut and gives R_far = (r + 1) w.  The rule picks the level
  with the smallest R_far among l = 1 .. min(floor(log_{2^d}(n / n_max)), floor(18 / d)),
  ties going to the coarser level, and falls back to the root (l = 0, r = 0, R_far = ext)
  when no level prunes anything;
* nodes: Mn = ceil(sigma L / pi) + 1, rounded up to an even number, at least 4.

A second structure meets the same budget without a far field (``near_only_level``): a uniform
tree at the deepest level l* >= 1 whose cells are at least R_cut wide, with the adjacent cells
as the near field; every pair closer than R_cut is then a near pair and the rest is pruned.
Which of the two a plan takes (the library switches when the far field would need more nodes
than its kernels are compiled for) is the library's engineering choice, not part of the rule;
the tests pin both structures against the direct sum and the pruned tail against its bound.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from scipy.special import erfc


@dataclass
class Params:
    sigma: float
    mn: int
    lc: int
    r: int
    rcut: float
    rfar: float
    L_req: float
    near_only: bool = False


def band_t(tol: float) -> float:
    lo, hi = 0.0, 40.0
    target = tol / 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if erfc(mid / math.sqrt(2.0)) > target:
            lo = mid
        else:
            hi = mid
    return hi


def aliasing_margin(s: float, tol: float) -> float:
    """s sqrt(2 ln(2/tol)): the Gaussian exp(-t^2 / (2 s^2)) is below tol / 2 from there on."""
    return s * math.sqrt(2.0 * math.log(2.0 / tol))


def gauss_params(s: float, tol: float, d: int, n: int, ext: float, n_max: int) -> Params:
    sigma = band_t(tol) / s
    rcut = s * math.sqrt(2.0 * math.log(4.0 / tol) + 1.0)
    margin = aliasing_margin(s, tol)
    lmax = 0
    if n > n_max:
        lmax = int(math.floor(math.log(n / n_max) / math.log(2.0 ** d)))
    lmax = max(0, min(lmax, 18 // d))
    best_l, best_r, best_far = 0, 0, ext
    for lev in range(1, lmax + 1):
        w = ext / (2 ** lev)
        r = 1 + int(math.floor(rcut / w))
        far = (r + 1) * w
        if far >= ext:
            continue
        if far < best_far:
            best_l, best_r, best_far = lev, r, far
    L = best_far + margin
    mn = int(math.ceil(sigma * L / math.pi)) + 1
    if mn % 2:
        mn += 1
    mn = max(mn, 4)
    return Params(sigma, mn, best_l, best_r, rcut, best_far, L)


def near_only_level(s: float, tol: float, d: int, ext: float) -> int:
    """The deepest level l >= 1 (at most floor(18 / d)) whose cells are at least R_cut wide, or
    0 when even the first level's cells are narrower."""
    rcut = s * math.sqrt(2.0 * math.log(4.0 / tol) + 1.0)
    lstar = 0
    while lstar + 1 <= 18 // d and ext / 2 ** (lstar + 1) >= rcut:
        lstar += 1
    return lstar
