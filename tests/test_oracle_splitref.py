"""Pins of oracle B (brute-force near/far split) and the tolerance rule -- CPU only."""
import numpy as np
import pytest

from oracle import direct, params, splitref
from oracle import tree as T
from workloads import c1, mixed_points, normal_weights, uniform_points


def test_single_leaf_is_the_direct_sum():
    x = uniform_points(90, 2, 2)
    lam = normal_weights(90, 3)
    u = splitref.split_reference(x, lam, "gaussian", 0.05, n_max=100, lc=0, r=0, sigma=50.0, mn=8)
    assert np.max(np.abs(u - direct.direct_sum(x, lam, "gaussian", 0.05))) < 1e-13


def test_wide_band_and_period_reproduce_direct_sum():
    """No pruning, sigma s = 8 and a period far beyond the domain: the far field is exact
    to the band-limit error erfc(8/sqrt 2) ~ 1e-15."""
    x = uniform_points(600, 2, 5)
    lam = normal_weights(600, 6)
    s = 0.1
    u = splitref.split_reference(x, lam, "gaussian", s, n_max=20, lc=0, r=0,
                                 sigma=8.0 / s, mn=80)
    ref = direct.direct_sum(x, lam, "gaussian", s)
    assert direct.rel_l2(u, ref) < 1e-12


def test_rule_on_c1_meets_tolerance():
    p = c1()
    tr0 = T.build(p.points, 64, max_level=3, min_level=3)
    lo, ext = T.root_cube(p.points)
    pr = params.gauss_params(p.shape, 1e-6, 2, 4096, ext, 64)
    assert pr.lc >= 1 and pr.mn % 2 == 0
    tr = T.build(p.points, 10 ** 9, max_level=3, min_level=3)
    u = splitref.split_reference(p.points, p.lam, "gaussian", p.shape, n_max=10 ** 9, lc=min(pr.lc, 3),
                                 r=pr.r if pr.lc <= 3 else 0, sigma=pr.sigma, mn=pr.mn,
                                 max_level=3, tree=tr)
    ref = direct.direct_sum(p.points, p.lam, "gaussian", p.shape)
    err = direct.rel_l2(u, ref)
    assert err < 1e-6, err
    assert tr0.nleaves == 64


def test_rule_fp32_tolerance_on_mixed_3d():
    x = mixed_points(6000, 3, 21, 4, 0.01)
    lam = normal_weights(6000, 22)
    lo, ext = T.root_cube(x)
    s = 0.03
    pr = params.gauss_params(s, 1e-4, 3, 6000, ext, 64)
    u = splitref.split_reference(x, lam, "gaussian", s, n_max=64, lc=pr.lc, r=pr.r,
                                 sigma=pr.sigma, mn=pr.mn)
    ref = direct.direct_sum(x, lam, "gaussian", s)
    assert direct.rel_l2(u, ref) < 1e-4


def _pruned_tail(x, lam, s, lc, r):
    """Exact contribution of every pair outside the coarse stencil: sum_{j outside} lam_j Phi."""
    tr = T.build(x, 10 ** 9, max_level=lc, min_level=lc)
    d = x.shape[1]
    cc = T.coarse_cell_coords(tr.coarse_cell(lc), d, lc)
    pcell = np.repeat(cc, np.diff(tr.leaf_begin), axis=0)
    xs = x[tr.perm].astype(np.float64)
    ls = np.asarray(lam, dtype=np.float64)[tr.perm]
    tail = np.zeros(x.shape[0])
    for i in range(x.shape[0]):
        out = np.any(np.abs(pcell - pcell[i]) > r, axis=1)
        dd = xs[out] - xs[i]
        tail[i] = np.exp(-(dd * dd).sum(1) / (2 * s * s)) @ ls[out]
    return tail, xs, ls


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_pruned_tail_is_within_its_bound(tol):
    """The coarse stencil of the rule drops only pairs farther apart than R_cut: their exact
    sum at every target is below sum |lambda| exp(-R_cut^2 / (2 s^2)), and its 2-norm is below
    tol / 4 of the product's (computed from the kernel itself, not from the fast method)."""
    x = mixed_points(3000, 3, 31, 4, 0.01)
    lam = normal_weights(3000, 32)
    s = 0.015
    lo, ext = T.root_cube(x)
    pr = params.gauss_params(s, tol, 3, 3000, ext, 8)
    assert pr.lc >= 1 and pr.r >= 1
    tail, xs, ls = _pruned_tail(x, lam, s, pr.lc, pr.r)
    bound = np.abs(ls).sum() * np.exp(-pr.rcut ** 2 / (2 * s * s))
    assert np.abs(tail).max() <= bound
    u = direct.direct_sum(xs, ls, "gaussian", s)
    assert np.linalg.norm(tail) <= 0.25 * tol * np.linalg.norm(u)


def test_near_only_structure_meets_tolerance():
    """Near-only plan: uniform tree at the deepest level with cells at least R_cut wide, the
    adjacent cells as the near field, no far field: the split reference meets tol against
    the direct sum."""
    x = mixed_points(4000, 2, 33, 3, 0.01)
    lam = normal_weights(4000, 34)
    s, tol = 0.01, 1e-6
    lo, ext = T.root_cube(x)
    lstar = params.near_only_level(s, tol, 2, ext)
    assert lstar >= 2
    tr = T.build(x, 10 ** 9, max_level=lstar, min_level=lstar)
    u = splitref.split_reference(x, lam, "gaussian", s, n_max=10 ** 9, lc=lstar, r=1, sigma=1.0, mn=4,
                                 max_level=lstar, tree=tr)
    ref = direct.direct_sum(x, lam, "gaussian", s)
    assert direct.rel_l2(u, ref) <= tol
