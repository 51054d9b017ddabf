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


def test_rule_values_c2_scale():
    pr = params.gauss_params(0.03, 1e-6, 3, 1 << 20, 1.0, 128)
    assert (pr.lc, pr.r) == (4, 3)
    assert abs(pr.rfar - 0.25) < 1e-15
    assert pr.mn == 24
