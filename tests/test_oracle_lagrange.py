"""Pins of the Lagrange transfer oracle (CPU only)."""
import os

import numpy as np
import pytest

from oracle import lagrange

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tab_halfwaveerror.txt")


def printed():
    """{K: (value, half a unit of its last printed digit)}"""
    from decimal import Decimal
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    return {int(k): (float(v), 0.5 * 10.0 ** Decimal(v).as_tuple().exponent) for k, v in rows}


@pytest.mark.parametrize("K", [5, 8, 12])
def test_basis_is_cardinal_and_exact_on_polynomials(K):
    xk = lagrange.nodes(K)
    assert np.allclose(lagrange.basis(xk, xk), np.eye(K), atol=1e-14)
    t = np.linspace(-2.0, 2.0, 37)
    P = lagrange.basis(xk, t)
    assert np.allclose(P.sum(1), 1.0, atol=1e-12)
    c = np.random.default_rng(K).standard_normal(K)          # a polynomial of degree K - 1
    assert np.allclose(P @ np.polyval(c, xk), np.polyval(c, t), rtol=0, atol=1e-10)


def test_error_decreases_with_K():
    e = [lagrange.halfwave_error(K) for K in range(5, 13)]
    assert all(b < a for a, b in zip(e, e[1:]))


def test_table_at_the_band_edge():
    """For K = 8, 11 and 12 the largest error sits at xi = +-pi, a point of every sampling of
    the band: the oracle reproduces the printed values to their digits."""
    tab = printed()
    for K in (8, 11, 12):
        v, half = tab[K]
        for nxi in (21, 1001):
            assert abs(lagrange.halfwave_error(K, nxi=nxi) - v) <= half, K


def test_table_between_sampled_and_continuous_maxima():
    """The table does not state how xi was sampled.  Every printed value lies between the maximum
    over 21 equispaced xi (the coarsest sampling tried) and the continuous maximum (10001 points),
    up to the rounding of the printed digits."""
    tab = printed()
    for K, (v, half) in tab.items():
        lo = lagrange.halfwave_error(K, nxi=21)
        hi = lagrange.halfwave_error(K, nxi=10001)
        assert lo - half <= v <= hi + half, (K, lo, v, hi)
