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


def test_transfer_of_a_centred_expansion_matches_its_definition():
    """A cell's expansion W(xi) = sum_j lam_j e^{-i xi.(x_j - c)} (points within half a cell
    width a of the centre c) known at one grid's nodes, moved to another grid's nodes by
    K-point stencils per axis: equals the expansion evaluated at the new nodes directly, to
    sum |lam| times d times the 1-D error of the stencils (largest |sum_k w_k e^{i xi_k y} -
    e^{i eta y}| over |y| <= a), and that error falls with K.  Grids as the banded far field
    has them: even node counts on [-sigma, sigma], target band limit below the source's."""
    rng = np.random.default_rng(4)
    d, a = 3, 0.0645
    src = np.linspace(-37.6, 37.6, 24)
    tgt = np.linspace(-27.0, 27.0, 24)
    x = rng.uniform(-a, a, (40, d))
    lam = rng.normal(0, 1, 40)

    def expansion(nodes):
        g = np.stack(np.meshgrid(*([nodes] * d), indexing="ij"), -1)
        return np.exp(-1j * (g @ x.T)) @ lam

    def err1(K):
        y = np.linspace(-a, a, 257)
        worst = 0.0
        for t in tgt:
            j, w = lagrange.stencil(src, t, K)
            worst = max(worst, np.abs(np.exp(1j * np.outer(y, src[j:j + K])) @ w - np.exp(1j * t * y)).max())
        return worst

    prev = np.inf
    for K in (6, 8, 10):
        got = lagrange.transfer(expansion(src), src, tgt, K)
        e1 = err1(K)
        assert e1 < prev
        prev = e1
        assert np.abs(got - expansion(tgt)).max() <= d * e1 * np.abs(lam).sum() * 1.01
    assert prev < 1e-9
