"""Pins of the polynomial augmentation oracle (CPU only)."""
import numpy as np
import pytest

from oracle import poly
from workloads import uniform_points


def test_term_counts():
    assert [poly.nterms(3, k) for k in (-1, 0, 1, 2)] == [0, 1, 4, 10]
    assert poly.nterms(2, 2) == 6 and poly.nterms(5, 2) == 21
    t = np.array([[0.5, 2.0], [1.0, -1.0]])
    # degree 2 in 2-D: 1, t1, t2, t1^2, t1 t2, t2^2
    assert np.array_equal(poly.monomials(t, 2), np.array([[1, 0.5, 2.0, 0.25, 1.0, 4.0],
                                                          [1, 1.0, -1.0, 1.0, -1.0, 1.0]]))


@pytest.mark.parametrize("kernel,d", [("thin_plate", 2), ("r5", 3), ("multiquadric", 3)])
def test_polynomial_reproduction(kernel, d):
    """A right-hand side in the polynomial space is interpolated by the polynomial alone: the
    unique solution has lambda = 0 and the polynomial's coefficients."""
    x = uniform_points(300, d, 60 + d) * 2.0 - 0.5
    deg = poly.DEGREE[kernel]
    P = poly.basis(x, deg)
    c_true = np.random.default_rng(61).standard_normal(P.shape[1])
    lam, c = poly.augmented_solve(x, kernel, 0.1, P @ c_true)
    assert np.max(np.abs(lam)) <= 1e-8 * np.max(np.abs(c_true))
    assert np.allclose(c, c_true, rtol=0, atol=1e-8)


@pytest.mark.parametrize("kernel,d", [("thin_plate", 2), ("r5", 3), ("multiquadric", 2)])
def test_side_and_interpolation_conditions(kernel, d):
    x = uniform_points(250, d, 70 + d)
    f = np.sin(3 * x[:, 0]) + x[:, 1] ** 2
    lam, c = poly.augmented_solve(x, kernel, 0.2, f)
    P = poly.basis(x, poly.DEGREE[kernel])
    assert np.max(np.abs(P.T @ lam)) <= 1e-9 * np.abs(lam).sum()
    r2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    from oracle import rbf
    u = rbf.phi_of_r2(kernel, r2, 0.2) @ lam + P @ c
    assert np.max(np.abs(u - f)) <= 1e-9 * np.max(np.abs(f))


def test_positive_definite_kernels_carry_no_polynomial():
    x = uniform_points(50, 3, 80)
    for k in ("gaussian", "inverse_multiquadric", "wendland"):
        assert poly.basis(x, poly.DEGREE[k]).shape == (50, 0)
