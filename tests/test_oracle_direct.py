"""Pins of oracle A (the direct sum of eq. 1) -- CPU only."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import direct
from workloads import normal_weights, uniform_points


def phi_of_r(r, kernel, shape):
    """The kernels of the paper's tables as functions of the distance, each written in a form
    other than the oracle's (Wendland's expanded polynomial, the inverse multiquadric by hypot)."""
    if kernel == "gaussian":
        return np.exp(-r ** 2 / (2 * shape ** 2))
    if kernel == "multiquadric":
        return np.sqrt(r ** 2 + shape ** 2)
    if kernel == "inverse_multiquadric":
        return 1.0 / np.hypot(r, shape)
    if kernel == "thin_plate":
        return np.where(r > 0.0, r * r * np.log(np.where(r > 0.0, r, 1.0)), 0.0)
    if kernel == "r5":
        return r ** 5
    x = shape * r
    return np.where(x < 1.0, 1.0 - 6.0 * x ** 2 + 8.0 * x ** 3 - 3.0 * x ** 4, 0.0)


def dense(x, kernel, shape):
    return phi_of_r(cdist(x, x), kernel, shape)


KERNELS = [("gaussian", 0.05), ("multiquadric", 0.02), ("inverse_multiquadric", 0.03), ("wendland", 4.0),
           ("thin_plate", 1.0), ("r5", 1.0)]


@pytest.mark.parametrize("kernel,shape", KERNELS)
@pytest.mark.parametrize("d", [2, 3, 5])
def test_against_dense_matrix(kernel, shape, d):
    x = uniform_points(700, d, 11 + d)
    lam = normal_weights(700, 12)
    ref = dense(x, kernel, shape) @ lam
    u = direct.direct_sum(x, lam, kernel, shape)
    assert np.max(np.abs(u - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    un = direct.direct_sum_numpy(x, lam, kernel, shape)
    assert np.max(np.abs(u - un)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_symmetry_one_hot():
    x = uniform_points(300, 2, 5)
    i, j = 17, 211
    ei = np.zeros(300); ei[i] = 1
    ej = np.zeros(300); ej[j] = 1
    a_col_j = direct.direct_sum(x, ej, "gaussian", 0.1)
    a_col_i = direct.direct_sum(x, ei, "gaussian", 0.1)
    assert a_col_j[i] == a_col_i[j]
    assert abs(a_col_j[j] - 1.0) < 1e-15          # Phi(0) on the diagonal


def test_translation_rotation_permutation():
    x = uniform_points(400, 3, 7)
    lam = normal_weights(400, 8)
    u = direct.direct_sum(x, lam, "gaussian", 0.2)
    ut = direct.direct_sum(x + np.array([3.5, -2.0, 0.25]), lam, "gaussian", 0.2)
    assert np.max(np.abs(u - ut)) < 1e-11
    q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((3, 3)))
    ur = direct.direct_sum(x @ q.T, lam, "gaussian", 0.2)
    assert np.max(np.abs(u - ur)) < 1e-11
    p = np.random.default_rng(1).permutation(400)
    up = direct.direct_sum(x[p], lam[p], "gaussian", 0.2)
    assert np.max(np.abs(up - u[p])) < 1e-12


def test_single_point_and_targets():
    x = np.array([[0.3, 0.4]])
    assert direct.direct_sum(x, np.array([2.5]), "multiquadric", 0.02)[0] == 2.5 * 0.02
    xs = uniform_points(200, 2, 3)
    lam = normal_weights(200, 4)
    full = direct.direct_sum(xs, lam, "gaussian", 0.05)
    sub = direct.direct_sum(xs, lam, "gaussian", 0.05, targets=xs[50:60])
    assert np.array_equal(sub, full[50:60])


@pytest.mark.parametrize("kernel,shape", KERNELS)
def test_separate_targets_against_dense_matrix(kernel, shape):
    """Targets that are not sources (inside and outside the sources' box): the rectangular
    matrix Phi(|y_t - x_j|) from cdist, applied to lambda."""
    x = uniform_points(500, 3, 21)
    lam = normal_weights(500, 22)
    y = uniform_points(300, 3, 23) * 1.6 - 0.3
    ref = phi_of_r(cdist(y, x), kernel, shape) @ lam
    u = direct.direct_sum(x, lam, kernel, shape, targets=y)
    assert np.max(np.abs(u - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    un = direct.direct_sum_numpy(x, lam, kernel, shape, targets=y)
    assert np.max(np.abs(u - un)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_one_source_at_separate_targets():
    """One source of weight w at x0: u(y) = w exp(-|y - x0|^2 / (2 s^2)), by the closed form."""
    x0 = np.array([[0.25, 0.5, 0.75]])
    y = np.array([[0.25, 0.5, 0.75], [0.35, 0.5, 0.75], [1.25, -0.5, 0.0]])
    u = direct.direct_sum(x0, np.array([-1.5]), "gaussian", 0.1, targets=y)
    r2 = np.array([0.0, 0.01, 1.0 + 1.0 + 0.5625])
    # the third exponent is -128: one rounding of 2 s^2 moves the value by ~1e-14 relative
    assert np.allclose(u, -1.5 * np.exp(-r2 / (2 * 0.1 ** 2)), rtol=1e-13, atol=0)
