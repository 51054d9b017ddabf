"""Pins of the oracle GMRES -- CPU only."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.gmres import gmres


def spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (q * ev) @ q.T


def test_finite_termination_matches_dense_solve():
    a = spd(60, 1)
    b = np.random.default_rng(2).standard_normal(60)
    x, info = gmres(lambda v: a @ v, b, restart=60, rtol=1e-13, maxiter=60)
    assert np.linalg.norm(x - np.linalg.solve(a, b)) / np.linalg.norm(x) < 1e-10
    assert info["iters"] <= 60


def test_minimal_residual_over_krylov_space():
    rng = np.random.default_rng(3)
    a = np.eye(40) + 0.3 * rng.standard_normal((40, 40)) / np.sqrt(40)
    b = rng.standard_normal(40)
    for k in (1, 3, 7, 12):
        x, info = gmres(lambda v: a @ v, b, restart=100, rtol=0.0, maxiter=k)
        # x_k minimises ||b - A y|| over y in K_k = span{b, Ab, ..., A^{k-1} b}
        K = np.zeros((40, k))
        v = b.copy()
        for j in range(k):
            K[:, j] = v
            v = a @ v
        q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(a @ q, b, rcond=None)
        best = np.linalg.norm(b - a @ (q @ y))
        assert abs(np.linalg.norm(b - a @ x) - best) <= 1e-10 * np.linalg.norm(b)


def test_restarted_against_scipy():
    rng = np.random.default_rng(4)
    a = np.eye(200) * 3 + rng.standard_normal((200, 200)) / np.sqrt(200)
    b = rng.standard_normal(200)
    x, info = gmres(lambda v: a @ v, b, restart=20, rtol=1e-10, maxiter=2000)
    xs, code = spla.gmres(a, b, restart=20, rtol=1e-12, maxiter=2000, atol=0.0)
    assert info["converged"] and code == 0
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8
    h = info["history"]
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))


def test_right_preconditioner_keeps_solution():
    a = spd(80, 5, cond=1e4)
    b = np.random.default_rng(6).standard_normal(80)
    dinv = 1.0 / np.diag(a)
    x, info = gmres(lambda v: a @ v, b, restart=80, rtol=1e-12, maxiter=400,
                    precond=lambda v: dinv * v)
    assert np.linalg.norm(a @ x - b) / np.linalg.norm(b) < 1e-11
