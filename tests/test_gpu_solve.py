"""GPU GMRES (rbf_interp_solve) against the oracle GMRES and the direct sum."""
import numpy as np
import pytest

from oracle import direct
from oracle.gmres import gmres
from workloads import c1, jittered_grid

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_well_conditioned_solve_matches_oracle():
    """Gaussian s = 0.01 on a jittered 64 x 64 grid (quasi-uniform, separation above half the
    spacing): well conditioned, GMRES(30) converges in a few dozen iterations."""
    from paper_1606_07652_amd import FmmPlan
    x = jittered_grid(64, 2, 31)
    f = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    print("[solve] well-conditioned n=4096", flush=True)
    p = FmmPlan(dev(x), kernel="gaussian", shape=0.01, tol=1e-8, n_max=64)
    lam, info = p.solve(dev(f), rtol=1e-9, restart=30, max_iters=300)
    lam = lam.cpu().numpy()
    assert info["converged"] and info["true_res"] <= 1e-9
    # the solution also solves the exact system to the product's accuracy
    ax = direct.direct_sum(x, lam, "gaussian", 0.01)
    assert np.linalg.norm(f - ax) / np.linalg.norm(f) < 1e-7
    xo, io = gmres(lambda v: direct.direct_sum(x, v, "gaussian", 0.01), f, restart=30, rtol=1e-9, maxiter=300)
    print(f"[solve] gpu iters={info['iters']} oracle iters={io['iters']}", flush=True)
    assert abs(info["iters"] - io["iters"]) <= max(3, 0.2 * io["iters"])
    assert np.linalg.norm(lam - xo) / np.linalg.norm(xo) < 1e-5


def test_capped_solve_reports_residual_history():
    from paper_1606_07652_amd import FmmPlan
    w = c1()
    p = FmmPlan(dev(w.points), kernel="gaussian", shape=w.shape, tol=1e-6, n_max=10 ** 9, max_level=3, min_level=3)
    lam, info = p.solve(dev(w.f), rtol=1e-8, restart=50, max_iters=200)
    assert not info["converged"] and info["iters"] == 200
    h = info["history"]
    assert len(h) >= 4 and all(h[i + 1] <= h[i] * (1 + 1e-9) for i in range(len(h) - 1))
    # the reported residual is the true residual of the fast operator
    u = p.matvec(lam).cpu().numpy()
    assert abs(np.linalg.norm(w.f - u) / np.linalg.norm(w.f) - info["true_res"]) < 1e-10
