"""Parity at the full sizes of the benchmark workloads, in the launch configurations
bench.py times, on sampled outputs the oracle computes one by one (or, for the solve,
properties that hold at any size).  The 2^20-point 3-D product is in test_gpu_fmm.py.

* 512 batched 3-D problems, autotuned, FP32 at tol 1e-4, graph launch: 12 sampled problems
  x 256 targets against the FP64 direct sum over all of each problem's sources;
* 5-D, N = 2^18, FP32 at tol 1e-5, leaf capacity 512: 512 sampled targets;
* the 2^21-point 3-D Gaussian solve (FP64 product at tol 1e-6): 50 GMRES(50) iterations;
  the reported true residual equals ||f - A lambda|| / ||f|| recomputed with a separate
  product, and A lambda agrees with the FP64 direct sum at 256 sampled points.
"""
import numpy as np
import pytest

from oracle import direct

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def test_batched_512_problems_sampled():
    from paper_1606_07652_amd import BatchPlan
    from workloads import c3
    probs = c3(512)
    off = np.concatenate([[0], np.cumsum([p.points.shape[0] for p in probs])]).astype(np.int64)
    X = torch.as_tensor(np.concatenate([p.points for p in probs]), device="cuda")
    lam = torch.as_tensor(np.concatenate([p.lam for p in probs]), device="cuda")
    shapes = np.array([p.shape for p in probs])
    print(f"[c3] {len(probs)} problems, n={int(off[-1])}", flush=True)
    b = BatchPlan(X, off, shapes, kernel="gaussian", tol=1e-4, autotune=True)
    u = b.matvec(lam)
    b.matvec(lam, u)   # a second call replays the graph
    u = u.double().cpu().numpy()
    rng = np.random.default_rng(321)
    worst = 0.0
    for q in np.sort(rng.choice(len(probs), 12, replace=False)):
        p = probs[q]
        n = p.points.shape[0]
        idx = np.sort(rng.choice(n, min(256, n), replace=False))
        xs = p.points.astype(np.float64)
        ref = direct.direct_sum(xs, p.lam.astype(np.float64), "gaussian", p.shape, targets=xs[idx])
        err = direct.rel_l2(u[off[q]:off[q + 1]][idx], ref)
        worst = max(worst, err)
        assert err <= 1e-4, (q, err)
    print(f"[c3] worst sampled rel-L2 {worst:.3e}", flush=True)
    b.close()


def test_five_d_2pow18_sampled():
    from paper_1606_07652_amd import FmmPlan
    from workloads import c4
    w = c4()
    p = FmmPlan(torch.as_tensor(w.points, device="cuda"), kernel="gaussian", shape=w.shape, tol=w.tol, n_max=512)
    inf = p.info()
    print(f"[c4] nodes={inf['nodes']} leaves={inf['nleaves']} far={inf['far_field']}", flush=True)
    u = p.matvec(torch.as_tensor(w.lam, device="cuda")).double().cpu().numpy()
    idx = np.sort(np.random.default_rng(322).choice(w.points.shape[0], 512, replace=False))
    xs = w.points.astype(np.float64)
    ref = direct.direct_sum(xs, w.lam.astype(np.float64), "gaussian", w.shape, targets=xs[idx])
    err = direct.rel_l2(u[idx], ref)
    print(f"[c4] sampled rel-L2 {err:.3e}", flush=True)
    assert err <= w.tol
    p.close()
    torch.cuda.empty_cache()


def test_solve_2pow21_true_residual_and_sampled_product():
    from paper_1606_07652_amd import FmmPlan
    from workloads import c5
    w = c5(kernel="gaussian")
    X = torch.as_tensor(w.points.astype(np.float64), device="cuda")
    p = FmmPlan(X, kernel="gaussian", shape=w.shape, tol=1e-6, n_max=256)
    f = torch.as_tensor(w.f, dtype=torch.float64, device="cuda")
    lam, info = p.solve(f, rtol=1e-8, restart=50, max_iters=50)
    print(f"[c5] iters={info['iters']} true_res={info['true_res']:.3e}", flush=True)
    assert info["iters"] == 50 and 0 < info["true_res"] < 1
    au = p.matvec(lam)
    res = float(torch.linalg.norm(f - au) / torch.linalg.norm(f))
    assert abs(res - info["true_res"]) <= 1e-6 * info["true_res"] + 1e-12
    idx = np.sort(np.random.default_rng(323).choice(w.points.shape[0], 256, replace=False))
    xs = w.points.astype(np.float64)
    ref = direct.direct_sum(xs, lam.cpu().numpy(), "gaussian", w.shape, targets=xs[idx])
    err = direct.rel_l2(au.cpu().numpy()[idx], ref)
    print(f"[c5] sampled product rel-L2 at the solution {err:.3e}", flush=True)
    assert err <= 1e-6
    p.close()
    torch.cuda.empty_cache()
