"""GPU parity of evaluation at separate targets (rbf_fmm_plan_eval / rbf_fmm_eval) against the
oracle's direct sum of eq. 1 taken at the targets (through the C ABI).

* FP64 and FP32 within the plan's tolerance, targets inside, near and outside the sources'
  box and some equal to sources; the device direct sum at the targets to rounding;
* 2-D and 5-D; the multiquadric (a single-leaf plan: the exact sum);
* targets equal to the sources: the product's values;
* no targets; plan-type errors; the full-size configuration on sampled targets.
"""
import numpy as np
import pytest

from oracle import direct
from workloads import c2, mixed_points, normal_weights, uniform_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def eval_plan(x, y, **kw):
    from paper_1606_07652_amd import EvalPlan
    print(f"[eval plan] n={x.shape[0]} m={y.shape[0]} d={x.shape[1]} {kw}", flush=True)
    return EvalPlan(x, y, **kw)


def targets_for(x, m, seed, widen=0.3):
    """A third of the targets uniform over the unit cube widened by `widen` on each side
    (some outside the sources' box), a third jittered copies of sources, a third exactly
    sources."""
    rng = np.random.default_rng(seed)
    n, d = x.shape
    k = m // 3
    far = rng.random((k, d)) * (1 + 2 * widen) - widen
    near = x[rng.choice(n, k, replace=False)] + rng.normal(0.0, 2e-3, (k, d))
    same = x[rng.choice(n, m - 2 * k, replace=False)]
    return np.concatenate([far, near, same]).astype(x.dtype)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-6), (torch.float32, 1e-4)])
def test_eval_mixed3d_meets_tolerance(dtype, tol):
    x = mixed_points(30000, 3, 31, 8, 0.01)
    lam = normal_weights(30000, 32)
    y = targets_for(x, 9000, 33)
    p = eval_plan(dev(x, dtype), dev(y, dtype), kernel="gaussian", shape=0.03, tol=tol, n_max=64)
    inf = p.info()
    assert inf["n"] == 39000 and inf["far_field"] == 1
    u = p.eval(dev(lam, dtype)).double().cpu().numpy()
    f = (lambda a: a.astype(np.float32).astype(np.float64)) if dtype == torch.float32 else (lambda a: a)
    ref = direct.direct_sum(f(x), f(lam), "gaussian", 0.03, targets=f(y))
    err = direct.rel_l2(u, ref)
    print(f"[eval mixed3d {dtype}] rel-L2 vs direct = {err:.3e}", flush=True)
    assert err <= tol
    ud = p.direct(dev(lam, dtype)).double().cpu().numpy()
    assert direct.rel_l2(ud, ref) < (1e-13 if dtype == torch.float64 else 2e-6)


@pytest.mark.parametrize("d,n,m,s,tol", [(2, 8000, 3000, 0.02, 1e-6), (5, 3000, 1000, 0.3, 1e-4)])
def test_eval_other_dimensions(d, n, m, s, tol):
    x = uniform_points(n, d, 40 + d)
    lam = normal_weights(n, 50 + d)
    y = targets_for(x, m, 60 + d, widen=0.3 if d == 2 else 0.0)   # 5-D: a wider box needs more nodes
    dtype = torch.float64 if d == 2 else torch.float32
    p = eval_plan(dev(x, dtype), dev(y, dtype), kernel="gaussian", shape=s, tol=tol, n_max=64)
    u = p.eval(dev(lam, dtype)).double().cpu().numpy()
    f = (lambda a: a.astype(np.float32).astype(np.float64)) if dtype == torch.float32 else (lambda a: a)
    ref = direct.direct_sum(f(x), f(lam), "gaussian", s, targets=f(y))
    err = direct.rel_l2(u, ref)
    print(f"[eval d={d}] rel-L2 = {err:.3e} far={p.info()['far_field']}", flush=True)
    assert err <= tol


def test_eval_multiquadric_is_the_exact_sum():
    x = mixed_points(6000, 3, 70, 4, 0.02)
    lam = normal_weights(6000, 71)
    y = targets_for(x, 2000, 72)
    p = eval_plan(dev(x), dev(y), kernel="multiquadric", shape=0.02, tol=1e-6, exact=True)
    assert p.info()["nleaves"] == 1 and p.info()["far_field"] == 0
    u = p.eval(dev(lam)).cpu().numpy()
    ref = direct.direct_sum(x, lam, "multiquadric", 0.02, targets=y)
    assert direct.rel_l2(u, ref) <= 1e-13


def test_eval_at_the_sources_gives_the_product():
    from paper_1606_07652_amd import FmmPlan
    x = mixed_points(12000, 3, 80, 6, 0.01)
    lam = normal_weights(12000, 81)
    ref = direct.direct_sum(x, lam, "gaussian", 0.03)
    pe = eval_plan(dev(x), dev(x), kernel="gaussian", shape=0.03, tol=1e-6, n_max=64)
    ue = pe.eval(dev(lam)).cpu().numpy()
    pm = FmmPlan(dev(x), kernel="gaussian", shape=0.03, tol=1e-6, n_max=64)
    um = pm.matvec(dev(lam)).cpu().numpy()
    assert direct.rel_l2(ue, ref) <= 1e-6 and direct.rel_l2(um, ref) <= 1e-6
    assert direct.rel_l2(ue, um) <= 2e-6


def test_eval_without_targets_and_plan_types():
    from paper_1606_07652_amd import FmmPlan, RbfError
    x = uniform_points(2000, 3, 90)
    lam = dev(normal_weights(2000, 91))
    p = eval_plan(dev(x), dev(np.zeros((0, 3))), kernel="gaussian", shape=0.05, tol=1e-6, n_max=64)
    assert p.eval(lam).shape == (0,)
    q = eval_plan(dev(x), dev(uniform_points(100, 3, 92)), kernel="gaussian", shape=0.05, tol=1e-6, n_max=64)
    with pytest.raises(RbfError):
        FmmPlan.matvec(q, dev(np.zeros(2100)))          # an evaluation plan has no product
    with pytest.raises(RbfError):
        q.solve(dev(np.zeros(2100)))
    m = FmmPlan(dev(x), kernel="gaussian", shape=0.05, tol=1e-6, n_max=64)
    from paper_1606_07652_amd import _lib as L
    with pytest.raises(RbfError):                       # an ordinary plan has no targets
        L.check(L.load().rbf_fmm_eval(m._h, lam.data_ptr(), dev(np.zeros(10)).data_ptr()))
    with pytest.raises(ValueError):
        q.eval(dev(np.zeros(5)))


def test_full_size_sampled_targets():
    """2^20 mixed sources (the benchmark's), 2^18 targets uniform over the unit cube: 512
    seeded targets against the FP64 direct sum over all sources."""
    w = c2("gaussian")
    xs = w.points.astype(np.float64)
    ls = w.lam.astype(np.float64)
    y = uniform_points(1 << 18, 3, 101)
    idx = np.sort(np.random.default_rng(102).choice(y.shape[0], 512, replace=False))
    ref = direct.direct_sum(xs, ls, "gaussian", w.shape, targets=y[idx])
    p = eval_plan(dev(xs), dev(y), kernel="gaussian", shape=w.shape, tol=1e-6, n_max=256)
    u = p.eval(dev(ls)).cpu().numpy()
    err = direct.rel_l2(u[idx], ref)
    print(f"[eval c2] sampled rel-L2 = {err:.3e}", flush=True)
    assert err <= 1e-6
    p.close()
    torch.cuda.empty_cache()
