"""GPU parity of the fast product against the oracle (through the C ABI).

* tree: keys order, leaves and near lists bit-exact against oracle.tree;
* plan: parameters equal to oracle.params' rule;
* FP64 fast product equal to oracle B (same split, brute force) up to rounding;
* FP64 / FP32 fast product within the tolerance of oracle A (direct sum);
* device direct sum against oracle A;
* edge cases: one point, one leaf, duplicate points, ragged leaves;
* full size (2^20 mixed points): sampled targets against oracle A.
"""
import math
import sys

import numpy as np
import pytest

from oracle import direct, params, splitref
from oracle import tree as T
from workloads import c1, c2, mixed_points, normal_weights, uniform_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def plan(x, **kw):
    from paper_1606_07652_amd import FmmPlan
    print(f"[plan] n={x.shape[0]} d={x.shape[1]} {kw}", flush=True)
    return FmmPlan(x, **kw)


def compare_tree(p, x, n_max, max_level, min_level):
    tr = T.build(x, n_max, max_level, min_level)
    g = p.tree()
    assert np.array_equal(g["perm"], tr.perm)
    assert np.array_equal(g["leaf_begin"], tr.leaf_begin)
    assert np.array_equal(g["leaf_level"], tr.leaf_level)
    assert np.array_equal(g["leaf_prefix"], tr.leaf_prefix)
    ptr, idx = T.near_lists(tr)
    assert np.array_equal(g["near_ptr"], ptr)
    assert np.array_equal(g["near_idx"], idx)
    return tr


@pytest.mark.parametrize("case", ["c1_depth3", "mixed3d", "mixed2d_f32", "uniform5d", "duplicates"])
def test_tree_bit_exact(case):
    if case == "c1_depth3":
        x = c1().points
        kw = dict(n_max=10 ** 9, max_level=3, min_level=3, coarse_level=3, coarse_radius=3, nodes=8)
        tdt = torch.float64
    elif case == "mixed3d":
        x = mixed_points(30000, 3, 7, 8, 0.01)
        kw = dict(n_max=64, coarse_level=2, coarse_radius=1, nodes=8)
        tdt = torch.float64
    elif case == "mixed2d_f32":
        x = mixed_points(20000, 2, 8, 5, 0.01, dtype=np.float32)
        kw = dict(n_max=40, coarse_level=3, coarse_radius=2, nodes=8)
        tdt = torch.float32
    elif case == "uniform5d":
        x = uniform_points(5000, 5, 9)
        kw = dict(n_max=100, coarse_level=1, coarse_radius=1, nodes=4)
        tdt = torch.float64
    else:
        x = np.repeat(uniform_points(40, 3, 10), 5, axis=0)  # every point five times
        kw = dict(n_max=3, coarse_level=1, coarse_radius=1, nodes=4)
        tdt = torch.float64
    p = plan(dev(x, tdt), kernel="gaussian", shape=0.05, tol=1e-6, **kw)
    inf = p.info()
    compare_tree(p, x, kw["n_max"], kw.get("max_level", 64), max(kw.get("min_level", 0), kw["coarse_level"]))
    lo, ext = T.root_cube(x)
    assert inf["ext"] == ext
    assert np.array_equal(np.array(inf["lo"]), lo)


@pytest.mark.parametrize("s,tol,n,d,nmax", [(0.05, 1e-6, 4096, 2, 64), (0.03, 1e-6, 1 << 20, 3, 128),
                                            (0.03, 1e-4, 1 << 20, 3, 128), (0.2, 1e-5, 1 << 14, 5, 512)])
def test_plan_parameters_meet_the_error_budget(s, tol, n, d, nmax):
    """The plan's parameters satisfy the error budget the oracle writes out (band limit, the
    stencil holding every pair closer than R_cut, the period exceeding the stencil by the
    aliasing margin), or form a near-only tree whose cells hold R_cut."""
    x = uniform_points(n, d, 3, dtype=np.float32)
    p = plan(dev(x, torch.float32), kernel="gaussian", shape=s, tol=tol, n_max=nmax)
    inf = p.info()
    lo, ext = T.root_cube(x)
    pr = params.gauss_params(s, tol, d, n, ext, nmax)
    margin = params.aliasing_margin(s, tol)
    if inf["far_field"] == 0:
        w = ext / 2 ** inf["coarse_level"]
        assert inf["coarse_level"] == params.near_only_level(s, tol, d, ext) and inf["coarse_radius"] == 1
        assert w >= pr.rcut
        return
    assert inf["band"] * s >= params.band_t(tol) * (1 - 1e-12)
    assert inf["nodes"] % 2 == 0
    if inf["coarse_level"] >= 1:
        w = ext / 2 ** inf["coarse_level"]
        assert inf["coarse_radius"] * w >= pr.rcut
        assert abs(inf["rfar"] - (inf["coarse_radius"] + 1) * w) < 1e-12
    assert inf["period"] >= inf["rfar"] + margin - 1e-12


SPLIT_CASES = {
    # name: (points, kwargs)   -- forced parameters, both sides use the same split
    "c1_depth3": (lambda: c1().points, dict(shape=0.05, n_max=10 ** 9, max_level=3, min_level=3,
                                             coarse_level=3, coarse_radius=3, nodes=28, band=103.15)),
    "c1_root": (lambda: c1().points, dict(shape=0.05, n_max=64, coarse_level=0, coarse_radius=0,
                                          nodes=46, band=110.0)),
    "mixed3d": (lambda: mixed_points(6000, 3, 12, 4, 0.01), dict(shape=0.03, n_max=48, coarse_level=2,
                                                                  coarse_radius=1, nodes=14, band=160.0)),
    "mixed2d_ragged": (lambda: mixed_points(3001, 2, 13, 3, 0.01), dict(shape=0.04, n_max=37, coarse_level=2,
                                                                         coarse_radius=1, nodes=18, band=120.0)),
    "uniform5d": (lambda: uniform_points(3000, 5, 14), dict(shape=0.3, n_max=40, coarse_level=1,
                                                           coarse_radius=1, nodes=6, band=15.0)),
}


@pytest.mark.parametrize("case", list(SPLIT_CASES))
def test_fp64_fast_product_equals_split_reference(case):
    """eq. (37) is an exact factorisation: the FP64 fast product reproduces oracle B to rounding."""
    mk, kw = SPLIT_CASES[case]
    x = mk()
    n = x.shape[0]
    lam = normal_weights(n, 77)
    p = plan(dev(x), kernel="gaussian", tol=1e-6, **kw)
    u = p.matvec(dev(lam)).cpu().numpy()
    ref = splitref.split_reference(x, lam, "gaussian", kw["shape"], n_max=kw["n_max"],
                                   lc=kw["coarse_level"], r=kw["coarse_radius"], sigma=kw["band"],
                                   mn=kw["nodes"], max_level=kw.get("max_level", 64))
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(u - ref)) / scale
    print(f"[{case}] max|fmm - splitref|/max|u| = {err:.3e}", flush=True)
    assert err < 1e-11


def test_fp64_c1_meets_tolerance_of_direct_sum():
    p1 = c1()
    p = plan(dev(p1.points), kernel="gaussian", shape=p1.shape, tol=1e-6, n_max=10 ** 9, max_level=3,
             min_level=3)
    u = p.matvec(dev(p1.lam)).cpu().numpy()
    ref = direct.direct_sum(p1.points, p1.lam, "gaussian", p1.shape)
    err = direct.rel_l2(u, ref)
    print(f"[c1 fp64] rel-L2 vs direct = {err:.3e}", flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("dtype,tol,bound", [(torch.float64, 1e-6, 1e-6), (torch.float32, 1e-4, 1e-4)])
def test_mixed3d_meets_tolerance(dtype, tol, bound):
    x = mixed_points(40000, 3, 15, 8, 0.01)
    lam = normal_weights(40000, 16)
    p = plan(dev(x, dtype), kernel="gaussian", shape=0.03, tol=tol, n_max=64)
    u = p.matvec(dev(lam, dtype)).double().cpu().numpy()
    xs = x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x
    ls = lam.astype(np.float32).astype(np.float64) if dtype == torch.float32 else lam
    ref = direct.direct_sum(xs, ls, "gaussian", 0.03)
    err = direct.rel_l2(u, ref)
    print(f"[mixed3d {dtype}] rel-L2 vs direct = {err:.3e} info={p.info()['nodes']}", flush=True)
    assert err <= bound


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_device_direct_sum(dtype):
    x = uniform_points(3000, 3, 17)
    lam = normal_weights(3000, 18)
    p = plan(dev(x, dtype), kernel="gaussian", shape=0.1, tol=1e-6, n_max=64)
    u = p.direct(dev(lam, dtype)).double().cpu().numpy()
    xs = x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x
    ls = lam.astype(np.float32).astype(np.float64) if dtype == torch.float32 else lam
    ref = direct.direct_sum(xs, ls, "gaussian", 0.1)
    assert direct.rel_l2(u, ref) < (1e-13 if dtype == torch.float64 else 2e-6)


def test_single_point_and_single_leaf():
    x = np.array([[0.25, 0.5]])
    p = plan(dev(x), kernel="gaussian", shape=0.05, tol=1e-6)
    u = p.matvec(dev(np.array([3.0]))).cpu().numpy()
    assert abs(u[0] - 3.0) < 1e-15
    x = uniform_points(100, 3, 19)
    lam = normal_weights(100, 20)
    p = plan(dev(x), kernel="gaussian", shape=0.1, tol=1e-6, n_max=128)
    u = p.matvec(dev(lam)).cpu().numpy()
    ref = direct.direct_sum(x, lam, "gaussian", 0.1)
    assert np.max(np.abs(u - ref)) < 1e-13 * np.max(np.abs(ref))


def test_bad_arguments_raise():
    from paper_1606_07652_amd import FmmPlan, RbfError
    x = dev(uniform_points(10, 2, 1))
    with pytest.raises(RbfError):
        FmmPlan(x, kernel="gaussian", shape=-1.0, tol=1e-6)
    with pytest.raises(RbfError):
        FmmPlan(x, kernel="gaussian", shape=0.1, tol=2.0)
    with pytest.raises(RbfError):
        FmmPlan(dev(uniform_points(10, 4, 1)), kernel="gaussian", shape=0.1, tol=1e-6)
    with pytest.raises(RbfError):
        FmmPlan(x, kernel="gaussian", shape=0.1, tol=1e-6, nodes=7)
    with pytest.raises(RbfError):
        FmmPlan(x, kernel="gaussian", shape=0.1, tol=1e-6, coarse_level=1, coarse_radius=0)


def test_full_size_mixed_sampled_targets():
    """2^20 mixed float32 points, Gaussian s=0.03: the benchmark's launch configuration,
    checked on 512 seeded targets against the FP64 direct sum over all sources."""
    w = c2("gaussian")
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(w.points.shape[0], 512, replace=False))
    xs = w.points.astype(np.float64)
    ls = w.lam.astype(np.float64)
    ref = direct.direct_sum(xs, ls, "gaussian", w.shape, targets=xs[idx])
    for dtype, tol in ((torch.float64, 1e-6), (torch.float32, 1e-4)):
        p = plan(dev(w.points, dtype), kernel="gaussian", shape=w.shape, tol=tol, n_max=256)   # bench.py's
        u = p.matvec(dev(w.lam, dtype)).double().cpu().numpy()
        err = direct.rel_l2(u[idx], ref)
        print(f"[c2 {dtype}] sampled rel-L2 = {err:.3e} info={p.info()}", flush=True)
        assert err <= tol
        p.close()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,bound", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
def test_multiquadric_plan_is_the_exact_sum(dtype, bound):
    """Multiquadric plans with opts.exact hold one leaf: the product is the exact sum (no far
    field; the banded far field is tested in test_gpu_banded.py)."""
    from paper_1606_07652_amd import FmmPlan
    from workloads import mixed_points
    x = mixed_points(3000, 3, 71)
    lam = normal_weights(3000, 72)
    X = torch.as_tensor(x, dtype=dtype, device="cuda")
    L = torch.as_tensor(lam, dtype=dtype, device="cuda")
    p = FmmPlan(X, kernel="multiquadric", shape=0.02, tol=1e-6, n_max=64, exact=True)
    inf = p.info()
    assert inf["nleaves"] == 1 and inf["far_field"] == 0
    u = p.matvec(L).double().cpu().numpy()
    xo = X.double().cpu().numpy()
    ref = direct.direct_sum(xo, L.double().cpu().numpy(), "multiquadric", 0.02)
    assert direct.rel_l2(u, ref) <= bound
    # the solve runs on it and reports the true residual of the product (checked in FP64,
    # where the returned iterate is the one the residual was computed for)
    ft = torch.as_tensor(np.sin(2 * np.pi * xo[:, 0]) * np.cos(2 * np.pi * xo[:, 1]), dtype=dtype, device="cuda")
    lam2, info = p.solve(ft, rtol=1e-6, restart=30, max_iters=60)
    assert np.isfinite(info["true_res"]) and info["iters"] > 0
    if dtype == torch.float64:
        fh = ft.cpu().numpy()
        r = fh - p.matvec(lam2).cpu().numpy()
        assert abs(np.linalg.norm(r) / np.linalg.norm(fh) - info["true_res"]) <= 1e-6 * info["true_res"] + 1e-12


@pytest.mark.parametrize("d,n,s,tol", [(2, 6000, 0.01, 1e-4), (5, 4000, 0.3, 1e-4)])
def test_fp32_matrix_core_path_meets_tolerance(d, n, s, tol):
    """FP32 aggregation/disaggregation on the matrix cores in 2-D (up to two 16-wide node
    tiles) and 5-D, against the FP64 direct sum of the same (float-rounded) inputs."""
    from paper_1606_07652_amd import FmmPlan
    x = uniform_points(n, d, 80 + d).astype(np.float32)
    lam = normal_weights(n, 90 + d).astype(np.float32)
    p = FmmPlan(torch.as_tensor(x, device="cuda"), kernel="gaussian", shape=s, tol=tol, n_max=64)
    inf = p.info()
    print(f"[fp32 d={d}] nodes={inf['nodes']} leaves={inf['nleaves']} far={inf['far_field']}", flush=True)
    assert inf["far_field"] == 1
    u = p.matvec(torch.as_tensor(lam, device="cuda")).double().cpu().numpy()
    ref = direct.direct_sum(x.astype(np.float64), lam.astype(np.float64), "gaussian", s)
    assert direct.rel_l2(u, ref) <= tol


def test_fp64_many_nodes_uses_the_small_target_tiles():
    """56 nodes per dimension in 3-D FP64: the disaggregation's phase tables for 32 targets
    would exceed 64 KiB of LDS, so it runs 16 targets per workgroup."""
    from paper_1606_07652_amd import FmmPlan
    x = uniform_points(5000, 3, 95)
    lam = normal_weights(5000, 96)
    p = FmmPlan(dev(x), kernel="gaussian", shape=0.03, tol=1e-6, n_max=64, nodes=56)
    inf = p.info()
    assert inf["nodes"] == 56 and inf["far_field"] == 1
    u = p.matvec(dev(lam)).cpu().numpy()
    assert direct.rel_l2(u, direct.direct_sum(x, lam, "gaussian", 0.03)) <= 1e-6


def test_fp64_near_field_exponential_over_its_range():
    """One unit source and targets at distances whose exponent r^2/(2 s^2) runs from 0 to about
    700, in one leaf of a plan for separate targets (near field only): every output is
    exp(-r^2/(2 s^2)) from the near-field kernel's exponential, checked element by element
    against the oracle's libm exp; the same for the device direct sum.  The bound allows the
    roundings of r^2 on both sides (about four each, fused on the device and not in the oracle:
    each moves the value by ~1.1e-16 times the exponent) on top of a few units in the last
    place."""
    from paper_1606_07652_amd import EvalPlan
    s = 0.03
    m = 4095
    rng = np.random.default_rng(200)
    t = np.sort(rng.uniform(0.0, 700.0, m))
    r = s * np.sqrt(2.0 * t)
    dirs = rng.normal(size=(m, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x0 = np.array([[0.5, 0.5, 0.5]])
    y = 0.5 + dirs * r[:, None]
    p = EvalPlan(dev(x0), dev(y), kernel="gaussian", shape=s, tol=1e-6, n_max=10 ** 6, coarse_level=0)
    inf = p.info()
    assert inf["nleaves"] == 1 and inf["far_field"] == 0
    ref = direct.direct_sum(x0, np.array([1.0]), "gaussian", s, targets=y)
    expo = ((y - x0) ** 2).sum(1) / (2 * s * s)
    ok = ref > 1e-300
    bound = 8e-16 * (1.0 + expo[ok])
    for name, u in (("near field", p.eval(dev(np.array([1.0])))), ("direct", p.direct(dev(np.array([1.0]))))):
        u = u.cpu().numpy()
        rel = np.abs(u[ok] - ref[ok]) / ref[ok]
        print(f"[exp range, {name}] max rel err {rel.max():.3e}, worst ratio to bound {(rel / bound).max():.3f}",
              flush=True)
        assert np.all(rel <= bound)
        assert np.all(u[~ok] <= 1e-290)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-6), (torch.float32, 1e-4)])
@pytest.mark.parametrize("d,n,s,lev", [(3, 30000, 0.01, 5), (2, 20000, 0.004, 6)])
def test_coarse_translation_on_large_grids(d, n, s, lev, dtype, tol):
    """Coarse grids of more than 16 cells a side (32 and 64): the box sums along each axis run
    as a running window along the line; the product meets the tolerance against the direct
    sum and repeats bit for bit."""
    from paper_1606_07652_amd import FmmPlan
    x = uniform_points(n, d, 90 + d)
    lam = normal_weights(n, 91 + d)
    X = torch.as_tensor(x, dtype=dtype, device="cuda")
    L = torch.as_tensor(lam, dtype=dtype, device="cuda")
    p = FmmPlan(X, kernel="gaussian", shape=s, tol=tol, coarse_level=lev)
    inf = p.info()
    print(f"[large grid] d={d} level={inf['coarse_level']} r={inf['coarse_radius']} nodes={inf['nodes']} "
          f"leaves={inf['nleaves']}", flush=True)
    assert inf["coarse_level"] == lev and inf["far_field"] == 1 and inf["coarse_radius"] >= 1
    u = p.matvec(L).double().cpu().numpy()
    ref = direct.direct_sum(X.double().cpu().numpy(), L.double().cpu().numpy(), "gaussian", s)
    err = direct.rel_l2(u, ref)
    print(f"  rel-L2 vs direct sum = {err:.3e}", flush=True)
    assert err <= tol
    assert np.array_equal(u, p.matvec(L).double().cpu().numpy())
    p.close()
