"""GPU parity of the inverse multiquadric and of Wendland's compactly supported function (the
kernels of the paper's numerical examples, section 5) against the oracle's direct sum of eq. 1,
through the C ABI.

* inverse multiquadric: single-leaf plans with opts.exact, the exact sum by the tiled direct
  kernel (its banded far field is tested in test_gpu_banded.py);
* Wendland: a uniform tree at the deepest level whose cells are at least the support radius
  wide, the adjacent cells as near field and no far field, so the product is exact; deep and
  single-leaf cases, 2-D, 3-D and 5-D, ragged sizes, blobs that crowd single cells;
* evaluation at separate targets; a batch of Wendland problems; the solve on a Wendland
  system; the full-size 2^20 mixed point set on sampled targets.

Bounds: FP64 rel-L2 1e-13 (every term is exact up to a few roundings and the sums only differ
in order); FP32 inputs are rounded to float first and the oracle takes the rounded inputs, with
rel-L2 1e-5 (about 2^-24 per term times the growth of sums of a few thousand terms).
"""
import math

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


def expected_level(ext, e, d):
    """The deepest level l <= 18 / d whose cells (ext / 2^l wide) hold the support radius 1/e."""
    l = 0
    while l + 1 <= 18 // d and ext / 2.0 ** (l + 1) >= 1.0 / e:
        l += 1
    return l


def plan(x, kernel, shape, dtype, **kw):
    """Plans of the multiquadric kernels take the exact sum here (their banded far field has
    its own tests in test_gpu_banded.py)."""
    from paper_1606_07652_amd import FmmPlan
    if kernel in ("multiquadric", "inverse_multiquadric"):
        kw.setdefault("exact", True)
    print(f"[plan] {kernel} shape={shape} n={x.shape[0]} d={x.shape[1]} {dtype}", flush=True)
    return FmmPlan(dev(x, dtype), kernel=kernel, shape=shape, tol=1e-6, **kw)


@pytest.mark.parametrize("dtype,bound", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
@pytest.mark.parametrize("d,n", [(2, 2500), (3, 3001)])
def test_inverse_multiquadric_is_the_exact_sum(dtype, bound, d, n):
    x = mixed_points(n, d, 300 + d)
    lam = normal_weights(n, 301)
    p = plan(x, "inverse_multiquadric", 0.03, dtype, n_max=64)
    inf = p.info()
    assert inf["nleaves"] == 1 and inf["far_field"] == 0
    X = dev(x, dtype)
    L = dev(lam, dtype)
    u = p.matvec(L).double().cpu().numpy()
    ref = direct.direct_sum(X.double().cpu().numpy(), L.double().cpu().numpy(), "inverse_multiquadric", 0.03)
    assert direct.rel_l2(u, ref) <= bound


@pytest.mark.parametrize("dtype,bound", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
@pytest.mark.parametrize("d,n,e", [(2, 5000, 20.0), (3, 6001, 10.0), (3, 4000, 25.0), (5, 3000, 3.0),
                                   (3, 1500, 0.8)])
def test_wendland_near_only_tree_is_exact(dtype, bound, d, n, e):
    """Blobs and a uniform part; e = 0.8 has a support radius wider than the box (one leaf)."""
    x = mixed_points(n, d, 310 + d, blob_sd=0.02)
    lam = normal_weights(n, 311)
    p = plan(x, "wendland", e, dtype)
    inf = p.info()
    lvl = expected_level(inf["ext"], e, d)
    print(f"[wendland] level={inf['coarse_level']} expected={lvl} leaves={inf['nleaves']} "
          f"near_pairs={inf['near_pairs']}", flush=True)
    assert inf["far_field"] == 0
    assert inf["coarse_level"] == lvl
    assert (inf["nleaves"] == 1) == (lvl == 0)
    X = dev(x, dtype)
    L = dev(lam, dtype)
    u = p.matvec(L).double().cpu().numpy()
    ref = direct.direct_sum(X.double().cpu().numpy(), L.double().cpu().numpy(), "wendland", e)
    assert direct.rel_l2(u, ref) <= bound
    # the plan's own device direct sum agrees too
    ud = p.direct(L).double().cpu().numpy()
    assert direct.rel_l2(ud, ref) <= bound


def test_wendland_pairs_outside_the_support_are_skipped():
    """Near pairs counted by the plan are far fewer than all pairs, yet the product is the
    whole sum: every pair closer than the support radius lies in adjacent cells."""
    x = uniform_points(8000, 3, 320)
    lam = normal_weights(8000, 321)
    p = plan(x, "wendland", 12.0, torch.float64)
    inf = p.info()
    assert inf["coarse_level"] >= 2
    assert inf["near_pairs"] < 0.25 * 8000 ** 2
    u = p.matvec(dev(lam)).cpu().numpy()
    assert direct.rel_l2(u, direct.direct_sum(x, lam, "wendland", 12.0)) <= 1e-13


@pytest.mark.parametrize("kernel,shape", [("inverse_multiquadric", 0.05), ("wendland", 8.0)])
@pytest.mark.parametrize("dtype,bound", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
def test_separate_targets(kernel, shape, dtype, bound):
    from paper_1606_07652_amd import EvalPlan
    x = uniform_points(3000, 3, 330)
    lam = normal_weights(3000, 331)
    y = uniform_points(1700, 3, 332) * 1.4 - 0.2
    y[:200] = x[:200]
    X, Y, L = dev(x, dtype), dev(y, dtype), dev(lam, dtype)
    print(f"[eval plan] {kernel} {dtype}", flush=True)
    p = EvalPlan(X, Y, kernel=kernel, shape=shape, tol=1e-6, exact=kernel == "inverse_multiquadric")
    assert p.info()["far_field"] == 0
    u = p.eval(L).double().cpu().numpy()
    ref = direct.direct_sum(X.double().cpu().numpy(), L.double().cpu().numpy(), kernel, shape,
                            targets=Y.double().cpu().numpy())
    assert direct.rel_l2(u, ref) <= bound
    assert direct.rel_l2(p.direct(L).double().cpu().numpy(), ref) <= bound


def test_wendland_batch_matches_oracle():
    from paper_1606_07652_amd import BatchPlan
    sizes = [3000, 777, 4100, 1]
    shapes = [10.0, 4.0, 25.0, 3.0]
    xs = [mixed_points(m, 3, 340 + k) for k, m in enumerate(sizes)]
    lams = [normal_weights(m, 350 + k) for k, m in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)])
    print("[batch] wendland", flush=True)
    b = BatchPlan(dev(np.concatenate(xs)), off, shapes, kernel="wendland", tol=1e-6)
    u = b.matvec(dev(np.concatenate(lams))).cpu().numpy()
    for k in range(len(sizes)):
        ref = direct.direct_sum(xs[k], lams[k], "wendland", shapes[k])
        assert direct.rel_l2(u[off[k]:off[k + 1]], ref) <= 1e-13


def test_wendland_solve_converges():
    """Wendland matrices are positive definite in 3-D: GMRES reaches the tolerance, and the
    oracle's product of the returned weights reproduces the right-hand side.  At e = 16 the
    matrix on these points has condition number 284 (the oracle's eigenvalues: 0.0107 to 3.03)."""
    x = uniform_points(4000, 3, 360)
    f = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]) + x[:, 2]
    p = plan(x, "wendland", 16.0, torch.float64)
    lam, info = p.solve(dev(f), rtol=1e-9, restart=50, max_iters=400)
    print(f"[wendland solve] iters={info['iters']} true_res={info['true_res']:.2e}", flush=True)
    assert info["converged"]
    r = f - direct.direct_sum(x, lam.cpu().numpy(), "wendland", 16.0)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 2e-9


def test_wendland_full_size_sampled():
    """The 2^20 mixed point set of the 3-D configuration, e = 25 (support radius 0.04), FP64:
    2048 seeded targets against all sources."""
    w = c2()
    x, lam = w.points, w.lam
    p = plan(x, "wendland", 25.0, torch.float64)
    inf = p.info()
    print(f"[wendland full] level={inf['coarse_level']} leaves={inf['nleaves']} "
          f"near_pairs={inf['near_pairs']:.3e}", flush=True)
    assert inf["far_field"] == 0
    u = p.matvec(dev(lam)).cpu().numpy()
    idx = np.random.default_rng(370).choice(x.shape[0], 2048, replace=False)
    ref = direct.direct_sum(x, lam, "wendland", 25.0, targets=x[idx])
    assert direct.rel_l2(u[idx], ref) <= 1e-13
    assert math.isfinite(float(np.abs(u).max()))


@pytest.mark.parametrize("kernel,shape,phi0", [("inverse_multiquadric", 0.05, 20.0), ("wendland", 8.0, 1.0)])
def test_block_jacobi_other_kernels(kernel, shape, phi0):
    """Block-Jacobi on the positive definite kernels: the default regularisation 1e-2 Phi(0)
    and an explicit one, against the oracle's block inverses (cdist-free, its own kernel)."""
    from oracle import precond as P
    from paper_1606_07652_amd import pc
    x = mixed_points(3000, 3, 380)
    v = normal_weights(3000, 381)
    p = plan(x, kernel, shape, torch.float64)
    z = pc.apply(p, "block_jacobi", dev(v)).cpu().numpy()
    inv, perm = P.block_inverses(x, kernel, shape, 1e-2 * phi0)
    ref = P.bj_apply(inv, perm, v)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    pc.block_jacobi(p, 1e-3 * phi0)
    z = pc.apply(p, "block_jacobi", dev(v)).cpu().numpy()
    inv, perm = P.block_inverses(x, kernel, shape, 1e-3 * phi0)
    ref = P.bj_apply(inv, perm, v)
    assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)


def test_wendland_solve_with_block_jacobi():
    x = uniform_points(4000, 3, 360)
    f = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]) + x[:, 2]
    p = plan(x, "wendland", 16.0, torch.float64)
    lam, info = p.solve(dev(f), rtol=1e-9, restart=50, max_iters=400, precond="block_jacobi")
    _, plain = p.solve(dev(f), rtol=1e-9, restart=50, max_iters=400)
    print(f"[wendland bj solve] iters={info['iters']} (plain {plain['iters']}) true_res={info['true_res']:.2e}",
          flush=True)
    assert info["converged"] and info["iters"] < plain["iters"]
    r = f - direct.direct_sum(x, lam.cpu().numpy(), "wendland", 16.0)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 2e-9


def test_preconditioner_kernel_errors():
    """The learned map's features take the Gaussian and the multiquadric kernels only;
    block-Jacobi takes the multiquadric (pivoted factorisation)."""
    from paper_1606_07652_amd import pc
    from paper_1606_07652_amd._lib import RBF_EUNSUPPORTED, RbfError
    x = uniform_points(500, 3, 390)
    pm = plan(x, "multiquadric", 0.05, torch.float64)
    pc.block_jacobi(pm)
    pc.learned_features(pm)
    pw = plan(x, "wendland", 4.0, torch.float64)
    with pytest.raises(RbfError) as e:
        pc.learned_features(pw)
    assert e.value.code == RBF_EUNSUPPORTED


@pytest.mark.parametrize("kind,c", [("uniform", 0.05), ("mixed", 0.02)])
def test_block_jacobi_multiquadric_pivoted(kind, c):
    """Multiquadric blocks are indefinite: the pivoted factorisation matches the oracle's
    block solves to the blocks' condition number times the FP64 unit roundoff."""
    from oracle import precond as P
    from paper_1606_07652_amd import pc
    x = (uniform_points if kind == "uniform" else mixed_points)(2500, 3, 385)
    v = normal_weights(2500, 386)
    p = plan(x, "multiquadric", c, torch.float64)
    reg = 1e-2 * c
    pc.block_jacobi(p, reg)
    z = pc.apply(p, "block_jacobi", dev(v)).cpu().numpy()
    inv, perm = P.block_inverses(x, "multiquadric", c, reg)
    ref = P.bj_apply(inv, perm, v)
    cond = max(np.linalg.cond(b) for b in inv)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"[mq bj {kind}] max block cond {cond:.2e}, rel diff {err:.2e}", flush=True)
    assert err <= 1e-13 * cond


@pytest.mark.parametrize("kernel", ["thin_plate", "r5"])
@pytest.mark.parametrize("dtype,bound", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
@pytest.mark.parametrize("d,n", [(2, 2300), (3, 3001)])
def test_piecewise_smooth_kernels_are_the_exact_sum(kernel, dtype, bound, d, n):
    """The thin-plate spline and r^5 (no shape): single-leaf plans, the exact sum, with
    duplicated points (r = 0 pairs beside the diagonal)."""
    x = uniform_points(n, d, 400 + d)
    x[n // 2:n // 2 + 50] = x[:50]
    lam = normal_weights(n, 401)
    p = plan(x, kernel, 1.0, dtype, n_max=64)
    inf = p.info()
    assert inf["nleaves"] == 1 and inf["far_field"] == 0
    X, L = dev(x, dtype), dev(lam, dtype)
    u = p.matvec(L).double().cpu().numpy()
    ref = direct.direct_sum(X.double().cpu().numpy(), L.double().cpu().numpy(), kernel, 1.0)
    assert np.all(np.isfinite(u))
    assert direct.rel_l2(u, ref) <= bound


@pytest.mark.parametrize("kernel", ["thin_plate", "r5"])
def test_piecewise_smooth_kernels_at_separate_targets(kernel):
    from paper_1606_07652_amd import EvalPlan
    x = uniform_points(2000, 3, 410)
    lam = normal_weights(2000, 411)
    y = uniform_points(900, 3, 412) * 1.4 - 0.2
    y[:100] = x[:100]
    p = EvalPlan(dev(x), dev(y), kernel=kernel, shape=1.0, tol=1e-6)
    u = p.eval(dev(lam)).cpu().numpy()
    assert direct.rel_l2(u, direct.direct_sum(x, lam, kernel, 1.0, targets=y)) <= 1e-13


def test_piecewise_smooth_kernels_reject_solve_and_block_jacobi():
    """Conditionally positive definite kernels: interpolation needs polynomial augmentation
    (not built), and their blocks are not positive definite."""
    from paper_1606_07652_amd import pc
    from paper_1606_07652_amd._lib import RBF_EUNSUPPORTED, RbfError
    x = uniform_points(400, 2, 420)
    f = np.sin(3 * x[:, 0])
    for kernel in ("thin_plate", "r5"):
        p = plan(x, kernel, 1.0, torch.float64)
        with pytest.raises(RbfError) as e:
            p.solve(dev(f), rtol=1e-6)
        assert e.value.code == RBF_EUNSUPPORTED
        with pytest.raises(RbfError) as e:
            pc.block_jacobi(p)
        assert e.value.code == RBF_EUNSUPPORTED


AUGMENTED = [("thin_plate", 2, 300, 1.0), ("r5", 3, 250, 1.0), ("multiquadric", 3, 300, 0.1), ("thin_plate", 3, 400, 1.0)]


@pytest.mark.parametrize("kernel,d,n,shape", AUGMENTED)
def test_augmented_solve_matches_oracle(kernel, d, n, shape):
    """[A P; P' 0][lambda; c] = [f; 0] by full GMRES (restart = n + q): the true residual of the
    returned vector under the oracle's augmented matrix meets the tolerance, and the vector is
    the oracle's dense solution to the condition number times the tolerance (cond <= 6e7 on
    these sets, so 1e-4 with margin)."""
    from oracle import poly
    x = uniform_points(n, d, 500 + d)
    f = np.sin(3 * x[:, 0]) + np.cos(2 * x[:, 1])
    p = plan(x, kernel, shape, torch.float64)
    q = p.poly_terms()
    assert q == poly.nterms(d, poly.DEGREE[kernel])
    lam, c, info = p.solve_poly(dev(f), rtol=1e-10, restart=n + q, max_iters=2 * (n + q))
    print(f"[augmented {kernel} d={d}] q={q} iters={info['iters']} true_res={info['true_res']:.2e}", flush=True)
    assert info["converged"]
    sol = np.concatenate([lam.cpu().numpy(), c.cpu().numpy()])
    M = poly.augmented_matrix(x, kernel, shape)
    rhs = np.concatenate([f, np.zeros(q)])
    assert np.linalg.norm(M @ sol - rhs) <= 2e-10 * np.linalg.norm(f)
    lo, co = poly.augmented_solve(x, kernel, shape, f)
    ref = np.concatenate([lo, co])
    assert np.linalg.norm(sol - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("kernel,d", [("thin_plate", 2), ("r5", 3)])
def test_augmented_solve_reproduces_polynomials(kernel, d):
    """A right-hand side in the polynomial space comes back as lambda = 0 and its coefficients
    (the oracle's monomials of the root cube's normalised coordinates), to what the stopping
    rule allows: a residual of rtol ||f|| moves the solution by at most rtol ||f|| / s_min, s_min
    the smallest singular value of the oracle's augmented matrix (twice that as the bound)."""
    from oracle import poly
    x = uniform_points(200, d, 520 + d) * 2.0 - 0.5
    P = poly.basis(x, poly.DEGREE[kernel])
    ct = np.random.default_rng(521).standard_normal(P.shape[1])
    f = P @ ct
    rtol = 1e-12
    smin = np.linalg.svd(poly.augmented_matrix(x, kernel, 1.0), compute_uv=False)[-1]
    bound = 2.0 * rtol * np.linalg.norm(f) / smin
    p = plan(x, kernel, 1.0, torch.float64)
    q = p.poly_terms()
    lam, c, info = p.solve_poly(dev(f), rtol=rtol, restart=200 + q, max_iters=2 * (200 + q))
    assert info["converged"]
    assert np.max(np.abs(c.cpu().numpy() - ct)) <= bound
    assert np.max(np.abs(lam.cpu().numpy())) <= bound


def test_augmented_solve_fp32_and_errors():
    """FP32 plans solve the augmented system in FP64 Krylov vectors (products in FP32); the
    positive definite kernels have q = 0; a preconditioner is refused for q > 0."""
    from oracle import poly
    from paper_1606_07652_amd._lib import RBF_EUNSUPPORTED, RbfError
    x = uniform_points(300, 2, 530)
    f = np.sin(3 * x[:, 0]) + x[:, 1]
    p = plan(x, "thin_plate", 1.0, torch.float32)
    # FP32 products carry ~1e-6 relative error times ||A|| ||lambda|| / ||f|| (about 30 here)
    lam, c, info = p.solve_poly(dev(f, torch.float32), rtol=1e-4, restart=303, max_iters=606)
    assert info["converged"]
    M = poly.augmented_matrix(x.astype(np.float32).astype(np.float64), "thin_plate", 1.0)
    sol = np.concatenate([lam.double().cpu().numpy(), c.double().cpu().numpy()])
    rhs = np.concatenate([f.astype(np.float32).astype(np.float64), np.zeros(3)])
    # the returned FP32 vector: its residual under the FP64 matrix is the solve's plus the
    # rounding of the vector to float
    assert np.linalg.norm(M @ sol - rhs) <= 1e-3 * np.linalg.norm(f)
    assert plan(x, "gaussian", 0.1, torch.float64).poly_terms() == 0
    p64 = plan(x, "thin_plate", 1.0, torch.float64)
    from paper_1606_07652_amd import _lib as L
    import ctypes
    o = L.RbfSolveOpts(30, 60, L.RBF_PC_BLOCK_JACOBI, 1, 0, 0.0)
    info_c = L.RbfSolveInfo()
    F = dev(f)
    lam0 = torch.zeros_like(F)
    cf = torch.zeros(3, dtype=torch.float64, device="cuda")
    code = L.load().rbf_interp_solve_poly(p64._h, F.data_ptr(), lam0.data_ptr(), cf.data_ptr(), 1e-6,
                                          ctypes.byref(o), ctypes.byref(info_c))
    assert code == RBF_EUNSUPPORTED
    with pytest.raises(RbfError):
        p64.solve(F, rtol=1e-6)


def test_wendland_batched_solve_matches_oracle():
    """GMRES on a batch of Wendland problems at once: every problem converges, and the
    oracle's product of its weights reproduces its right-hand side."""
    from paper_1606_07652_amd import BatchPlan
    sizes = [1500, 900, 2200]
    shapes = [12.0, 10.0, 16.0]
    xs = [uniform_points(m, 3, 540 + k) for k, m in enumerate(sizes)]
    fs = [np.sin(2 * np.pi * x[:, 0]) + x[:, 1] for x in xs]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    print("[batch solve] wendland", flush=True)
    b = BatchPlan(dev(np.concatenate(xs)), off, shapes, kernel="wendland", tol=1e-6)
    lam, infos = b.solve(dev(np.concatenate(fs)), rtol=1e-9, restart=50, max_iters=600)
    lam = lam.cpu().numpy()
    for k in range(len(sizes)):
        assert infos[k]["converged"], (k, infos[k])
        lk = lam[off[k]:off[k + 1]]
        r = fs[k] - direct.direct_sum(xs[k], lk, "wendland", shapes[k])
        assert np.linalg.norm(r) <= 2e-9 * np.linalg.norm(fs[k])


def test_augmented_solve_edge_cases():
    """Zero right-hand side (zero weights and coefficients, no iterations); a missing coefficient
    buffer and an evaluation plan are refused; the positive definite kernels need no buffer."""
    import ctypes
    from paper_1606_07652_amd import EvalPlan
    from paper_1606_07652_amd import _lib as L
    x = uniform_points(200, 2, 550)
    p = plan(x, "thin_plate", 1.0, torch.float64)
    lam, c, info = p.solve_poly(dev(np.zeros(200)), rtol=1e-8, restart=50, max_iters=100)
    assert info["converged"] and info["iters"] == 0
    assert torch.count_nonzero(lam).item() == 0 and torch.count_nonzero(c).item() == 0
    o = L.RbfSolveOpts(50, 100, L.RBF_PC_NONE, 1, 0, 0.0)
    inf = L.RbfSolveInfo()
    F = dev(np.ones(200))
    out = torch.zeros_like(F)
    code = L.load().rbf_interp_solve_poly(p._h, F.data_ptr(), out.data_ptr(), None, 1e-6, ctypes.byref(o),
                                          ctypes.byref(inf))
    assert code == L.RBF_EINVAL
    g = plan(x, "gaussian", 0.1, torch.float64)
    code = L.load().rbf_interp_solve_poly(g._h, F.data_ptr(), out.data_ptr(), None, 1e-6, ctypes.byref(o),
                                          ctypes.byref(inf))
    assert code in (L.RBF_OK, L.RBF_ENOCONV) and inf.iters > 0
    e = EvalPlan(dev(x), dev(uniform_points(50, 2, 551)), kernel="thin_plate", shape=1.0, tol=1e-6)
    code = L.load().rbf_interp_solve_poly(e._h, F.data_ptr(), out.data_ptr(), None, 1e-6, ctypes.byref(o),
                                          ctypes.byref(inf))
    assert code == L.RBF_EINVAL
    with pytest.raises(ValueError):
        p.solve_poly(dev(np.ones(200)), coeffs=torch.zeros(2, dtype=torch.float64, device="cuda"))
