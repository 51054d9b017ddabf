"""Batched products, the autotuner and near-only plans (GPU, through the C ABI)."""
import numpy as np
import pytest

from oracle import direct, splitref
from workloads import normal_weights, uniform_points

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def small_batch(nprob=12, seed=5):
    rng = np.random.default_rng(seed)
    ns = rng.integers(300, 6000, nprob)
    ss = np.exp(rng.uniform(np.log(0.02), np.log(0.1), nprob))
    pts = [uniform_points(int(n), 3, 1000 + q) for q, n in enumerate(ns)]
    lams = [normal_weights(int(n), 2000 + q) for q, n in enumerate(ns)]
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    return pts, lams, ss, off


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-6), (torch.float32, 1e-4)])
def test_batch_equals_single_plans(dtype, tol):
    """The batched launch runs the same kernels on the same descriptors: results are
    identical to one plan per problem, and each meets the tolerance of the direct sum."""
    from paper_1606_07652_amd import BatchPlan, FmmPlan
    pts, lams, ss, off = small_batch()
    X = dev(np.concatenate(pts), dtype)
    lam = dev(np.concatenate(lams), dtype)
    print(f"[batch] {len(ss)} problems, n={off[-1]}, {dtype}", flush=True)
    b = BatchPlan(X, off, ss, kernel="gaussian", tol=tol, n_max=64)
    u = b.matvec(lam).double().cpu().numpy()
    for q in range(len(ss)):
        sl = slice(off[q], off[q + 1])
        p = FmmPlan(X[sl].contiguous(), kernel="gaussian", shape=float(ss[q]), tol=tol, n_max=64)
        uq = p.matvec(lam[sl].contiguous()).double().cpu().numpy()
        assert np.array_equal(u[sl], uq), q
        xs = X[sl].double().cpu().numpy()
        ls = lam[sl].double().cpu().numpy()
        ref = direct.direct_sum(xs, ls, "gaussian", float(ss[q]))
        assert direct.rel_l2(u[sl], ref) <= tol, q
        p.close()
    b.close()


def test_graph_replays_match_eager():
    """Graph replays (same vectors, new contents, eager work in between) equal direct launches."""
    from paper_1606_07652_amd import BatchPlan
    pts, lams, ss, off = small_batch(8, 7)
    X = dev(np.concatenate(pts), torch.float32)
    b = BatchPlan(X, off, ss, kernel="gaussian", tol=1e-4, n_max=64)
    lam = torch.empty(int(off[-1]), dtype=torch.float32, device="cuda")
    out_g = torch.empty_like(lam)
    out_e = torch.empty_like(lam)
    for it in range(4):
        torch.manual_seed(it)
        lam.copy_(torch.randn(int(off[-1]), device="cuda"))
        b.set_graph(True)
        b.matvec(lam, out_g)
        junk = (lam * 2.0).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
        b.set_graph(False)
        b.matvec(lam, out_e)
        torch.cuda.synchronize()
        assert torch.equal(out_g, out_e), it
        assert torch.isfinite(junk)
    # new output pointer: the graph is captured again
    b.set_graph(True)
    out2 = b.matvec(lam)
    torch.cuda.synchronize()
    assert torch.equal(out2, out_e)
    b.close()


def test_autotuned_batch_meets_tolerance():
    from paper_1606_07652_amd import BatchPlan
    pts, lams, ss, off = small_batch(6, 11)
    ss = np.array([0.01, 0.1, 0.03, 0.015, 0.06, 0.02])
    X = dev(np.concatenate(pts), torch.float32)
    lam = dev(np.concatenate(lams), torch.float32)
    b = BatchPlan(X, off, ss, kernel="gaussian", tol=1e-4, autotune=True)
    inf = b.info()
    print(f"[autotune batch] n_max={inf['n_max']} nodes={inf['nodes']} far={inf['nfar']}", flush=True)
    u = b.matvec(lam).double().cpu().numpy()
    for q in range(len(ss)):
        sl = slice(off[q], off[q + 1])
        xs = X[sl].double().cpu().numpy()
        ls = lam[sl].double().cpu().numpy()
        ref = direct.direct_sum(xs, ls, "gaussian", float(ss[q]))
        assert direct.rel_l2(u[sl], ref) <= 1e-4, q
    b.close()


def test_near_only_plan_is_exact_split():
    """Narrow Gaussian on a uniform tree at the pruning level: every kept pair is near, so
    the product equals the oracle's split reference (which then has no far pairs)."""
    from paper_1606_07652_amd import FmmPlan
    x = uniform_points(4000, 3, 21)
    lam = normal_weights(4000, 22)
    s = 0.01
    kw = dict(n_max=1 << 30, min_level=4, max_level=4, coarse_level=4, coarse_radius=1, nodes=4)
    p = FmmPlan(dev(x, torch.float64), kernel="gaussian", shape=s, tol=1e-6, **kw)
    assert p.info()["far_field"] == 0
    u = p.matvec(dev(lam, torch.float64)).cpu().numpy()
    ref = splitref.split_reference(x, lam, "gaussian", s, n_max=1 << 30, lc=4, r=1, sigma=100.0, mn=4,
                                   max_level=4)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert direct.rel_l2(u, direct.direct_sum(x, lam, "gaussian", s)) < 1e-6


def test_autotune_single_problem():
    from paper_1606_07652_amd import FmmPlan, autotune
    x = uniform_points(20000, 3, 31)
    lam = normal_weights(20000, 32)
    X = dev(x, torch.float32)
    opts, ms = autotune(X, kernel="gaussian", shape=0.03, tol=1e-4, reps=2)
    print(f"[autotune] {opts} {ms:.3f} ms", flush=True)
    assert ms > 0
    p = FmmPlan(X, kernel="gaussian", shape=0.03, tol=1e-4, **opts)
    u = p.matvec(dev(lam, torch.float32)).double().cpu().numpy()
    ref = direct.direct_sum(x.astype(np.float32).astype(np.float64), lam.astype(np.float32).astype(np.float64),
                            "gaussian", 0.03)
    assert direct.rel_l2(u, ref) <= 1e-4


def test_single_leaf_plan_is_the_direct_sum():
    """A tree of one leaf (the autotuner's candidate when nothing can be pruned) evaluates
    every pair in the near field: it equals the device direct sum and the oracle."""
    from paper_1606_07652_amd import FmmPlan, autotune
    x = uniform_points(3000, 5, 41)
    lam = normal_weights(3000, 42)
    X = dev(x, torch.float64)
    kw = dict(n_max=1 << 30, max_level=0, min_level=0, coarse_level=0, coarse_radius=0, nodes=4)
    p = FmmPlan(X, kernel="gaussian", shape=0.2, tol=1e-6, **kw)
    inf = p.info()
    assert inf["nleaves"] == 1 and inf["far_field"] == 0 and inf["near_pairs"] == 3000 * 3000
    L = dev(lam, torch.float64)
    u = p.matvec(L).cpu().numpy()
    ud = p.direct(L).cpu().numpy()
    assert np.max(np.abs(u - ud)) <= 1e-12 * np.max(np.abs(ud))
    assert direct.rel_l2(u, direct.direct_sum(x, lam, "gaussian", 0.2)) <= 1e-13
    opts, ms = autotune(X, kernel="gaussian", shape=0.2, tol=1e-6, reps=2)
    print(f"[autotune 5-D] {opts} {ms:.3f} ms", flush=True)
    q = FmmPlan(X, kernel="gaussian", shape=0.2, tol=1e-6, **opts)
    assert direct.rel_l2(q.matvec(L).cpu().numpy(), direct.direct_sum(x, lam, "gaussian", 0.2)) <= 1e-6


@pytest.mark.parametrize("dtype,rtol", [(torch.float64, 1e-9), (torch.float32, 1e-5)])
def test_batched_solve_matches_single_solves(dtype, rtol):
    """GMRES on all problems of a batch at once equals one solve per problem: the operators
    are identical and only the blocking of the FP64 reductions differs.  One problem has a
    zero right-hand side (converged at once, zero solution)."""
    from paper_1606_07652_amd import BatchPlan, FmmPlan
    from workloads import fourier_modes_rhs, jittered_grid
    sides = [20, 28, 35, 24, 40, 30]
    pts = [jittered_grid(sd, 2, 300 + k) for k, sd in enumerate(sides)]
    ss = np.array([0.5 / sd for sd in sides])
    fs = [fourier_modes_rhs(x, 400 + k) for k, x in enumerate(pts)]
    fs[3] = np.zeros_like(fs[3])
    off = np.concatenate([[0], np.cumsum([x.shape[0] for x in pts])]).astype(np.int64)
    X = dev(np.concatenate(pts), dtype)
    F = dev(np.concatenate(fs), dtype)
    tol = 1e-8 if dtype == torch.float64 else 1e-4
    b = BatchPlan(X, off, ss, kernel="gaussian", tol=tol)
    lam, infos = b.solve(F, rtol=rtol, restart=30, max_iters=300)
    lam = lam.double().cpu().numpy()
    for q in range(len(sides)):
        sl = slice(off[q], off[q + 1])
        iq = infos[q]
        print(f"[batch solve {dtype}] problem {q}: iters={iq['iters']} res={iq['true_res']:.2e}", flush=True)
        assert iq["converged"] and iq["true_res"] <= rtol
        if q == 3:
            assert iq["iters"] == 0 and np.all(lam[sl] == 0)
            continue
        p = FmmPlan(X[sl].contiguous(), kernel="gaussian", shape=float(ss[q]), tol=tol)
        l1, i1 = p.solve(F[sl].contiguous(), rtol=rtol, restart=30, max_iters=300)
        assert i1["converged"] and abs(i1["iters"] - iq["iters"]) <= 2
        assert np.linalg.norm(lam[sl] - l1.double().cpu().numpy()) <= 1e3 * rtol * np.linalg.norm(lam[sl])
        # the batched solution's residual under the problem's own operator
        u = p.matvec(dev(lam[sl], dtype)).double().cpu().numpy()
        fq = F[sl].double().cpu().numpy()
        assert np.linalg.norm(fq - u) / np.linalg.norm(fq) <= 10 * rtol
    b.close()


def test_more_groups_than_streams():
    """Eleven problems whose shapes give eleven different padded half grids (the tolerance rule of
    oracle/params.py): more groups than the batch's eight streams, so groups share streams.  Direct
    launches and graph replays equal one plan per problem exactly."""
    from paper_1606_07652_amd import BatchPlan, FmmPlan
    shapes = [0.004, 0.284, 0.1557, 0.1062, 0.0808, 0.0649, 0.0551, 0.0419, 0.0337, 0.0286, 0.0243]
    sizes = [1500 + 150 * k for k in range(len(shapes))]
    pts = [uniform_points(m, 3, 700 + k) for k, m in enumerate(sizes)]
    lams = [normal_weights(m, 800 + k) for k, m in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = dev(np.concatenate(pts), torch.float64)
    lam = dev(np.concatenate(lams), torch.float64)
    print(f"[batch] {len(shapes)} problems, n={off[-1]}", flush=True)
    b = BatchPlan(X, off, shapes, kernel="gaussian", tol=1e-4, n_max=64)
    assert b.info()["ngroups"] >= 9
    b.set_graph(False)
    u_direct = b.matvec(lam).cpu().numpy()
    b.set_graph(True)
    u1 = b.matvec(lam).cpu().numpy()
    u2 = b.matvec(lam).cpu().numpy()
    assert np.array_equal(u1, u_direct) and np.array_equal(u2, u_direct)
    for q in range(len(shapes)):
        sl = slice(off[q], off[q + 1])
        p = FmmPlan(X[sl].contiguous(), kernel="gaussian", shape=shapes[q], tol=1e-4, n_max=64)
        uq = p.matvec(lam[sl].contiguous()).cpu().numpy()
        assert np.array_equal(u_direct[sl], uq), q
        p.close()
    b.close()


def test_batched_block_jacobi_solve():
    """Block-Jacobi flexible GMRES on all problems of a batch at once.  Three jittered grids
    (well conditioned) and two uniform random sets with s = 0.5 / sqrt(n) (condition numbers
    near 4e4, where plain GMRES(30) stalls): every problem converges to the true residual
    asked for, with the iteration count of the single-plan solve with the same preconditioner
    (+-2; only the blocking of the FP64 reductions differs); its residual under the exact
    dense matrix is at that level; the random sets need fewer iterations than without the
    preconditioner; and on the two smallest problems the oracle (restarted GMRES with the
    oracle's block inverses as the right preconditioner and exact dense products) takes the
    same iteration count +-2 and reaches the same solution."""
    from oracle import gmres as G
    from oracle import precond as P
    from paper_1606_07652_amd import BatchPlan, FmmPlan
    from workloads import fourier_modes_rhs, jittered_grid
    pts = [jittered_grid(sd, 2, 500 + k) for k, sd in enumerate((22, 30, 37))]
    pts += [uniform_points(1500, 2, 510), uniform_points(900, 2, 511)]
    ss = np.array([0.5 / 22, 0.5 / 30, 0.5 / 37, 0.5 / np.sqrt(1500), 0.5 / 30])
    fs = [fourier_modes_rhs(x, 520 + k) for k, x in enumerate(pts)]
    off = np.concatenate([[0], np.cumsum([x.shape[0] for x in pts])]).astype(np.int64)
    X = dev(np.concatenate(pts), torch.float64)
    F = dev(np.concatenate(fs), torch.float64)
    rtol = 1e-8

    def dense(q):
        x = pts[q]
        return np.exp(-((x[:, None, :] - x[None, :, :]) ** 2).sum(-1) / (2 * ss[q] ** 2))

    b = BatchPlan(X, off, ss, kernel="gaussian", tol=1e-10)
    _, inf0 = b.solve(F, rtol=rtol, restart=30, max_iters=600)
    lam, infos = b.solve(F, rtol=rtol, restart=30, max_iters=2000, precond="block_jacobi")
    lam = lam.cpu().numpy()
    for q in range(len(pts)):
        sl = slice(off[q], off[q + 1])
        iq = infos[q]
        print(f"[batch bj] problem {q} (n={off[q + 1] - off[q]}): iters {iq['iters']} "
              f"(none: {inf0[q]['iters']}, res {inf0[q]['true_res']:.1e}) res={iq['true_res']:.2e}", flush=True)
        assert iq["converged"] and iq["true_res"] <= rtol
        if q >= 3:
            assert iq["iters"] < inf0[q]["iters"]
        r = fs[q] - dense(q) @ lam[sl]
        assert np.linalg.norm(r) <= 10 * rtol * np.linalg.norm(fs[q])
        p = FmmPlan(X[sl].contiguous(), kernel="gaussian", shape=float(ss[q]), tol=1e-10)
        l1, i1 = p.solve(F[sl].contiguous(), rtol=rtol, restart=30, max_iters=2000, precond="block_jacobi")
        assert i1["converged"] and abs(i1["iters"] - iq["iters"]) <= 2
        if q < 3:
            l1 = l1.cpu().numpy()
            assert np.linalg.norm(lam[sl] - l1) <= 1e-5 * np.linalg.norm(l1)
        p.close()
    for q in np.argsort(np.diff(off), kind="stable")[:2]:
        sl = slice(off[q], off[q + 1])
        A = dense(q)
        inv, perm = P.block_inverses(pts[q], "gaussian", float(ss[q]), 1e-2)
        lr, ir = G.gmres(lambda v: A @ v, fs[q], restart=30, rtol=rtol, maxiter=2000,
                         precond=lambda v: P.bj_apply(inv, perm, v))
        print(f"[batch bj] oracle problem {q}: iters {ir['iters']} vs {infos[q]['iters']}", flush=True)
        assert ir["converged"] and abs(ir["iters"] - infos[q]["iters"]) <= 2
        assert np.linalg.norm(lam[sl] - lr) <= 1e-5 * np.linalg.norm(lr)
    b.close()
