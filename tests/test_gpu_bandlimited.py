"""GPU parity of the band-limited Gaussian as a basis (section 3, eq. 16 with the box cut-off of
eq. 28): Phi_sigma(x) = prod_k phi_sigma(x_k), through the C ABI, against the oracle's direct sum
with the closed form of phi_sigma (scipy's Faddeeva function, pinned in test_oracle_bandlimit.py).

The plan tabulates phi_sigma per axis with a measured error of at most tol phi_sigma(0) / (4 d),
so every pair's value is within tol / 4 of Phi_sigma and the sums within
(tol / 4 + n 2^-53) sum |lam| in FP64 (the second term bounds the rounding of the sum).  FP32
plans take float coordinates (the oracle takes the same rounded inputs) but evaluate the
differences and the tables in float: a difference rounded by 2^-24 moves phi_sigma by up to
sigma 2^-24 (about 1e-5 at sigma = 200), which the rel-L2 bound of 1e-4 covers.
"""
import math

import numpy as np
import pytest

from oracle import bandlimit
from workloads import mixed_points, normal_weights, uniform_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(x, s, sigma, dtype, tol):
    from paper_1606_07652_amd import FmmPlan
    print(f"[plan] gaussian_bandlimited s={s} sigma={sigma} n={x.shape[0]} d={x.shape[1]} {dtype} tol={tol}",
          flush=True)
    return FmmPlan(dev(x, dtype), kernel="gaussian_bandlimited", shape=s, tol=tol, band=sigma)


CASES = [(2, 2500, 0.03, 1.5, "mixed"), (3, 1800, 0.05, 3.0, "uniform"), (3, 2001, 0.03, 6.0, "mixed"),
         (2, 777, 0.1, 0.7, "uniform")]


def points(kind, n, d, seed):
    return mixed_points(n, d, seed) if kind == "mixed" else uniform_points(n, d, seed)


# s = 0.003 with s sigma = 1.2 (sigma = 400) needs about 1000 pieces: 64 KB in FP64, past the
# direct kernel's LDS staging limit, so the pieces are read from global memory; and one 5-D set
@pytest.mark.parametrize("d,n,s,ssig,kind", CASES + [(3, 600, 0.003, 1.2, "uniform"), (5, 700, 0.2, 2.0, "uniform")])
def test_product_fp64_matches_oracle(d, n, s, ssig, kind):
    tol = 1e-10
    x = points(kind, n, d, 700 + n)
    lam = normal_weights(n, 701)
    p = make(x, s, ssig / s, torch.float64, tol)
    inf = p.info()
    assert inf["nleaves"] == 1 and inf["far_field"] == 0
    u = p.matvec(dev(lam)).cpu().numpy()
    ref = bandlimit.direct_sum_phi_sigma(x, lam, s, ssig / s)
    err = np.abs(u - ref).max()
    bound = (tol / 4 + n * 2.0 ** -53) * np.abs(lam).sum()
    print(f"    max err {err:.3e} bound {bound:.3e} rel-L2 {rel_l2(u, ref):.3e}", flush=True)
    assert err <= bound


@pytest.mark.parametrize("d,n,s,ssig,kind", CASES[:3])
def test_product_fp32_matches_oracle(d, n, s, ssig, kind):
    x = points(kind, n, d, 710 + n).astype(np.float32).astype(np.float64)
    lam = normal_weights(n, 711).astype(np.float32).astype(np.float64)
    p = make(x, s, ssig / s, torch.float32, 1e-5)
    u = p.matvec(dev(lam, torch.float32)).double().cpu().numpy()
    ref = bandlimit.direct_sum_phi_sigma(x, lam, s, ssig / s)
    e = rel_l2(u, ref)
    print(f"    rel-L2 {e:.3e}", flush=True)
    assert e <= 1e-4


def test_direct_and_product_are_the_same_kernel():
    """Both entry points run the tiled direct kernel: equal bits."""
    x = mixed_points(3001, 3, 720)
    lam = normal_weights(3001, 721)
    p = make(x, 0.04, 100.0, torch.float64, 1e-9)
    L = dev(lam)
    assert torch.equal(p.matvec(L), p.direct(L))


@pytest.mark.parametrize("dtype,bound", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
def test_separate_targets(dtype, bound):
    """Evaluation at points that are not centres (targets partly outside the sources' box, a few
    on sources) runs the near-field kernel over the joint point set."""
    from paper_1606_07652_amd import EvalPlan
    s, sigma = 0.04, 90.0
    x = uniform_points(2000, 3, 730)
    lam = normal_weights(2000, 731)
    y = uniform_points(1300, 3, 732) * 1.4 - 0.2
    y[:100] = x[:100]
    if dtype == torch.float32:
        x, y, lam = (a.astype(np.float32).astype(np.float64) for a in (x, y, lam))
    print(f"[eval plan] gaussian_bandlimited {dtype}", flush=True)
    p = EvalPlan(dev(x, dtype), dev(y, dtype), kernel="gaussian_bandlimited", shape=s, tol=1e-10, band=sigma)
    assert p.info()["far_field"] == 0
    L = dev(lam, dtype)
    ref = bandlimit.direct_sum_phi_sigma(x, lam, s, sigma, targets=y)
    u = p.eval(L).double().cpu().numpy()
    ud = p.direct(L).double().cpu().numpy()
    print(f"    rel-L2 eval {rel_l2(u, ref):.3e} direct {rel_l2(ud, ref):.3e}", flush=True)
    assert rel_l2(u, ref) <= bound
    assert rel_l2(ud, ref) <= bound


@pytest.mark.parametrize("s,ssig", [(0.03, 5.0), (0.05, 3.0)])
def test_interpolation_solve(s, ssig):
    """GMRES on A lambda = f with A_ij = Phi_sigma(x_i - x_j), positive definite (section 3.1):
    the oracle's product of the returned weights reproduces f.  The oracle's matrices on these
    points have condition numbers 239 and 1170."""
    x = uniform_points(1000, 3, 7)
    f = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]) + x[:, 2]
    p = make(x, s, ssig / s, torch.float64, 1e-12)
    lam, info = p.solve(dev(f), rtol=1e-10, restart=50, max_iters=1000)
    lam = lam.cpu().numpy()
    r = f - bandlimit.direct_sum_phi_sigma(x, lam, s, ssig / s)
    res = np.linalg.norm(r) / np.linalg.norm(f)
    print(f"    iters={info['iters']} true_res={info['true_res']:.2e} oracle residual {res:.2e}", flush=True)
    assert info["converged"]
    assert res <= 1e-8


def test_edge_cases():
    """One point (u = lam phi_sigma(0)^d, phi_sigma(0) = erf(s sigma / sqrt 2)); coincident
    points; a size one past a whole number of 256-source tiles."""
    s, sigma = 0.05, 60.0
    x1 = np.array([[0.3, 0.7, 0.1]])
    p = make(x1, s, sigma, torch.float64, 1e-10)
    u = p.matvec(dev(np.array([2.5]))).cpu().numpy()
    assert abs(u[0] - 2.5 * math.erf(s * sigma / math.sqrt(2)) ** 3) <= 1e-12
    x = uniform_points(257, 2, 740)
    x[5] = x[6] = x[100]
    lam = normal_weights(257, 741)
    p = make(x, s, sigma, torch.float64, 1e-10)
    u = p.matvec(dev(lam)).cpu().numpy()
    ref = bandlimit.direct_sum_phi_sigma(x, lam, s, sigma)
    assert np.abs(u - ref).max() <= (1e-10 / 4 + 257 * 2.0 ** -53) * np.abs(lam).sum()


def test_batch_matches_oracle():
    """A batch of problems with their own widths (one bandwidth) runs each exact sum through the
    near-field kernel, the table read from global memory; every problem against the oracle."""
    from paper_1606_07652_amd import BatchPlan
    sizes, shapes, sigma = [900, 257, 1400, 1], [0.03, 0.05, 0.08, 0.04], 70.0
    xs = [uniform_points(m, 3, 760 + k) for k, m in enumerate(sizes)]
    lams = [normal_weights(m, 770 + k) for k, m in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)])
    print("[batch] gaussian_bandlimited", flush=True)
    b = BatchPlan(dev(np.concatenate(xs)), off, shapes, kernel="gaussian_bandlimited", tol=1e-10, band=sigma,
                  autotune=True)
    u = b.matvec(dev(np.concatenate(lams))).cpu().numpy()
    for k, m in enumerate(sizes):
        ref = bandlimit.direct_sum_phi_sigma(xs[k], lams[k], shapes[k], sigma)
        err = np.abs(u[off[k]:off[k + 1]] - ref).max()
        assert err <= (1e-10 / 4 + m * 2.0 ** -53) * np.abs(lams[k]).sum(), (k, err)


def test_errors():
    from paper_1606_07652_amd import FmmPlan, autotune, pc
    from paper_1606_07652_amd._lib import RBF_EINVAL, RBF_EUNSUPPORTED, RbfError
    x = uniform_points(600, 3, 750)
    X = dev(x)
    with pytest.raises(RbfError) as e:
        FmmPlan(X, kernel="gaussian_bandlimited", shape=0.05, tol=1e-8)      # no bandwidth
    assert e.value.code == RBF_EINVAL
    with pytest.raises(RbfError) as e:   # sigma times the box side far beyond the table's cap
        FmmPlan(X, kernel="gaussian_bandlimited", shape=1e-4, tol=1e-8, band=1e5)
    assert e.value.code == RBF_EUNSUPPORTED
    with pytest.raises(RbfError) as e:
        autotune(X, kernel="gaussian_bandlimited", shape=0.05, tol=1e-8, band=60.0)
    assert e.value.code == RBF_EUNSUPPORTED
    p = make(x, 0.05, 60.0, torch.float64, 1e-8)
    with pytest.raises(RbfError) as e:
        pc.block_jacobi(p)
    assert e.value.code == RBF_EUNSUPPORTED
    with pytest.raises(RbfError) as e:
        p.solve(dev(np.ones(600)), precond="block_jacobi")
    assert e.value.code == RBF_EUNSUPPORTED
