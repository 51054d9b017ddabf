"""Pins of the preconditioner oracle (block-Jacobi, MLP, Adam, training pairs)."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import precond as P
from oracle import tree as otree
from workloads import uniform_points

torch = pytest.importorskip("torch")


def rand_params(layers, seed, scale=None):
    rng = np.random.default_rng(seed)
    out = []
    for i, o in layers:
        sc = scale if scale is not None else 1.0 / np.sqrt(i)
        out.append(rng.normal(0, sc, (o, i)).ravel())
        out.append(rng.normal(0, 0.1, o))
    return np.concatenate(out)


def test_nparams():
    assert P.nparams() == 164672


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100)])
    # exact ties between two bfloat16 neighbours (8 significant bits): both parities of the kept bit
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(2 + 2.0 ** -7), 3 * (1 + 2.0 ** -8), 0.0, -0.0])
    vals = np.concatenate([vals, ties]).astype(np.float32)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(P.round_bf16(vals), ref)
    assert P.round_bf16(np.float32(1 + 2.0 ** -8)) == 1.0            # tie to even (down)
    assert P.round_bf16(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6  # tie to even (up)


def test_forward_hand_example():
    # two layers: h = relu(W1 x + b1), g = W2 h + b2, worked by hand
    layers = [(2, 2), (2, 1)]
    params = np.array([1.0, -1.0, 2.0, 0.5, 0.5, -1.0, 3.0, -2.0, 0.25])
    X = np.array([[1.0, 2.0], [-1.0, 0.5]])
    # row 0: W1 x + b1 = (1 - 2 + 0.5, 2 + 1 - 1) = (-0.5, 2) -> (0, 2); g = -4 + 0.25
    # row 1: (-1 - 0.5 + 0.5, -2 + 0.25 - 1) = (-1, -2.75) -> (0, 0); g = 0.25
    G, _ = P.forward(params, X, layers)
    assert np.array_equal(G[:, 0], [-3.75, 0.25])


def test_all_active_relus_reduce_to_affine_product():
    layers = [(6, 9), (9, 8), (8, 5)]
    rng = np.random.default_rng(1)
    params = np.abs(rand_params(layers, 2)) + 0.01
    X = rng.uniform(0.1, 1.0, (7, 6))
    Ws = P.unpack(params, layers)
    M = Ws[2][0] @ Ws[1][0] @ Ws[0][0]
    c = Ws[2][0] @ (Ws[1][0] @ Ws[0][1] + Ws[1][1]) + Ws[2][1]
    G, _ = P.forward(params, X, layers)
    assert np.allclose(G, X @ M.T + c, rtol=1e-13, atol=0)


@pytest.mark.parametrize("layers", [[(5, 7), (7, 6), (6, 4)], P.LAYERS])
def test_grad_matches_central_differences(layers):
    rng = np.random.default_rng(3)
    params = rand_params(layers, 4)
    fin = layers[0][0]
    fout = layers[-1][1]
    X = rng.normal(0, 1, (9, fin))
    T = rng.normal(0, 1, (9, fout))
    w = rng.uniform(0.1, 2.0, 9)
    L, g = P.grad(params, X, T, w, layers)
    assert abs(L - P.loss(params, X, T, w, layers)) <= 1e-14 * abs(L)
    # coordinates: all of them for the small net, 60 spread over every tensor for the full one
    n = params.shape[0]
    coords = np.arange(n) if n < 500 else np.unique(np.concatenate([
        rng.choice(n, 50, replace=False), np.cumsum([0] + [i * o + o for i, o in layers])[:-1] + 1,
        np.cumsum([i * o + o for i, o in layers]) - 1]))
    h = 1e-6
    for k in coords:
        pp = params.copy()
        pp[k] += h
        lp = P.loss(pp, X, T, w, layers)
        pp[k] -= 2 * h
        lm = P.loss(pp, X, T, w, layers)
        fd = (lp - lm) / (2 * h)
        # 1e-5: room for the rare ReLU kink within h of a pre-activation; a missing mask, a
        # transposed operand or a wrong factor is off by far more
        assert abs(fd - g[k]) <= 1e-5 * max(abs(g[k]), 1e-3 * np.max(np.abs(g))), (k, fd, g[k])


def test_adam_first_steps_move_by_lr():
    rng = np.random.default_rng(5)
    p0 = rng.normal(0, 1, 1000)
    g = rng.normal(0, 1, 1000)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    lr = 1e-3
    p1, m, v = P.adam(p0, g, m, v, 1, lr)
    # bias-corrected moments of one step are g and g^2: the step is lr g / (|g| + eps)
    assert np.allclose(p1 - p0, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a constant gradient keeps the corrected moments at g and g^2
    p2, m, v = P.adam(p1, g, m, v, 2, lr)
    assert np.allclose(p2 - p1, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)


def test_sorted_order_is_the_tree_order():
    x = uniform_points(500, 3, 7)
    t = otree.build(x, n_max=64)
    assert np.array_equal(P.sorted_order(x), t.perm)


def test_block_jacobi_solves_the_regularised_blocks():
    x = uniform_points(200, 3, 8)          # blocks of 64, 64, 64 and a ragged 8
    s, reg = 0.1, 1e-3
    inv, perm = P.block_inverses(x, "gaussian", s, reg)
    assert [Ai.shape[0] for Ai in inv] == [64, 64, 64, 8]
    v = np.random.default_rng(9).normal(0, 1, 200)
    y = P.bj_sorted(inv, perm, v)
    xs = x[perm]
    for a, b in P.blocks(200):
        A = np.exp(-cdist(xs[a:b], xs[a:b], "sqeuclidean") / (2 * s * s)) + reg * np.eye(b - a)
        res = A @ y[a:b] - v[perm][a:b]
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(v[perm][a:b]) * np.linalg.cond(A)
    z = P.bj_apply(inv, perm, v)
    assert np.array_equal(z[perm], y)


def test_block_jacobi_of_far_apart_points_is_a_scaling():
    # points 10 s apart: off-diagonal kernel values exp(-50) ~ 2e-22 vanish next to 1
    x = np.zeros((100, 2))
    x[:, 0] = np.arange(100) * 1.0
    s, reg = 0.1, 0.25
    inv, perm = P.block_inverses(x, "gaussian", s, reg)
    v = np.random.default_rng(10).normal(0, 1, 100)
    assert np.allclose(P.bj_apply(inv, perm, v), v / (1.0 + reg), rtol=1e-15, atol=0)


def test_pairs_identity_and_zero_correction():
    x = uniform_points(300, 3, 11)
    inv, perm = P.block_inverses(x, "gaussian", 0.08, 1e-4)
    rng = np.random.default_rng(12)
    r = rng.normal(0, 1, 300)
    e = rng.normal(0, 1, 300)
    params = rand_params(P.LAYERS, 13)
    X, T, w = P.pairs(inv, perm, r, e)
    G, _ = P.forward(params, X)
    z = P.learned_apply(inv, perm, params, r, bf16=False)
    lhs = float(np.sum(w[:, None] * (G - T) ** 2))
    full = perm[:256]                      # the four full blocks; the ragged fifth has weight 0
    rhs = float(np.sum((z[full] - e[full]) ** 2) / np.sum(e * e))
    assert w[4] == 0.0 and np.all(w[:4] > 0)
    assert abs(lhs - rhs) <= 1e-12 * rhs
    # features are unit rows; s_b (x_b + t_b) rebuilds the error
    y = P.bj_sorted(inv, perm, r)
    Y, s = P._rows(y)
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0, rtol=1e-14)
    Erows, _ = P._rows(e[perm])
    assert np.allclose(s[:, None] * (X + T), Erows, rtol=0, atol=1e-12 * np.max(np.abs(e)))
    # a zero last layer leaves the block-Jacobi output
    p0 = params.copy()
    p0[-(256 * 64 + 64):] = 0.0
    assert np.allclose(P.learned_apply(inv, perm, p0, r), P.bj_apply(inv, perm, r), rtol=1e-15, atol=0)
