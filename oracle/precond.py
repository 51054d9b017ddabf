"""Right preconditioners for the GMRES solve (oracle, FP64).  Test infrastructure only.

The paper solves A lambda = f with a Krylov method (section 1 names GMRES) and says nothing
about preconditioning; both preconditioners here are additions of the library, written
out plainly so that the device path can be checked against them:

* Blocks.  The points in the tree's Morton order (``oracle.tree``) are cut into blocks of
  64 consecutive points; block b holds sorted points [64 b, min(64 b + 64, n)).
* Block-Jacobi.  y_b = (A_bb + reg I)^{-1} v_b for every block, A_bb the exact kernel
  matrix of the block's points.
* Learned correction.  z_b = y_b + s_b g(y_b / s_b) with s_b = ||y_b||_2 (z_b = 0 when
  s_b = 0) and g a multilayer perceptron 64 -> 256 -> 256 -> 256 -> 64 with ReLU after
  each hidden layer.  Rows shorter than 64 (the ragged last block) are zero-padded; the
  outputs beyond the block's length are ignored.
* Training pairs.  From a residual r and its error e = A^{-1} r (both in caller order):
  features x_b = y_b / s_b, targets t_b = (e_b - y_b) / s_b and weights
  w_b = s_b^2 / ||e||^2, so that sum_b w_b ||g(x_b) - t_b||^2 = ||z - e||^2 / ||e||^2 over
  the full blocks.  A ragged last block gets weight 0 (its padded outputs are unused, so
  they carry no target).
* Loss over a set of rows: L = sum_r w_r ||g(x_r) - t_r||^2 / sum_r w_r, minimised with
  Adam (Kingma and Ba, 2015: bias-corrected first and second moment estimates).

Parameter vector (FP32 on the device, FP64 here), in this order: W1 (256 x 64, row-major
[out][in]), b1 (256), W2 (256 x 256), b2, W3 (256 x 256), b3, W4 (64 x 256), b4 (64):
164672 values.

BF16 emulation (``forward(..., bf16=True)``): the inference kernel rounds its inputs, its
weights and each hidden activation to bfloat16 (round to nearest even) and accumulates
products in FP32; the oracle rounds the same values the same way and accumulates in FP64.

Pins (tests/test_oracle_precond.py): the gradient against central finite differences, a
hand-worked two-layer example, a network whose ReLUs are all active reducing to the
product of its affine maps, Adam's first step moving each parameter by lr in the
direction of -sign(g), bfloat16 rounding against torch's conversion, block-Jacobi output
solving the regularised block systems, the closed form of a block of far-apart points,
and the pair identity above.
"""
from __future__ import annotations

import numpy as np

from . import rbf
from . import tree as otree

BLOCK = 64
LAYERS = [(64, 256), (256, 256), (256, 256), (256, 64)]   # (in, out) per layer


def nparams(layers=LAYERS) -> int:
    return sum(i * o + o for i, o in layers)


def unpack(params, layers=LAYERS):
    """Split the flat parameter vector into [(W (out, in), b (out,)), ...]."""
    p = np.asarray(params, dtype=np.float64)
    out, k = [], 0
    for i, o in layers:
        W = p[k:k + i * o].reshape(o, i)
        k += i * o
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.shape[0], "parameter vector has the wrong length"
    return out


def round_bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the top 16 bits of an IEEE float32; the value is first rounded to
    float32, then the low 16 bits are rounded off with ties going to an even result.
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, X, layers=LAYERS, bf16: bool = False):
    """g(X) for rows X (m, in).  Returns (G, acts) with acts[l] the input of layer l."""
    Ws = unpack(params, layers)
    h = np.asarray(X, dtype=np.float64)
    if bf16:
        h = round_bf16(h)
    acts = []
    for l, (W, b) in enumerate(Ws):
        acts.append(h)
        Wl = round_bf16(W) if bf16 else W
        z = h @ Wl.T + b
        if l + 1 < len(Ws):
            h = np.maximum(z, 0.0)
            if bf16:
                h = round_bf16(h)
        else:
            h = z
    return h, acts


def loss(params, X, T, w, layers=LAYERS) -> float:
    G, _ = forward(params, X, layers)
    w = np.asarray(w, dtype=np.float64)
    return float(np.sum(w[:, None] * (G - T) ** 2) / np.sum(w))


def grad(params, X, T, w, layers=LAYERS):
    """(loss, dL/dparams) by backpropagation through the layers in reverse order."""
    Ws = unpack(params, layers)
    G, acts = forward(params, X, layers)
    w = np.asarray(w, dtype=np.float64)
    W_sum = float(np.sum(w))
    L = float(np.sum(w[:, None] * (G - T) ** 2) / W_sum)
    delta = 2.0 * w[:, None] * (G - T) / W_sum          # dL/d(output of the last layer)
    grads = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        W, _ = Ws[l]
        grads[l] = (delta.T @ acts[l], delta.sum(axis=0))
        if l > 0:
            delta = (delta @ W) * (acts[l] > 0.0)            # through the ReLU of layer l-1
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam(params, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update at step t (1-based); returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# -- block-Jacobi and the learned correction ----------------------------------------------

def blocks(n: int):
    return [(b, min(b + BLOCK, n)) for b in range(0, n, BLOCK)]


def sorted_order(points) -> np.ndarray:
    """perm[i] = caller index of the i-th point in Morton order (the tree's sort)."""
    x = np.asarray(points)
    B = otree.bits_per_dim(x.shape[1])
    lo, ext = otree.root_cube(x)
    keys = otree.morton(otree.quantize(x, lo, ext, B), B)
    return np.argsort(keys, kind="stable").astype(np.int64)


def block_inverses(points, kernel: str, shape: float, reg: float):
    """[(A_bb + reg I)^{-1}] for the blocks of the Morton order, and that order."""
    x = np.asarray(points, dtype=np.float64)
    perm = sorted_order(points)
    xs = x[perm]
    inv = []
    for a, b in blocks(x.shape[0]):
        p = xs[a:b]
        r2 = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
        A = rbf.phi_of_r2(kernel, r2, shape) + reg * np.eye(b - a)
        inv.append(np.linalg.inv(A))
    return inv, perm


def bj_sorted(inv, perm, v):
    """Block-Jacobi output y in Morton order."""
    vs = np.asarray(v, dtype=np.float64)[perm]
    y = np.empty_like(vs)
    for (a, b), Ai in zip(blocks(vs.shape[0]), inv):
        y[a:b] = Ai @ vs[a:b]
    return y


def bj_apply(inv, perm, v):
    z = np.empty(len(perm))
    z[perm] = bj_sorted(inv, perm, v)
    return z


def _rows(y):
    """Zero-padded rows (nblocks, 64) of a Morton-ordered vector, and the block norms."""
    n = y.shape[0]
    nb = (n + BLOCK - 1) // BLOCK
    R = np.zeros((nb, BLOCK))
    for k, (a, b) in enumerate(blocks(n)):
        R[k, :b - a] = y[a:b]
    return R, np.sqrt((R * R).sum(axis=1))


def learned_apply(inv, perm, params, v, bf16: bool = True):
    y = bj_sorted(inv, perm, v)
    Y, s = _rows(y)
    X = np.divide(Y, s[:, None], out=np.zeros_like(Y), where=s[:, None] > 0)
    G, _ = forward(params, X, bf16=bf16)
    zs = np.empty_like(y)
    for k, (a, b) in enumerate(blocks(y.shape[0])):
        zs[a:b] = y[a:b] + s[k] * G[k, :b - a] if s[k] > 0 else 0.0
    z = np.empty_like(zs)
    z[perm] = zs
    return z


def pairs(inv, perm, r, e):
    """Training rows (X, T, w) of one (residual, error) pair; one row per block."""
    y = bj_sorted(inv, perm, r)
    es = np.asarray(e, dtype=np.float64)[perm]
    Y, s = _rows(y)
    E, _ = _rows(es)
    enorm2 = float(np.sum(es * es))
    ok = s > 0
    full = np.array([b - a == BLOCK for a, b in blocks(y.shape[0])])
    X = np.zeros_like(Y)
    T = np.zeros_like(Y)
    X[ok] = Y[ok] / s[ok, None]
    T[ok] = (E[ok] - Y[ok]) / s[ok, None]
    w = np.where(ok & full, s * s / enorm2, 0.0) if enorm2 > 0 else np.zeros_like(s)
    return X, T, w
