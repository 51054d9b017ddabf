"""Lagrange transfer between frequency grids of the interpolating multilevel scheme (oracle, FP64).
Test infrastructure only.

Section 4.1 moves expansions between levels whose frequency grids differ by a factor of two: a
phase e^{i (xi/2) x} on the coarse level is written through the fine-level nodes xi_k by local
Lagrange interpolation, e^{i (xi/2) x} ~ sum_k P_k(xi/2) e^{i xi_k x}, with P_k the Lagrange basis
polynomial of node k.  The printed basis has its indices garbled; the standard basis
P_k(t) = prod_{l != k} (t - xi_l) / (xi_k - xi_l) is used (it reproduces the paper's table).

``transfer`` moves a centred expansion between two grids the way the interpolating scheme
moves it between levels: the values at the target nodes from K consecutive source nodes around
each target node (the standard basis on those nodes), along every axis of a tensor grid.  It is
used by the banded far field between the grids of its bands; pinned against the direct
definition of the target expansion (tests/test_oracle_lagrange.py).

``halfwave_error`` is the table's quantity: the largest deviation over xi in [-sigma, sigma] and
x in [-a, a], for K equispaced nodes on [-sigma, sigma] including both ends (sigma = pi, a = 1 in
the table).  Pinned by the paper's Table "Lagrange interpolation error" (tests/golden/) and by
exactness on polynomials of degree < K (tests/test_oracle_lagrange.py).
"""
from __future__ import annotations

import numpy as np


def nodes(K: int, sigma: float = np.pi) -> np.ndarray:
    return np.linspace(-sigma, sigma, K)


def basis(xk, t) -> np.ndarray:
    """(len(t), K) matrix of the Lagrange basis polynomials of the nodes xk at the points t."""
    xk = np.asarray(xk, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    K = xk.shape[0]
    out = np.ones((t.shape[0], K))
    for k in range(K):
        for l in range(K):
            if l != k:
                out[:, k] *= (t - xk[l]) / (xk[k] - xk[l])
    return out


def halfwave_error(K: int, a: float = 1.0, sigma: float = np.pi, nxi: int = 21, nx: int = 201) -> float:
    """max over xi (nxi points on [-sigma, sigma]) and x (nx points on [-a, a]) of
    |e^{i (xi/2) x} - sum_k P_k(xi/2) e^{i xi_k x}|."""
    xk = nodes(K, sigma)
    xi = np.linspace(-sigma, sigma, nxi)
    x = np.linspace(-a, a, nx)
    P = basis(xk, xi / 2.0)                                  # (nxi, K)
    approx = P @ np.exp(1j * xk[:, None] * x[None, :])       # (nxi, nx)
    exact = np.exp(1j * (xi / 2.0)[:, None] * x[None, :])
    return float(np.max(np.abs(exact - approx)))


def stencil(src, t: float, K: int):
    """First index and Lagrange weights of the K consecutive source nodes around t: the node
    interval holding t with K/2 nodes on either side, shifted inwards at the ends of the grid."""
    src = np.asarray(src, dtype=np.float64)
    h = src[1] - src[0]
    j = int(np.floor((t - src[0]) / h)) - K // 2 + 1
    j = max(0, min(len(src) - K, j))
    return j, basis(src[j:j + K], t)[0]


def transfer(V, src, tgt, K: int):
    """Values at the tensor grid tgt^d of the function whose values at src^d are V (complex,
    shape (len(src),) * d), interpolated axis by axis with K-point stencils."""
    out = np.asarray(V, dtype=np.complex128)
    d = out.ndim
    M = np.zeros((len(tgt), len(src)))
    for i, t in enumerate(tgt):
        j, w = stencil(src, t, K)
        M[i, j:j + K] = w
    for k in range(d):
        out = np.moveaxis(np.tensordot(M, np.moveaxis(out, k, 0), axes=(1, 0)), 0, k)
    return out
