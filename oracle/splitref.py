"""Oracle B: the near/far split of eq. (38), evaluated pair by pair.  Test infrastructure only.

eq. (38) writes the matrix-vector product as a near field (exact kernel over the
neighbour groups N_a of the target's group) plus a far field evaluated through the
quadrature kernel of eq. (35)/(37).  Because eq. (37) is an exact factorisation of the
quadrature kernel, a fast evaluation of the far field must reproduce, up to rounding,
the brute-force sum written here:

    u_i = sum_{j in near(a_i)} lam_j Phi(x_i - x_j)
        + sum_{j in far(a_i)}  lam_j Phi^Q(x_i - x_j),

with near(a) = points of the leaves in the near list U(a) (``tree.near_lists``), and
far(a) = points whose coarse cell (level lc) lies within Chebyshev distance r of the
coarse cell of a, minus near(a).  Pairs outside that stencil are dropped (the pruning
of the Gaussian's negligible interactions; with lc = 0 nothing is dropped).

Phi^Q for the Gaussian is the tensor trapezoid quadrature of ``bandlimit``.
"""
from __future__ import annotations

import numpy as np

from . import bandlimit
from .rbf import GAUSSIAN, phi_of_r2
from .tree import build, coarse_cell_coords, near_lists


def split_reference(points, lam, kernel: str, shape: float, n_max: int, lc: int, r: int,
                    sigma: float, mn: int, max_level: int = 64, tree=None):
    if kernel != GAUSSIAN:
        raise NotImplementedError("split reference is written for the Gaussian quadrature")
    x = np.asarray(points)
    n, d = x.shape
    if tree is None:
        tree = build(x, n_max, max_level, min_level=lc)
    ptr, idx = near_lists(tree)
    perm = tree.perm
    xs = x[perm].astype(np.float64)
    ls = np.asarray(lam, dtype=np.float64)[perm]
    lb = tree.leaf_begin
    cc = coarse_cell_coords(tree.coarse_cell(lc), d, lc)          # (nleaves, d)
    counts = np.diff(lb)
    pcell = np.repeat(cc, counts, axis=0)                          # (n, d) per sorted point
    u = np.zeros(n)
    for a in range(tree.nleaves):
        t0, t1 = int(lb[a]), int(lb[a + 1])
        T = xs[t0:t1]
        near_mask = np.zeros(n, dtype=bool)
        for b in idx[ptr[a]:ptr[a + 1]]:
            near_mask[lb[b]:lb[b + 1]] = True
        stencil = np.all(np.abs(pcell - cc[a]) <= r, axis=1)
        far_mask = stencil & ~near_mask
        jn = np.nonzero(near_mask)[0]
        jf = np.nonzero(far_mask)[0]
        dn = T[:, None, :] - xs[None, jn, :]
        val = phi_of_r2(kernel, (dn * dn).sum(-1), shape) @ ls[jn]
        if jf.size:
            for c0 in range(0, jf.size, 4096):
                jj = jf[c0:c0 + 4096]
                df = T[:, None, :] - xs[None, jj, :]
                val = val + bandlimit.phi_q_gauss(df, shape, sigma, mn) @ ls[jj]
        u[t0:t1] = val
    out = np.empty(n)
    out[perm] = u
    return out
