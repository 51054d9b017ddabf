"""Restarted GMRES(m) in FP64 (oracle).  Test infrastructure only.

The paper solves the interpolation system A lambda = f with a Krylov method and names
GMRES (section 1; section 4 before eq. 38) without fixing its details.  This is the
method of Saad and Schultz as usually stated: x0 = 0 (or a given guess), Arnoldi with
modified Gram-Schmidt, Givens rotations for the small least-squares problem, restart
after m steps, and a stop test on the true residual ||f - A x|| / ||f|| recomputed at
every restart.  An optional right preconditioner is applied flexibly (the basis of
preconditioned vectors Z is kept, as in FGMRES), so a nonlinear map is allowed.

Pinned by: agreement with a dense solve, the minimal-residual property of each iterate
over its Krylov space (brute-force least squares), finite termination on small cases and
scipy.sparse.linalg.gmres (tests/test_oracle_gmres.py).
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, restart: int = 50, rtol: float = 1e-8, maxiter: int = 1000, x0=None,
          precond=None):
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return np.zeros(n), {"iters": 0, "restarts": 0, "true_res": 0.0, "history": [0.0],
                             "converged": True}
    hist = []
    its = 0
    restarts = 0
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / bnorm)
        if beta / bnorm <= rtol or its >= maxiter:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = precond(V[j]) if precond is not None else V[j]
            Z[j] = z
            w = matvec(z)
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            hj1 = H[j + 1, j]
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = H[j, j] / den, hj1 / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if hj1 == 0.0 or abs(g[j + 1]) / bnorm <= rtol or its >= maxiter:
                break
            V[j + 1] = w / hj1
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        restarts += 1
    return x, {"iters": its, "restarts": restarts, "true_res": hist[-1], "history": hist,
               "converged": hist[-1] <= rtol}
