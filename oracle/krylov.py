"""Flexible GMRES(m) (test infrastructure, see the package docstring).

The paper solves the Newton systems with right-preconditioned GMRES (Sec. 4):
A M^{-1} dy = -F, dx = M^{-1} dy.  Flexible GMRES (Saad 1993) keeps the preconditioned
vectors z_j = M^{-1} v_j and forms x = x0 + Z y; for a fixed linear M it produces the same
iterates as right-preconditioned GMRES.  Orthogonalisation is modified Gram-Schmidt and
the Hessenberg least-squares problem is reduced with Givens rotations
(r = hypot(a, b), c = a / r, s = b / r).  Convergence: |g_{j+1}| <= rtol ||b||; at the end
of each cycle the true residual is recomputed and the cycle restarts from x if it is not
below the tolerance.  The iteration count is the number of preconditioner applications.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    x: np.ndarray
    iters: int
    converged: bool
    true_relres: float
    history: list = field(default_factory=list)


def fgmres(matvec, precond, b, x0=None, restart=30, rtol=1e-8, maxit=1000) -> Result:
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return Result(np.zeros(n), 0, True, 0.0, [0.0])
    tol = rtol * bnorm
    its = 0
    hist = []
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / bnorm)
        if beta <= tol:
            return Result(x, its, True, beta / bnorm, hist)
        if its >= maxit:
            return Result(x, its, False, beta / bnorm, hist)
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
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = float(np.dot(V[i], w))
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            rr = math.hypot(a, bb)
            cs[j], sn[j] = a / rr, bb / rr
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol or hn == 0.0 or its >= maxit:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + Z[:k].T @ y
