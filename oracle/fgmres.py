"""Restarted flexible GMRES (right preconditioning).

Oracle (test infrastructure only): used for the CPU baseline timings and for
iteration-count context, never for parity of the solution (the solution's
reference is the direct solve in ``kkt.solve_direct``).

Paper passage followed: Section 5 solves the KKT systems with flexible GMRES
(Saad 1993) and stops on the relative residual ||r_k|| / ||b||.  Reading:
restart length m (the paper does not restart), zero initial guess, modified
Gram-Schmidt Arnoldi, Givens rotations for the small least-squares problem,
and acceptance on the true residual at the end of each cycle.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_A, apply_P, b: np.ndarray, tol: float = 1e-8, restart: int = 30,
           max_iter: int = 1000):
    """Solve A x = b.  Returns (x, info) with info = dict(iters, rel_res, history)."""
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    history = []
    it = 0
    if bnorm == 0.0:
        return x, dict(iters=0, rel_res=0.0, history=history, converged=True)
    r = b - apply_A(x)
    beta = np.linalg.norm(r)
    while it < max_iter:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            Z[j] = apply_P(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x, dict(iters=it, rel_res=beta / bnorm, history=history, converged=True)
    return x, dict(iters=it, rel_res=beta / bnorm, history=history, converged=False)
