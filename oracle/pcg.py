"""Projected preconditioned conjugate gradients (oracle; test infrastructure only).

Solves sign_k * Q_perp^T M Q_perp u = sign_k * Q_perp^T f (eq. phs_linsys_solve)
in the n-dimensional form: unknown w = Q_perp u kept in range(Pi), Pi = I - Q Q^T,
operator Pi M Pi, preconditioner Pi U~ U~^T Pi (the paper's Q_perp^T Sigma^{-1}
Q_perp with the Vecchia factor in place of the exact inverse, Sec. 2.2).

Reading of the stopping rule ("relative and absolute tolerances", Sec. 3): stop
when ||r_k||_2 <= max(rtol * ||Pi f||_2, atol), r_k the recursively updated,
unpreconditioned residual, x_0 = 0.  Parity unpinned beyond the textbook
properties tested (one iteration with the exact inverse as preconditioner, CG
iterates with the identity preconditioner).
"""
from __future__ import annotations

import numpy as np


def pcg_projected(matvec, precond, Q: np.ndarray, f: np.ndarray, sign: int,
                  rtol: float = 1e-8, atol: float = 0.0, maxit: int = 1000):
    def proj(v):
        return v - Q @ (Q.T @ v)

    b = sign * proj(np.asarray(f, dtype=np.float64))
    w = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    tol = max(rtol * bn, atol)
    hist = [np.linalg.norm(r)]
    if hist[0] <= tol:
        return w, 0, hist
    z = proj(precond(r))
    rho = r @ z
    p = z.copy()
    for it in range(1, maxit + 1):
        q = sign * proj(matvec(p))
        alpha = rho / (p @ q)
        w += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol:
            return w, it, hist
        z = proj(precond(r))
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return w, maxit, hist
