"""Nystrom PCG (Section 5.2, algorithm "Nystrom PCG") and reference solves.

Left-preconditioned CG on (A + mu I) x = b:
  r0 = b - (A + mu I) x0;  z0 = P^{-1} r0;  p0 = z0
  while not converged:
      v = (A + mu I) p0
      alpha = (r0^T z0) / (p0^T v)
      x = x0 + alpha p0;  r = r0 - alpha v
      z = P^{-1} r;  beta = (r^T z) / (r0^T z0)
      x0 <- x, r0 <- r, p0 <- z + beta p0, z0 <- z
Readings: the step size uses the current p and v (the printed step-size line
carries stale subscripts); the stopping test is applied to the recursively
updated residual and is relative, ||r||_2 <= tol ||b||_2 (the paper's
experiments use an absolute threshold; the relative form is the same test with
eta = tol ||b||); the iteration cap defaults to 500, the cap used in the
experiments of Section 6.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def nystrom_pcg(matvec, b: np.ndarray, mu: float, pinv, x0=None, tol: float = 1e-10,
                maxit: int = 500, history: bool = False) -> dict:
    """Solve (A + mu I) x = b for one right-hand side.  ``matvec(p)`` returns A p;
    ``pinv(r)`` returns P^{-1} r.  Returns x, iteration count and flags."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    r = b - (matvec(x) + mu * x)
    z = pinv(r)
    p = z.copy()
    rz = r @ z
    it = 0
    hist = [np.linalg.norm(r) / bnorm] if history else None
    converged = np.linalg.norm(r) <= tol * bnorm
    breakdown = False
    while not converged and it < maxit:
        v = matvec(p) + mu * p
        pv = p @ v
        if not pv > 0.0:
            breakdown = True
            break
        alpha = rz / pv
        x = x + alpha * p
        r = r - alpha * v
        z = pinv(r)
        rz_new = r @ z
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        it += 1
        rn = np.linalg.norm(r)
        if history:
            hist.append(rn / bnorm)
        converged = rn <= tol * bnorm
    return dict(x=x, iters=it, converged=bool(converged), breakdown=breakdown, history=hist)


def true_relres(op, mu: float, x: np.ndarray, b: np.ndarray) -> float:
    """||b - (A + mu I) x||_2 / ||b||_2 evaluated in float64."""
    r = b - (op.matmat(x) + mu * x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def dense_solve(A: np.ndarray, mu: float, b: np.ndarray) -> np.ndarray:
    """Exact solution of (A + mu I) x = b by a dense Cholesky factorisation (LAPACK)."""
    n = A.shape[0]
    c = sla.cho_factor(A + mu * np.eye(n), lower=True)
    return sla.cho_solve(c, b)
