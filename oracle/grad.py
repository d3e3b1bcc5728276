"""Gradients of a scalar loss through the solution x = (A + mu I)^{-1} b.

The paper does not treat differentiation; these are the standard adjoint
(implicit-function) formulas.  With lambda = (A + mu I)^{-1} dL/dx:
  dL/db     = lambda
  dL/dmu    = -lambda^T x
  dL/dsigma = (explicit part) - lambda^T (dK/dsigma) x,
              dK_ij/dsigma = K_ij ||x_i - x_j||^2 / sigma^3        (RBF operator)
  dL/dX     = -(X x lambda^T + X lambda x^T) * scale                (A = scale X^T X)
"""
from __future__ import annotations

import numpy as np

from .operators import RBFOp, XtXOp, rbf_kernel_block


def adjoint_gradients(op, mu: float, x: np.ndarray, gx: np.ndarray, solve) -> dict:
    """``solve(rhs)`` must return (A + mu I)^{-1} rhs in float64."""
    lam = solve(gx)
    out = dict(lam=lam, gb=lam, gmu=-float(lam @ x))
    if isinstance(op, RBFOp):
        out["gsigma"] = -float(lam @ op.dsigma_matmat(x))
    if isinstance(op, XtXOp):
        X = op.X
        out["gX"] = -op.scale * (np.outer(X @ x, lam) + np.outer(X @ lam, x))
    return out


def validation_loss(Xtr, Xval, yval, sigma: float, x: np.ndarray) -> float:
    """L = ||K_val,tr x - y_val||^2."""
    Kv = rbf_kernel_block(Xval, Xtr, sigma)
    r = Kv @ x - yval
    return float(r @ r)


def validation_loss_grads(Xtr, Xval, yval, sigma: float, mu: float, x: np.ndarray, solve) -> dict:
    """Value and gradients (mu, sigma, b) of L = ||K_val,tr x(mu, sigma) - y_val||^2,
    where x solves (K_tr + mu I) x = b."""
    Xtr = np.asarray(Xtr, dtype=np.float64)
    Xval = np.asarray(Xval, dtype=np.float64)
    Kv = rbf_kernel_block(Xval, Xtr, sigma)
    rv = Kv @ x - yval
    L = float(rv @ rv)
    gx = 2.0 * (Kv.T @ rv)
    # explicit sigma dependence of K_val: 2 r_val^T (dK_val/dsigma) x
    d2 = (Xval * Xval).sum(1)[:, None] + (Xtr * Xtr).sum(1)[None, :] - 2.0 * (Xval @ Xtr.T)
    np.maximum(d2, 0.0, out=d2)
    dKv = Kv * d2 / sigma ** 3
    explicit = 2.0 * float(rv @ (dKv @ x))
    g = adjoint_gradients(RBFOp(Xtr, sigma), mu, x, gx, solve)
    g["gsigma"] = explicit + g["gsigma"]
    g["L"] = L
    g["gx"] = gx
    return g
