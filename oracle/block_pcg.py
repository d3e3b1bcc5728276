"""Block Nystrom PCG (Section "Block Nystrom PCG"): the Nystrom preconditioner
inside O'Leary's block conjugate gradient method, after Feng, Owen and Peric's
orthogonalisation of the right-hand sides, in float64.

TEST INFRASTRUCTURE ONLY: see the package docstring.

The paper names the two methods but prints no steps; these are the published
preconditioned block CG recurrences, restated (s right-hand sides sharing mu,
A_mu = A + mu I, P^{-1} the Nystrom preconditioner of eq. (NysPre)):
  pre-processing: B = Q0 T0 (thin QR; B must have full column rank); the
                  iteration solves A_mu Xt = Q0 and returns X = Xt T0
  Xt = 0, R = Q0, Z = P^{-1} R, D = Z, rho = Z^T R              (s x s)
  repeat:
     V = A_mu D
     alpha = (D^T V)^{-1} rho                                   (s x s solve)
     Xt = Xt + D alpha,  R = R - V alpha
     stop when every column c of R T0 (the residual of the original system)
       has ||(R T0)[:, c]|| <= tol ||B[:, c]||
     Z = P^{-1} R,  rho_new = Z^T R,  beta = rho^{-1} rho_new   (s x s solve)
     D = Z + D beta,  rho = rho_new
Readings: the orthogonalisation is taken to be a thin QR of the right-hand
side block before the iteration (the form in which it needs no further
orthogonalisation steps, as the paper says); the block stops when all columns
meet the tolerance (no deflation); a non-positive-definite D^T V or rho is a
breakdown; the iteration cap defaults to 500 as for the single-vector solver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def block_nystrom_pcg(matmat, B: np.ndarray, mu: float, pinv, tol: float = 1e-10, maxit: int = 500) -> dict:
    """Solve (A + mu I) X = B for the columns of B.  ``matmat(V)`` returns A V,
    ``pinv(R)`` returns P^{-1} R.  Returns X, iteration count and flags."""
    B = np.asarray(B, dtype=np.float64)
    Q0, T0 = np.linalg.qr(B)
    bn = np.linalg.norm(B, axis=0)
    s = B.shape[1]
    Xt = np.zeros_like(Q0)
    R = Q0.copy()
    Z = pinv(R)
    D = Z.copy()
    rho = Z.T @ R
    it = 0
    converged = bool(np.all(np.linalg.norm(R @ T0, axis=0) <= tol * bn))
    breakdown = False
    while not converged and it < maxit:
        V = matmat(D) + mu * D
        G = D.T @ V
        try:
            alpha = sla.cho_solve(sla.cho_factor(0.5 * (G + G.T)), rho)
        except np.linalg.LinAlgError:
            breakdown = True
            break
        Xt = Xt + D @ alpha
        R = R - V @ alpha
        it += 1
        converged = bool(np.all(np.linalg.norm(R @ T0, axis=0) <= tol * bn))
        if converged:
            break
        Z = pinv(R)
        rho_new = Z.T @ R
        try:
            beta = sla.cho_solve(sla.cho_factor(0.5 * (rho + rho.T)), rho_new)
        except np.linalg.LinAlgError:
            breakdown = True
            break
        D = Z + D @ beta
        rho = rho_new
    assert s == Xt.shape[1]
    return dict(X=Xt @ T0, iters=it, converged=converged, breakdown=breakdown)
