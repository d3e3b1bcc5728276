"""Nystrom preconditioner (Section 5.1.2, eq. (NysPre)).

With A_hat = U Lambda U^T and lam_l its l-th (smallest) eigenvalue:
  P      = (1/(lam_l + mu)) U (Lambda + mu I) U^T + (I - U U^T)
  P^{-1} = (lam_l + mu) U (Lambda + mu I)^{-1} U^T + (I - U U^T)
Lambda is stored descending, so lam_l = lam[-1].
"""
from __future__ import annotations

import numpy as np


def precond_inv_apply(U: np.ndarray, lam: np.ndarray, mu: float, R: np.ndarray,
                      lam_l=None) -> np.ndarray:
    """P^{-1} R for a vector or an n x k block R, as the two terms of eq. (NysPre).
    ``lam_l`` overrides the scalar lam_l (the optimal preconditioner of
    eq. (OptLowRankPre) uses lambda_{l+1} there)."""
    lam_l = lam[-1] if lam_l is None else lam_l
    UtR = U.T @ R
    scale = (lam_l + mu) / (lam + mu)
    first = U @ (scale[:, None] * UtR if UtR.ndim == 2 else scale * UtR)
    second = R - U @ UtR
    return first + second


def precond_matrix(U: np.ndarray, lam: np.ndarray, mu: float, lam_l=None) -> np.ndarray:
    n = U.shape[0]
    lam_l = lam[-1] if lam_l is None else lam_l
    return (U * (lam + mu)) @ U.T / (lam_l + mu) + (np.eye(n) - U @ U.T)


def precond_inv_matrix(U: np.ndarray, lam: np.ndarray, mu: float, lam_l=None) -> np.ndarray:
    n = U.shape[0]
    lam_l = lam[-1] if lam_l is None else lam_l
    return (lam_l + mu) * (U / (lam + mu)) @ U.T + (np.eye(n) - U @ U.T)
