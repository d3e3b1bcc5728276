"""Nystrom sketch-and-solve (Section "Nystrom sketch-and-solve", algorithm of
the same name) in float64.

TEST INFRASTRUCTURE ONLY: see the package docstring.

Given the factored approximation A_hat = U diag(lam) U^T, the proxy system
(A_hat + mu I) x = b is solved with the Woodbury form of the lemma on
approximate regularized inversion, eq. (Woodbury):
  x_hat = U (Lambda + mu I)^{-1} U^T b + (1/mu) (I - U U^T) b.
"""
from __future__ import annotations

import numpy as np


def nystrom_sketch_solve(U: np.ndarray, lam: np.ndarray, mu: float, b: np.ndarray) -> np.ndarray:
    if not mu > 0:
        raise ValueError("sketch-and-solve needs mu > 0")
    Utb = U.T @ b
    inner = Utb / (lam + mu) if Utb.ndim == 1 else Utb / (lam + mu)[:, None]
    return U @ inner + (b - U @ Utb) / mu
