"""Randomized power estimate of ||E|| = ||A - U Lambda U^T|| (Appendix,
algorithm "Randomized Power method for estimating ||E||").

  v0 = g / ||g||
  repeat q times:  v = A v0 - U (Lambda (U^T v0));  E = v0^T v;  v0 = v / ||v||
The starting vector g is a random input.
"""
from __future__ import annotations

import numpy as np


def rand_pow_err_est(op, U: np.ndarray, lam: np.ndarray, q: int, g: np.ndarray) -> float:
    v0 = np.asarray(g, dtype=np.float64) / np.linalg.norm(g)
    E = 0.0
    for _ in range(q):
        v = op.matmat(v0) - U @ (lam * (U.T @ v0))
        E = float(v0 @ v)
        v0 = v / np.linalg.norm(v)
    return E
