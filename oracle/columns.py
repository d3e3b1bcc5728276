"""Nystrom approximation from sampled columns (Section "Random projection
versus column sampling"; the kernel ridge regression experiments build the
preconditioner this way) in float64.

TEST INFRASTRUCTURE ONLY: see the package docstring.

The test matrix has 1-sparse columns: Omega = I[:, S] for a set S of l
distinct column indices (an input).  Everything else is the base algorithm
("Randomized Nystrom Approximation"): Omega is already orthonormal, so its QR
step returns it unchanged (up to column signs, which the approximation does
not depend on); Y = A Omega = A[:, S]; then steps 4-9 unchanged.
Reading: the paper does not state the sampling law; S is uniform without
replacement (the caller draws it).
"""
from __future__ import annotations

import numpy as np

from .nystrom import nystrom_factor


def selection_matrix(n: int, idx) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.int64)
    Om = np.zeros((n, idx.shape[0]), dtype=np.float64)
    Om[idx, np.arange(idx.shape[0])] = 1.0
    return Om


def column_nystrom(op, n: int, idx, shift: str = "fro") -> dict:
    """Y = A Omega with Omega = I[:, idx], then the factorisation steps."""
    Om = selection_matrix(n, idx)
    Y = op.matmat(Om)
    return nystrom_factor(Om, Y, shift=shift)
