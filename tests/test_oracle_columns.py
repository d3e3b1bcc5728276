"""Pins of the oracle's column-sampling Nystrom approximation against facts
fixed independently of its code."""
import numpy as np

from oracle import DenseOp, RBFOp, column_nystrom, selection_matrix
from workloads import column_sample, krr_small, lowrank_psd


def _approx(r):
    return (r["U"] * r["lam"]) @ r["U"].T


def test_selection_matrix_is_orthonormal_and_selects():
    idx = column_sample(50, 7, 1)
    Om = selection_matrix(50, idx)
    assert np.array_equal(Om.T @ Om, np.eye(7))
    A = np.arange(2500.0).reshape(50, 50)
    assert np.array_equal(A @ Om, A[:, idx])


def test_column_formula_for_a_kernel_matrix():
    """A_hat = A(:,S) A(S,S)^{-1} A(S,:) (the Nystrom approximation of eq.
    (nys-unstable) with Omega = I[:, S]), here for an RBF kernel matrix."""
    w = krr_small(n=400, d=8, ell=10, seed=3)
    op = RBFOp(w["X"], w["sigma"])
    A = op.dense()
    idx = column_sample(400, 60, 4)
    r = column_nystrom(op, 400, idx)
    C = A[:, idx]
    W = A[np.ix_(idx, idx)]
    closed = C @ np.linalg.solve(W, C.T)
    assert np.linalg.norm(_approx(r) - closed, 2) <= 1e-9 * np.linalg.norm(A, 2)
    assert np.all(r["lam"][:-1] >= r["lam"][1:]) and r["lam"][-1] >= 0


def test_exact_recovery_of_low_rank_and_interpolation():
    A = lowrank_psd(120, 9, 5)
    idx = column_sample(120, 9, 6)
    r = column_nystrom(DenseOp(A), 120, idx)
    assert np.linalg.norm(_approx(r) - A, 2) <= 1e-10 * np.linalg.norm(A, 2)
    # full-rank A: the approximation reproduces A on the sampled rows and columns
    w = krr_small(n=200, d=3, ell=10, seed=8)
    op = RBFOp(w["X"], 2.0)
    A = op.dense()
    idx = column_sample(200, 25, 9)
    Ah = _approx(column_nystrom(op, 200, idx))
    assert np.abs(Ah[:, idx] - A[:, idx]).max() <= 1e-8 * np.abs(A).max()
    assert np.abs(Ah[idx, :] - A[idx, :]).max() <= 1e-8 * np.abs(A).max()
