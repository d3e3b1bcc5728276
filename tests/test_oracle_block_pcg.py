"""Pins of the oracle's block Nystrom PCG against facts fixed independently of
its code."""
import math

import numpy as np
import scipy.sparse.linalg as spla

from oracle import (RBFOp, block_nystrom_pcg, dense_solve, precond_inv_matrix, randomized_nystrom)
from workloads import krr_small, spectrum_psd


def _case(n=260, ell=20, seed=51, mu=1e-2):
    w = krr_small(n=n, d=5, ell=ell, seed=seed)
    op = RBFOp(w["X"], 1.5)
    r = randomized_nystrom(op, w["omega0"])
    return op, r, mu


def test_one_column_has_the_iterates_of_scipy_cg():
    op, r, mu = _case()
    n = op.n
    Amu = op.dense() + mu * np.eye(n)
    Pi = precond_inv_matrix(r["U"], r["lam"], mu)
    M = spla.LinearOperator((n, n), matvec=lambda v: Pi @ v)
    b = np.random.default_rng(52).standard_normal(n)
    for k in (1, 2, 4, 7):
        ours = block_nystrom_pcg(op.matmat, b[:, None], mu, lambda R: Pi @ R, tol=0.0, maxit=k)
        ref, _ = spla.cg(Amu, b, rtol=0.0, atol=0.0, maxiter=k, M=M)
        assert ours["iters"] == k
        np.testing.assert_allclose(ours["X"][:, 0], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_iterates_are_the_galerkin_solutions_on_the_block_krylov_space():
    """After k steps each column minimises the A_mu-norm error over
    span{Z0, (P^{-1} A_mu) Z0, ..., (P^{-1} A_mu)^{k-1} Z0}, Z0 = P^{-1} B:
    X_k = W (W^T A_mu W)^{-1} W^T B for an orthonormal basis W of that space."""
    op, r, mu = _case(n=220, seed=53)
    n, s = op.n, 3
    Amu = op.dense() + mu * np.eye(n)
    Pi = precond_inv_matrix(r["U"], r["lam"], mu)
    B = np.random.default_rng(54).standard_normal((n, s))
    for k in (1, 2, 4):
        blocks = [Pi @ B]
        for _ in range(k - 1):
            blocks.append(Pi @ (Amu @ blocks[-1]))
        W, _ = np.linalg.qr(np.hstack(blocks))
        want = W @ np.linalg.solve(W.T @ Amu @ W, W.T @ B)
        got = block_nystrom_pcg(op.matmat, B, mu, lambda R: Pi @ R, tol=0.0, maxit=k)["X"]
        np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-8 * np.abs(want).max())


def test_terminates_near_ceil_n_over_s_steps():
    """Block CG (identity preconditioner) on an n x n matrix with s generic
    right-hand sides spans the whole space after ceil(n / s) steps, so in exact
    arithmetic it terminates there; in float64 it reaches 1e-10 within a few
    more, while one column alone needs several times as many."""
    n, s = 48, 4
    A = spectrum_psd(np.logspace(0, 2, n), 55)
    B = np.random.default_rng(56).standard_normal((n, s))
    out = block_nystrom_pcg(lambda V: A @ V, B, 0.0, lambda R: R.copy(), tol=1e-10, maxit=100)
    assert out["converged"] and out["iters"] <= math.ceil(n / s) + 3
    single = block_nystrom_pcg(lambda V: A @ V, B[:, :1], 0.0, lambda R: R.copy(), tol=1e-10, maxit=200)
    assert single["converged"] and single["iters"] >= 3 * out["iters"]


def test_block_solution_equals_dense_solves():
    op, r, mu = _case(n=300, seed=57, mu=1e-3)
    Pi = precond_inv_matrix(r["U"], r["lam"], mu)
    B = np.random.default_rng(58).standard_normal((300, 5))
    out = block_nystrom_pcg(op.matmat, B, mu, lambda R: Pi @ R, tol=1e-12, maxit=500)
    assert out["converged"] and not out["breakdown"]
    xs = np.stack([dense_solve(op.dense(), mu, B[:, c]) for c in range(5)], axis=1)
    Amu = op.dense() + mu * np.eye(300)
    assert np.all(np.linalg.norm(Amu @ out["X"] - B, axis=0) <= 1e-11 * np.linalg.norm(B, axis=0))
    assert np.linalg.norm(out["X"] - xs) <= 1e-6 * np.linalg.norm(xs)
