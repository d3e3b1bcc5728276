"""Pins for the oracle's Nystrom PCG: LAPACK Cholesky solves, scipy's CG
iterates, the CG convergence theorem with the exact condition number, the
special cases rank(A) < l and rank(A) = l, and the expectation bound of
Theorem "Nystrom preconditioning"."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import (DenseOp, RBFOp, dense_solve, nystrom_pcg, precond_inv_apply,
                    precond_inv_matrix, randomized_nystrom, true_relres)
from workloads import krr_small, lowrank_psd, spectrum_psd


def _rbf_case(n=400, ell=40, seed=30, mu=1e-3):
    w = krr_small(n=n, d=8, ell=ell, seed=seed)
    op = RBFOp(w["X"], w["sigma"])
    b = op.matmat(w["w"]) + w["noise"] * w["eps"]
    r = randomized_nystrom(op, w["omega0"])
    return op, b, r, mu


def test_pcg_matches_dense_cholesky():
    op, b, r, mu = _rbf_case()
    out = nystrom_pcg(op.matmat, b, mu, lambda v: precond_inv_apply(r["U"], r["lam"], mu, v), tol=1e-12,
                      maxit=2000)
    assert out["converged"]
    xs = dense_solve(op.dense(), mu, b)
    K = op.dense()
    ev = np.linalg.eigvalsh(K)
    kappa = (ev.max() + mu) / (max(ev.min(), 0) + mu)
    assert true_relres(op, mu, out["x"], b) <= 1e-11
    assert np.linalg.norm(out["x"] - xs) / np.linalg.norm(xs) <= kappa * 1e-12


def test_pcg_iterates_match_scipy_cg():
    """Same iterates as scipy.sparse.linalg.cg with M = P^{-1} (any iteration count)."""
    op, b, r, mu = _rbf_case(n=250, ell=20, seed=31, mu=1e-2)
    n = op.n
    Amu = op.dense() + mu * np.eye(n)
    Pi = precond_inv_matrix(r["U"], r["lam"], mu)
    M = spla.LinearOperator((n, n), matvec=lambda v: Pi @ v)
    for k in (1, 2, 3, 5, 8):
        ours = nystrom_pcg(op.matmat, b, mu, lambda v: Pi @ v, tol=0.0, maxit=k)
        ref, _ = spla.cg(Amu, b, rtol=0.0, atol=0.0, maxiter=k, M=M)
        assert ours["iters"] == k
        np.testing.assert_allclose(ours["x"], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_error_follows_cg_bound():
    """||x_t - x*||_{A_mu} / ||x*||_{A_mu} <= 2 ((sqrt k - 1)/(sqrt k + 1))^t with k the exact
    condition number of P^{-1/2} A_mu P^{-1/2} (standard CG theorem used in Section 5.3)."""
    n, ell, mu = 300, 20, 1e-3
    lam = 1.0 / np.arange(1, n + 1) ** 1.5
    A = spectrum_psd(lam, 32)
    r = randomized_nystrom(DenseOp(A), np.random.default_rng(33).standard_normal((n, ell)))
    Pi = precond_inv_matrix(r["U"], r["lam"], mu)
    Amu = A + mu * np.eye(n)
    ev = np.real(np.linalg.eigvals(Pi @ Amu))
    kappa = ev.max() / ev.min()
    b = np.random.default_rng(34).standard_normal(n)
    xs = np.linalg.solve(Amu, b)
    q = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    nx = np.sqrt(xs @ Amu @ xs)
    for t in range(1, 25):
        x = nystrom_pcg(lambda v: A @ v, b, mu, lambda v: Pi @ v, tol=0.0, maxit=t)["x"]
        e = x - xs
        assert np.sqrt(e @ Amu @ e) / nx <= 2 * q ** t * (1 + 1e-6) + 1e-13


@pytest.mark.parametrize("ell,maxit", [(64, 2), (40, 3)])
def test_low_rank_iteration_counts(ell, maxit):
    """rank(A) < l: A_hat = A so P^{-1} A_mu has one eigenvalue (1 step in exact
    arithmetic); rank(A) = l: two distinct eigenvalues (2 steps)."""
    A = lowrank_psd(512, 40, seed=35)
    mu = 1e-3
    r = randomized_nystrom(DenseOp(A), np.random.default_rng(36).standard_normal((512, ell)))
    b = np.random.default_rng(37).standard_normal(512)
    out = nystrom_pcg(lambda v: A @ v, b, mu, lambda v: precond_inv_apply(r["U"], r["lam"], mu, v),
                      tol=1e-10, maxit=50)
    assert out["converged"] and out["iters"] <= maxit


def test_identity_preconditioner_is_plain_cg():
    op, b, _, mu = _rbf_case(n=200, ell=10, seed=38, mu=1e-1)
    n = op.n
    Amu = op.dense() + mu * np.eye(n)
    ours = nystrom_pcg(op.matmat, b, mu, lambda v: v.copy(), tol=0.0, maxit=6)
    ref, _ = spla.cg(Amu, b, rtol=0.0, atol=0.0, maxiter=6)
    np.testing.assert_allclose(ours["x"], ref, rtol=1e-10, atol=1e-12)


def test_expected_condition_number_below_28():
    """Theorem (Nystrom preconditioning): l = 2 ceil(1.5 d_eff) + 1 gives E[kappa] < 28."""
    n, mu = 512, 1e-3
    lam = 1.0 / np.arange(1, n + 1) ** 2
    deff = float(np.sum(lam / (lam + mu)))
    ell = 2 * int(np.ceil(1.5 * deff)) + 1
    assert ell == 143
    A = spectrum_psd(lam, 39)
    Amu = A + mu * np.eye(n)
    ks = []
    for s in range(20):
        om = np.random.default_rng(1000 + s).standard_normal((n, ell))
        r = randomized_nystrom(DenseOp(A), om)
        ev = np.real(np.linalg.eigvals(precond_inv_matrix(r["U"], r["lam"], mu) @ Amu))
        ks.append(ev.max() / ev.min())
    assert np.mean(ks) < 28.0


def test_maxit_and_breakdown_flags():
    op, b, r, mu = _rbf_case(n=200, ell=10, seed=40)
    out = nystrom_pcg(op.matmat, b, mu, lambda v: precond_inv_apply(r["U"], r["lam"], mu, v), tol=1e-14,
                      maxit=3)
    assert out["iters"] == 3 and not out["converged"]
    # indefinite operator: p^T v <= 0 stops the iteration
    Aneg = -np.eye(50)
    out = nystrom_pcg(lambda v: Aneg @ v, np.ones(50), 0.0, lambda v: v, tol=1e-10, maxit=10)
    assert out["breakdown"] and not out["converged"]
