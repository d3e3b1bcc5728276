"""Pins for the Nystrom preconditioner (eq. (NysPre)) and the spectrum bounds
of Proposition "Nystrom preconditioner: deterministic bound"."""
import numpy as np
import pytest

from oracle import (DenseOp, precond_inv_apply, precond_inv_matrix, precond_matrix,
                    randomized_nystrom)
from workloads import spectrum_psd


def _case(n=300, ell=25, seed=20, mu=1e-3):
    lam = 1.0 / np.arange(1, n + 1) ** 1.5
    A = spectrum_psd(lam, seed)
    om = np.random.default_rng(seed + 1).standard_normal((n, ell))
    r = randomized_nystrom(DenseOp(A), om)
    return A, lam, r, mu


def test_p_times_pinv_is_identity():
    A, _, r, mu = _case()
    P = precond_matrix(r["U"], r["lam"], mu)
    Pi = precond_inv_matrix(r["U"], r["lam"], mu)
    np.testing.assert_allclose(P @ Pi, np.eye(A.shape[0]), atol=1e-12)
    rng = np.random.default_rng(21)
    R = rng.standard_normal((A.shape[0], 3))
    np.testing.assert_allclose(precond_inv_apply(r["U"], r["lam"], mu, R), Pi @ R, atol=1e-12)
    np.testing.assert_allclose(precond_inv_apply(r["U"], r["lam"], mu, R[:, 0]), Pi @ R[:, 0], atol=1e-12)


def test_pinv_spectrum():
    """eig(P^{-1}) lies in [(lam_l+mu)/(lam_1+mu), 1] and reaches 1 when l < n."""
    A, _, r, mu = _case()
    e = np.linalg.eigvalsh(precond_inv_matrix(r["U"], r["lam"], mu))
    lh = r["lam"]
    assert e.max() == pytest.approx(1.0, abs=1e-12)
    assert e.min() >= (lh[-1] + mu) / (lh[0] + mu) * (1 - 1e-10)


@pytest.mark.parametrize("mu", [1e-1, 1e-3, 1e-5])
def test_preconditioned_spectrum_bounds(mu):
    """mu <= lambda_min(P^{-1/2} A_mu P^{-1/2}) and
    lambda_max <= lam_l + mu + ||E||; kappa within the proposition's two-sided bound."""
    A, lam, r, _ = _case(mu=mu)
    n = A.shape[0]
    U, lh = r["U"], r["lam"]
    Pi = precond_inv_matrix(U, lh, mu)
    w, V = np.linalg.eigh(Pi)
    Pih = (V * np.sqrt(w)) @ V.T
    M = Pih @ (A + mu * np.eye(n)) @ Pih
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    E = np.linalg.norm(A - (U * lh) @ U.T, 2)
    lam_n = lam.min()
    assert ev.min() >= mu * (1 - 1e-8)
    assert ev.max() <= (lh[-1] + mu + E) * (1 + 1e-10)
    kappa = ev.max() / ev.min()
    lower = max((lh[-1] + mu) / (lam_n + mu), 1.0)
    upper = (lh[-1] + mu + E) * min(1 / mu, (lh[-1] + lam_n + 2 * mu) / ((lh[-1] + mu) * (lam_n + mu)))
    assert lower * (1 - 1e-8) <= kappa <= upper * (1 + 1e-8)


def test_optimal_preconditioner_condition_number():
    """With exact eigenpairs and lambda_{l+1} in place of lam_l:
    kappa = (lambda_{l+1} + mu) / (lambda_n + mu)  (eq. (OptCondNumber))."""
    n, ell, mu = 200, 15, 1e-3
    lam = 1.0 / np.arange(1, n + 1) ** 2
    A = spectrum_psd(lam, 22)
    w, V = np.linalg.eigh(A)
    idx = np.argsort(w)[::-1]
    w, V = w[idx], V[:, idx]
    Pi = precond_inv_matrix(V[:, :ell], w[:ell], mu, lam_l=w[ell])
    ev = np.sort(np.real(np.linalg.eigvals(Pi @ (A + mu * np.eye(n)))))
    assert ev[-1] / ev[0] == pytest.approx((w[ell] + mu) / (w[-1] + mu), rel=1e-8)


def test_woodbury_and_sketch_and_solve_bound():
    """(A_hat + mu I)^{-1} = U (Lambda + mu I)^{-1} U^T + (I - U U^T)/mu and the
    sketch-and-solve error bound ||x_hat - x*|| / ||x*|| <= ||E|| / mu."""
    A, _, r, mu = _case(mu=1e-2)
    n = A.shape[0]
    U, lh = r["U"], r["lam"]
    Ahat = (U * lh) @ U.T
    W = (U / (lh + mu)) @ U.T + (np.eye(n) - U @ U.T) / mu
    np.testing.assert_allclose(W, np.linalg.inv(Ahat + mu * np.eye(n)), atol=1e-9)
    b = np.random.default_rng(23).standard_normal(n)
    xs = np.linalg.solve(A + mu * np.eye(n), b)
    xh = W @ b
    E = np.linalg.norm(A - Ahat, 2)
    assert np.linalg.norm(xh - xs) / np.linalg.norm(xs) <= E / mu * (1 + 1e-10)
