"""Pins for the adjoint gradients (central finite differences of LAPACK solves,
and a closed form), the randomized power error estimate, and the Philox
generator (Random123 known-answer vectors)."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import (DenseOp, RBFOp, XtXOp, adjoint_gradients, dense_solve, gaussian_philox,
                    philox4x32_10, rand_pow_err_est, randomized_nystrom)
from oracle.grad import validation_loss, validation_loss_grads
from workloads import spectrum_psd


def _K(X, s):
    return np.exp(-cdist(X, X, "sqeuclidean") / (2 * s * s))


def test_gradients_rbf_vs_central_differences():
    rng = np.random.default_rng(50)
    n = 120
    X = rng.standard_normal((n, 3))
    sigma, mu = 1.3, 0.05
    b = rng.standard_normal(n)
    c = rng.standard_normal(n)
    loss = lambda x: float(c @ x + 0.5 * x @ x)
    solve = lambda s, m, bb: np.linalg.solve(_K(X, s) + m * np.eye(n), bb)
    x = solve(sigma, mu, b)
    g = adjoint_gradients(RBFOp(X, sigma), mu, x, c + x, lambda v: solve(sigma, mu, v))
    h = 1e-4
    fd_mu = (loss(solve(sigma, mu * (1 + h), b)) - loss(solve(sigma, mu * (1 - h), b))) / (2 * h * mu)
    fd_s = (loss(solve(sigma * (1 + h), mu, b)) - loss(solve(sigma * (1 - h), mu, b))) / (2 * h * sigma)
    assert g["gmu"] == pytest.approx(fd_mu, rel=1e-6)
    assert g["gsigma"] == pytest.approx(fd_s, rel=1e-6)
    for i in (0, 7, 50):
        e = np.zeros(n)
        e[i] = h
        fd_b = (loss(solve(sigma, mu, b + e)) - loss(solve(sigma, mu, b - e))) / (2 * h)
        assert g["gb"][i] == pytest.approx(fd_b, rel=1e-6, abs=1e-9)


def test_gradient_mu_closed_form():
    """L = c^T x:  dL/dmu = -c^T (A + mu I)^{-2} b (eigendecomposition)."""
    n, mu = 80, 0.01
    A = spectrum_psd(1.0 / np.arange(1, n + 1), 51)
    rng = np.random.default_rng(52)
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    w, V = np.linalg.eigh(A)
    closed = -float((V.T @ c) @ ((V.T @ b) / (w + mu) ** 2))
    x = dense_solve(A, mu, b)
    g = adjoint_gradients(DenseOp(A), mu, x, c, lambda v: dense_solve(A, mu, v))
    assert g["gmu"] == pytest.approx(closed, rel=1e-10)


def test_gradient_xtx_data_vs_central_differences():
    rng = np.random.default_rng(53)
    m, n, mu = 30, 12, 0.1
    X = rng.standard_normal((m, n))
    b = rng.standard_normal(n)
    c = rng.standard_normal(n)
    solve = lambda XX, v: np.linalg.solve(XX.T @ XX + mu * np.eye(n), v)
    x = solve(X, b)
    g = adjoint_gradients(XtXOp(X), mu, x, c, lambda v: solve(X, v))
    h = 1e-5
    for (i, j) in [(0, 0), (5, 3), (29, 11)]:
        E = np.zeros_like(X)
        E[i, j] = h
        fd = (c @ solve(X + E, b) - c @ solve(X - E, b)) / (2 * h)
        assert g["gX"][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_validation_loss_gradients():
    rng = np.random.default_rng(54)
    n, nv = 100, 40
    Xtr = rng.standard_normal((n, 2))
    Xv = rng.standard_normal((nv, 2))
    yv = rng.standard_normal(nv)
    b = rng.standard_normal(n)
    sigma, mu = 1.1, 0.2
    solve = lambda s, m, v: np.linalg.solve(_K(Xtr, s) + m * np.eye(n), v)
    x = solve(sigma, mu, b)
    g = validation_loss_grads(Xtr, Xv, yv, sigma, mu, x, lambda v: solve(sigma, mu, v))
    L = lambda s, m: validation_loss(Xtr, Xv, yv, s, solve(s, m, b))
    assert g["L"] == pytest.approx(L(sigma, mu), rel=1e-12)
    h = 1e-4
    assert g["gmu"] == pytest.approx((L(sigma, mu * (1 + h)) - L(sigma, mu * (1 - h))) / (2 * h * mu), rel=1e-6)
    assert g["gsigma"] == pytest.approx((L(sigma * (1 + h), mu) - L(sigma * (1 - h), mu)) / (2 * h * sigma),
                                        rel=1e-6)


def test_power_estimate_approaches_norm_of_error():
    n, ell = 200, 10
    A = spectrum_psd(np.exp(-np.arange(n) / 5.0), 55)
    r = randomized_nystrom(DenseOp(A), np.random.default_rng(56).standard_normal((n, ell)))
    E = np.linalg.norm(A - (r["U"] * r["lam"]) @ r["U"].T, 2)
    est = rand_pow_err_est(DenseOp(A), r["U"], r["lam"], 60, np.random.default_rng(57).standard_normal(n))
    assert est <= E * (1 + 1e-12)
    assert est >= 0.99 * E


def load_philox_kat():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


def test_philox_known_answers():
    kat = load_philox_kat()
    assert len(kat) == 3
    for ctr, key, want in kat:
        got = tuple(int(v) for v in philox4x32_10(ctr, key))
        assert got == want


def test_gaussian_philox_is_standard_normal():
    Z = gaussian_philox(12345, 400, 500)
    assert abs(Z.mean()) < 0.01 and abs(Z.var() - 1) < 0.01
    # same seed, a prefix of the rows is the prefix of the matrix
    np.testing.assert_array_equal(gaussian_philox(12345, 3, 500), Z[:3])
    assert not np.allclose(gaussian_philox(12346, 3, 500), Z[:3])
