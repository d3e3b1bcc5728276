"""Pins of the oracle's Nystrom sketch-and-solve against facts fixed
independently of its code."""
import math

import numpy as np
import pytest

from oracle import DenseOp, effective_dimension, nystrom_sketch_solve, randomized_nystrom
from workloads import lowrank_psd, spectrum_psd


def test_equals_a_dense_solve_of_the_proxy_system():
    rng = np.random.default_rng(1)
    n, ell, mu = 80, 12, 0.03
    U, _ = np.linalg.qr(rng.standard_normal((n, ell)))
    lam = np.sort(rng.uniform(0.1, 5.0, ell))[::-1]
    B = rng.standard_normal((n, 3))
    want = np.linalg.solve((U * lam) @ U.T + mu * np.eye(n), B)
    np.testing.assert_allclose(nystrom_sketch_solve(U, lam, mu, B), want, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(nystrom_sketch_solve(U, lam, mu, B[:, 0]), want[:, 0], rtol=1e-12, atol=1e-12)
    with pytest.raises(ValueError):
        nystrom_sketch_solve(U, lam, 0.0, B)


def test_exact_when_the_approximation_is_exact():
    A = lowrank_psd(100, 8, 2)
    r = randomized_nystrom(DenseOp(A), np.random.default_rng(3).standard_normal((100, 10)))
    b = np.random.default_rng(4).standard_normal(100)
    mu = 1e-2
    x = nystrom_sketch_solve(r["U"], r["lam"], mu, b)
    xs = np.linalg.solve(A + mu * np.eye(100), b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_expected_relative_error_bound():
    """Theorem on sketch-and-solve: with l = 2 ceil(1.5 d_eff(eps mu)) + 1 the
    expected relative error is at most 26 eps (mean over 10 seeds)."""
    n = 300
    eigs = np.exp(-np.arange(n) / 6.0)
    A = spectrum_psd(eigs, 5)
    mu, eps = 1e-2, 0.05
    ell = 2 * math.ceil(1.5 * effective_dimension(eigs, eps * mu)) + 1
    b = np.random.default_rng(6).standard_normal(n)
    xs = np.linalg.solve(A + mu * np.eye(n), b)
    errs = []
    for seed in range(10):
        r = randomized_nystrom(DenseOp(A), np.random.default_rng(100 + seed).standard_normal((n, ell)))
        errs.append(np.linalg.norm(nystrom_sketch_solve(r["U"], r["lam"], mu, b) - xs) / np.linalg.norm(xs))
    assert np.mean(errs) <= 26 * eps
    # and a rank well below the prescription leaves a large error
    r = randomized_nystrom(DenseOp(A), np.random.default_rng(7).standard_normal((n, 4)))
    assert np.linalg.norm(nystrom_sketch_solve(r["U"], r["lam"], mu, b) - xs) / np.linalg.norm(xs) > eps
