"""Pins of the oracle's adaptive rank selection (Section "Adaptive rank
selection", Strategies 1 and 2; Appendix, algorithm "Adaptive Randomized
Nystrom Approximation") against facts fixed independently of its code."""
import math

import numpy as np
import pytest

from oracle import DenseOp, ada_rand_nystrom, effective_dimension, orthonormalize, randomized_nystrom
from workloads import spectrum_psd


def _draws(n, seed):
    blocks = {}

    def draw_block(j, m):
        blocks[j] = np.random.default_rng(seed * 1000 + 2 * j).standard_normal((n, m))
        return blocks[j]

    def draw_g(j):
        return np.random.default_rng(seed * 1000 + 2 * j + 1).standard_normal(n)

    return draw_block, draw_g, blocks


def _approx(r):
    return (r["U"] * r["lam"]) @ r["U"].T


def _decay_matrix(n=160, rate=8.0, seed=3):
    eigs = np.exp(-np.arange(n) / rate)
    return spectrum_psd(eigs, seed), eigs


def test_no_doubling_is_the_base_algorithm():
    A, _ = _decay_matrix()
    db, dg, blocks = _draws(A.shape[0], 1)
    r = ada_rand_nystrom(DenseOp(A), 12, 12, 20, 1e-30, 1.0, db, dg)
    base = randomized_nystrom(DenseOp(A), blocks[0])
    assert r["ell"] == 12 and r["capped"]
    assert np.allclose(_approx(r), _approx(base), rtol=0, atol=1e-14)


def test_concatenated_sketch_is_the_closed_form_on_the_joint_range():
    """After one doubling the approximation is A W (W^T A W)^{-1} W^T A for
    W = [Omega1 Omega2] (eq. (nys-unstable)); it depends only on range(W)."""
    A, _ = _decay_matrix(n=120, rate=30.0)
    db, dg, blocks = _draws(A.shape[0], 2)
    r = ada_rand_nystrom(DenseOp(A), 10, 20, 20, 1e-30, 1.0, db, dg)
    assert r["ell"] == 20 and [h[0] for h in r["history"]] == [10, 20]
    W = np.hstack([orthonormalize(blocks[0]), orthonormalize(blocks[1])])
    AW = A @ W
    closed = AW @ np.linalg.solve(W.T @ AW, AW.T)
    assert np.linalg.norm(_approx(r) - closed, 2) <= 1e-9 * np.linalg.norm(A, 2)
    # and it differs from the approximation of the first block alone
    first = AW[:, :10] @ np.linalg.solve(W[:, :10].T @ AW[:, :10], AW[:, :10].T)
    assert np.linalg.norm(first - closed, 2) > 1e-6


def test_stops_at_the_first_stage_whose_exact_error_meets_the_tolerance():
    A, _ = _decay_matrix(n=200, rate=10.0, seed=5)
    n = A.shape[0]
    db, dg, blocks = _draws(n, 3)
    mu = 1e-3
    # exact ||E|| of each doubling stage, from the concatenated blocks
    r_all = ada_rand_nystrom(DenseOp(A), 8, 128, 80, 1e-30, mu, db, dg)
    stages = [h[0] for h in r_all["history"]]
    assert stages == [8, 16, 32, 64, 128]
    W = np.hstack([orthonormalize(blocks[j]) for j in range(len(stages))])
    exact = []
    for l in stages:
        AW = A @ W[:, :l]
        Ahat = AW @ np.linalg.solve(W[:, :l].T @ AW, AW.T)
        exact.append(np.linalg.norm(A - Ahat, 2))
    assert all(a > b for a, b in zip(exact, exact[1:]))
    # the estimates are Rayleigh quotients of E: below ||E||, and close after 80 steps
    for (l, E, _), ex in zip(r_all["history"], exact):
        assert E <= ex * (1 + 1e-9) and E >= 0.95 * ex
    # tolerance between the exact errors of stages 3 and 4 (32 and 64 columns)
    tau = math.sqrt(exact[2] * exact[3]) / mu
    db, dg, _ = _draws(n, 3)
    r = ada_rand_nystrom(DenseOp(A), 8, 128, 80, tau, mu, db, dg)
    assert r["ell"] == 64 and not r["capped"]
    assert r["E"] <= tau * mu


def test_cap_at_lmax_that_is_not_a_doubling_stage():
    A, _ = _decay_matrix(n=150, rate=40.0)
    db, dg, _ = _draws(A.shape[0], 4)
    r = ada_rand_nystrom(DenseOp(A), 10, 70, 10, 1e-30, 1e-3, db, dg)
    assert [h[0] for h in r["history"]] == [10, 20, 40, 70]
    assert r["ell"] == 70 and r["capped"] and math.isnan(r["E"])
    assert r["U"].shape == (150, 70)
    assert np.allclose(r["U"].T @ r["U"], np.eye(70), atol=1e-12)


def test_strategy2_stops_when_lam_l_over_mu_meets_the_tolerance():
    A, _ = _decay_matrix(n=180, rate=12.0, seed=7)
    db, dg, _ = _draws(A.shape[0], 5)
    mu, tau = 1e-4, 10.0
    r = ada_rand_nystrom(DenseOp(A), 8, 160, 0, tau, mu, db, dg, criterion="ratio")
    lam_ls = [h[2] for h in r["history"]]
    assert lam_ls[-1] <= tau * mu and all(v > tau * mu for v in lam_ls[:-1])
    # lam_l of a rank-l Nystrom approximation is at most the l-th eigenvalue of A
    eigs = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert lam_ls[-1] <= eigs[r["ell"] - 1] * (1 + 1e-10)


def test_final_sketch_size_bound_of_the_theorem():
    """Corollary of the theorem on adaptive rank selection (tau = 44, delta =
    1/4): with probability >= 3/4 the final l <= 4 ceil(2 d_eff(mu)) + 2 and
    the sketch size doubles at most ceil(log2(l_tilde / l0)) times, l_tilde =
    2 ceil(2 d_eff(mu)) + 1.  Checked as a frequency over 12 seeds."""
    n = 300
    eigs = 1.0 / (1.0 + np.arange(n)) ** 2
    A = spectrum_psd(eigs, 11)
    mu, tau, l0 = 1e-3, 44.0, 4
    deff = effective_dimension(eigs, mu)
    bound = 4 * math.ceil(2 * deff) + 2
    l_tilde = 2 * math.ceil(2 * deff) + 1
    max_doublings = math.ceil(math.log2(l_tilde / l0))
    ok = 0
    for seed in range(12):
        db, dg, _ = _draws(n, 100 + seed)
        r = ada_rand_nystrom(DenseOp(A), l0, n, 10, tau, mu, db, dg, criterion="err_lam")
        doublings = len(r["history"]) - 1
        ok += r["ell"] <= bound and doublings <= max_doublings and not r["capped"]
    assert ok >= 9


def test_effective_dimension_is_the_trace_formula():
    A, eigs = _decay_matrix(n=50, rate=5.0)
    mu = 0.01
    assert effective_dimension(eigs, mu) == pytest.approx(np.trace(A @ np.linalg.inv(A + mu * np.eye(50))),
                                                           rel=1e-10)
