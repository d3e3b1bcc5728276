"""Pins for the oracle's operators and randomized Nystrom approximation.

Each check compares against something other than the oracle itself: a library
routine (scipy cdist, numpy spacing, pinv), a closed form, or a property the
paper proves (Lemma "Nystrom properties"; eq. (nys-unstable)).
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import DenseOp, RBFOp, XtXOp, matlab_eps, randomized_nystrom
from workloads import lowrank_psd, spectrum_psd


def test_matlab_eps_closed_form():
    assert matlab_eps(1.0) == 2.0 ** -52
    assert matlab_eps(1000.0) == 2.0 ** -43          # 512 <= 1000 < 1024
    assert matlab_eps(0.5) == 2.0 ** -53
    rng = np.random.default_rng(0)
    for x in 10.0 ** rng.uniform(-30, 30, 200):
        assert matlab_eps(x) == np.spacing(x)


def test_rbf_operator_threaded_blocks_match_cdist():
    """The threaded row-block product (used for full-size residuals) against
    scipy's cdist kernel, with more points than one block so several blocks
    and a ragged last block are evaluated."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((4500, 4))
    sigma = 2.3
    V = rng.standard_normal((4500, 2))
    K = np.exp(-cdist(X, X, "sqeuclidean") / (2 * sigma ** 2))
    np.testing.assert_allclose(RBFOp(X, sigma).matmat(V, workers=4, block=512), K @ V, rtol=1e-12, atol=1e-10)


def test_rbf_operator_matches_cdist():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((300, 5)) * 2
    sigma = 1.7
    K = np.exp(-cdist(X, X, "sqeuclidean") / (2 * sigma ** 2))
    V = rng.standard_normal((300, 3))
    op = RBFOp(X, sigma)
    np.testing.assert_allclose(op.matmat(V), K @ V, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(op.dense(), K, rtol=0, atol=1e-13)
    # dK/dsigma = K * d^2 / sigma^3: compare with a central difference of cdist form
    h = 1e-6
    Kp = np.exp(-cdist(X, X, "sqeuclidean") / (2 * (sigma + h) ** 2))
    Km = np.exp(-cdist(X, X, "sqeuclidean") / (2 * (sigma - h) ** 2))
    np.testing.assert_allclose(op.dsigma_matmat(V), (Kp - Km) @ V / (2 * h), rtol=1e-6, atol=1e-8)


def test_xtx_operator_matches_explicit():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((50, 20)).astype(np.float32)
    op = XtXOp(X, scale=0.5)
    V = rng.standard_normal((20, 4))
    X64 = X.astype(np.float64)
    np.testing.assert_allclose(op.matmat(V), 0.5 * np.einsum("ki,kj,jc->ic", X64, X64, V), rtol=1e-12)


def _decay_case(n=256, seed=3):
    lam = 1.0 / np.arange(1, n + 1) ** 2
    return spectrum_psd(lam, seed), lam


def test_closed_form_nystrom():
    """A_hat = Y (Omega^T Y)^+ Y^T (eq. (nys-unstable)) on a well-conditioned core."""
    A, _ = _decay_case()
    rng = np.random.default_rng(4)
    om = rng.standard_normal((A.shape[0], 12))
    res = randomized_nystrom(DenseOp(A), om)
    Ahat = (res["U"] * res["lam"]) @ res["U"].T
    Y = A @ om
    closed = Y @ np.linalg.pinv(om.T @ Y) @ Y.T
    assert np.linalg.norm(Ahat - closed) <= 1e-9 * np.linalg.norm(closed)


def test_depends_only_on_range():
    """Lemma (Nystrom properties), item 2: the QR step does not change A_hat."""
    A, _ = _decay_case(seed=5)
    om = np.random.default_rng(6).standard_normal((A.shape[0], 20))
    a = randomized_nystrom(DenseOp(A), om, use_qr=True)
    b = randomized_nystrom(DenseOp(A), om, use_qr=False)
    Aa = (a["U"] * a["lam"]) @ a["U"].T
    Ab = (b["U"] * b["lam"]) @ b["U"].T
    assert np.linalg.norm(Aa - Ab) <= 1e-9 * np.linalg.norm(Aa)
    np.testing.assert_allclose(a["Omega"].T @ a["Omega"], np.eye(20), atol=1e-14)


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_lemma_properties(seed):
    """psd, rank <= l, A_hat <= A (Loewner), lambda_j(A_hat) <= lambda_j(A)."""
    n, ell = 200, 30
    lam = np.exp(-np.arange(n) / 15.0)
    A = spectrum_psd(lam, seed)
    om = np.random.default_rng(seed + 100).standard_normal((n, ell))
    r = randomized_nystrom(DenseOp(A), om)
    U, lh = r["U"], r["lam"]
    np.testing.assert_allclose(U.T @ U, np.eye(ell), atol=1e-12)
    assert np.all(lh >= 0) and np.all(np.diff(lh) <= 0)
    Ahat = (U * lh) @ U.T
    tol = 1e-12 * n * np.linalg.norm(A, 2)
    assert np.linalg.eigvalsh(Ahat).min() >= -tol
    assert np.linalg.matrix_rank(Ahat, tol=1e-10) <= ell
    assert np.linalg.eigvalsh(A - Ahat).min() >= -tol
    ea = np.sort(np.linalg.eigvalsh(A))[::-1]
    eh = np.sort(np.linalg.eigvalsh(Ahat))[::-1]
    assert np.all(eh <= ea + tol)


@pytest.mark.parametrize("ell,gate", [(64, 1e-12), (48, 1e-12), (40, 1e-9)])
def test_exact_recovery_low_rank(ell, gate):
    """rank(A) <= l: the Nystrom approximation reproduces A."""
    A = lowrank_psd(512, 40, seed=10)
    om = np.random.default_rng(11).standard_normal((512, ell))
    r = randomized_nystrom(DenseOp(A), om)
    Ahat = (r["U"] * r["lam"]) @ r["U"].T
    assert np.linalg.norm(A - Ahat, 2) <= gate * np.linalg.norm(A, 2)


def test_shift_is_matlab_eps_of_frobenius_norm():
    A, _ = _decay_case(seed=12)
    om = np.random.default_rng(13).standard_normal((A.shape[0], 10))
    r = randomized_nystrom(DenseOp(A), om)
    assert r["nu"] == np.spacing(np.linalg.norm(r["Y"], "fro"))
    r2 = randomized_nystrom(DenseOp(A), om, shift="ada")
    assert r2["nu"] == pytest.approx(np.sqrt(A.shape[0]) * np.spacing(np.linalg.norm(r2["Y"], 2)), rel=1e-15)


@pytest.mark.parametrize("nu", [1e-3, 1e-1])
def test_shifted_steps_match_closed_form(nu):
    """Steps 5-9 with an observable shift: U (Lambda + nu) U^T is the Nystrom
    approximation of A + nu I, i.e. Y_nu (Omega^T Y_nu)^+ Y_nu^T (pinv + eigh)."""
    A, _ = _decay_case(n=150, seed=14)
    om = np.random.default_rng(15).standard_normal((150, 12))
    r = randomized_nystrom(DenseOp(A), om, nu=nu)
    Om = r["Omega"]
    Ynu = A @ Om + nu * Om
    closed = Ynu @ np.linalg.pinv(Om.T @ Ynu) @ Ynu.T
    ev = np.sort(np.linalg.eigvalsh(0.5 * (closed + closed.T)))[::-1][:12]
    np.testing.assert_allclose(r["lam"], np.maximum(0.0, ev - nu), rtol=1e-9, atol=1e-12)
