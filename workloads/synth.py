"""Random draws for each workload (see the package docstring for the rules).

All generators use ``numpy.random.default_rng(seed)`` and draw in the order
listed in each function, so a recipe is reproducible from its seed alone.
"""
from __future__ import annotations

import numpy as np


def gaussian_test_matrix(n: int, ell: int, seed: int) -> np.ndarray:
    """Standard normal n x ell test matrix (row-major, float64)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, ell))


def column_sample(n: int, ell: int, seed: int) -> np.ndarray:
    """ell distinct column indices drawn uniformly from 0..n-1 (int64)."""
    rng = np.random.default_rng(seed)
    return rng.choice(n, size=ell, replace=False).astype(np.int64)


def krr_small(n: int = 2048, d: int = 8, ell: int = 100, seed: int = 20211001) -> dict:
    """Kernel ridge regression, small: points i.i.d. N(0, I_d), sigma = sqrt(d).

    Draw order: X (n x d), w (n), eps (n), Omega0 (n x ell).
    The right-hand side is b = K w + 0.01 eps with K the RBF kernel matrix.
    """
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    w = rng.standard_normal(n)
    eps = rng.standard_normal(n)
    omega0 = rng.standard_normal((n, ell))
    return dict(kind="rbf", X=X, sigma=float(np.sqrt(d)), mu=1e-3, ell=ell,
                w=w, eps=eps, noise=0.01, omega0=omega0, tol=1e-10)


def ridge_dense(m: int = 20000, n: int = 4000, ell: int = 500, seed: int = 20211002,
                with_omega: bool = True) -> dict:
    """Dense ridge regression: X = G diag(j^-1/2) stored as float32, G ~ N(0, 1/m).

    Draw order: G (m x n), y (m), Omega0 (n x ell).
    The system is (X^T X + mu I) x = X^T y with X the stored float32 matrix.
    """
    rng = np.random.default_rng(seed)
    X = np.empty((m, n), dtype=np.float32)
    colscale = 1.0 / np.sqrt(np.arange(1, n + 1, dtype=np.float64))
    step = 2048
    inv = 1.0 / np.sqrt(m)
    for i in range(0, m, step):
        g = rng.standard_normal((min(step, m - i), n))
        X[i:i + g.shape[0]] = (g * inv * colscale).astype(np.float32)
    y = rng.standard_normal(m)
    omega0 = rng.standard_normal((n, ell)) if with_omega else None
    return dict(kind="xtx", X=X, mu=1e-4, ell=ell, y=y, omega0=omega0, tol=1e-10)


def logistic_weights(m: int, seed: int = 20211007, zero_every: int = 17) -> np.ndarray:
    """Hessian weights of a logistic model, d_i = p_i (1 - p_i) in [0, 1/4],
    with p_i = 1 / (1 + exp(-2 z_i)), z ~ N(0, 1) (a fitted model's spread of
    confidences); every zero_every-th weight is 0 (points the model fits with
    certainty), 0 for none."""
    z = np.random.default_rng(seed).standard_normal(m)
    p = 1.0 / (1.0 + np.exp(-2.0 * z))
    d = p * (1.0 - p)
    if zero_every > 0:
        d[::zero_every] = 0.0
    return d


def _mixture(rng, n: int, d: int, k: int = 10):
    means = 2.0 * rng.standard_normal((k, d))
    lab = rng.integers(0, k, n)
    X = means[lab] + rng.standard_normal((n, d))
    return means, lab, X


def krr_mixture(n: int = 100000, d: int = 32, ell: int = 1000, seed: int = 20211003,
                with_omega: bool = True) -> dict:
    """Kernel ridge regression on a 10-component Gaussian mixture.

    Means ~ N(0, 4 I), unit covariance, equal weights; X stored float32;
    sigma = sqrt(d); mu = 1e-6 n.  Draw order: means, labels, X, w, eps, Omega0.
    b = K w + 0.01 eps.
    """
    rng = np.random.default_rng(seed)
    _, _, X = _mixture(rng, n, d)
    X = X.astype(np.float32)
    w = rng.standard_normal(n)
    eps = rng.standard_normal(n)
    omega0 = rng.standard_normal((n, ell)) if with_omega else None
    return dict(kind="rbf", X=X, sigma=float(np.sqrt(d)), mu=1e-6 * n, ell=ell,
                w=w, eps=eps, noise=0.01, omega0=omega0, tol=1e-10)


def batched_cv(n: int = 50000, d: int = 16, ell: int = 800, nmu: int = 32, nrhs: int = 8,
               nprob: int = 64, mrange=(1000, 20001), seed: int = 20211004,
               with_omega: bool = True, with_ragged: bool = True) -> dict:
    """Batched cross-validation: one RBF system, a mu grid and several right-hand
    sides, plus a ragged list of independent ridge problems.

    RBF part: mixture law of ``krr_mixture`` at dimension d, sigma = 4,
    mu_k = n 10^(-8 + 6k/(nmu-1)), B ~ N(0,1) n x nrhs.
    Ragged part (k = 0..nprob-1): m_k ~ U{mrange}, N_k = m_k // 4,
    X_k = N(0, 1/m_k) diag(j^-1/2) as float32, y_k ~ N(0,1), b_k = X_k^T y_k,
    mu = 1e-4, ell_k = 16 ceil(N_k / 128).
    Draw order: means, labels, X, B, Omega0, then per problem (m_k, X_k, y_k, Omega0_k).
    """
    rng = np.random.default_rng(seed)
    _, _, X = _mixture(rng, n, d)
    X = X.astype(np.float32)
    B = rng.standard_normal((n, nrhs))
    omega0 = rng.standard_normal((n, ell)) if with_omega else None
    mus = n * 10.0 ** (-8.0 + 6.0 * np.arange(nmu) / max(nmu - 1, 1))
    probs = []
    if with_ragged:
        for _ in range(nprob):
            mk = int(rng.integers(mrange[0], mrange[1]))
            nk = mk // 4
            cs = 1.0 / np.sqrt(np.arange(1, nk + 1, dtype=np.float64))
            Xk = (rng.standard_normal((mk, nk)) / np.sqrt(mk) * cs).astype(np.float32)
            yk = rng.standard_normal(mk)
            ellk = int(16 * -(-nk // 128))
            om = rng.standard_normal((nk, ellk)) if with_omega else None
            probs.append(dict(kind="xtx", X=Xk, y=yk, mu=1e-4, ell=ellk, omega0=om))
    return dict(kind="rbf", X=X, sigma=4.0, mus=mus, B=B, ell=ell, omega0=omega0,
                ragged=probs, tol=1e-10)


def differentiation(n: int = 100000, nval: int = 10000, d: int = 16, ell: int = 1000,
                    seed: int = 20211005, with_omega: bool = True) -> dict:
    """Differentiation workload: RBF system on a mixture (d = 16, sigma = 4, mu = 0.1)
    and a validation set from the same means.

    Draw order: means, labels, X_tr, labels_val, X_val, w, eps, eps_val, Omega0.
    b = K_tr w + 0.01 eps;  y_val = K_val,tr w + 0.01 eps_val.
    """
    rng = np.random.default_rng(seed)
    means, _, Xtr = _mixture(rng, n, d)
    lab_v = rng.integers(0, means.shape[0], nval)
    Xval = means[lab_v] + rng.standard_normal((nval, d))
    w = rng.standard_normal(n)
    eps = rng.standard_normal(n)
    eps_val = rng.standard_normal(nval)
    omega0 = rng.standard_normal((n, ell)) if with_omega else None
    return dict(kind="rbf", X=Xtr.astype(np.float32), Xval=Xval.astype(np.float32),
                sigma=4.0, mu=0.1, ell=ell, w=w, eps=eps, eps_val=eps_val, noise=0.01,
                omega0=omega0, tol=1e-10)


def spectrum_psd(lam: np.ndarray, seed: int) -> np.ndarray:
    """Symmetric psd test matrix Q diag(lam) Q^T with a Haar-random orthogonal Q."""
    rng = np.random.default_rng(seed)
    n = lam.shape[0]
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    q = q * np.sign(np.diag(r))
    A = (q * lam) @ q.T
    return 0.5 * (A + A.T)


def lowrank_psd(n: int, rank: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Exactly low-rank psd test matrix G G^T with G ~ N(0, scale^2) of size n x rank."""
    rng = np.random.default_rng(seed)
    G = scale * rng.standard_normal((n, rank))
    return G @ G.T
