"""Adaptive rank selection for the Nystrom preconditioner (Section "Adaptive
rank selection": Strategy 1, a posteriori error estimation, and Strategy 2,
monitoring lam_l / mu; Appendix, algorithm "Adaptive Randomized Nystrom
Approximation") in float64.

TEST INFRASTRUCTURE ONLY: see the package docstring.

Steps, in the appendix algorithm's order (l = columns so far, m = size of the
next block, starting with l = 0, m = l0):
  1. Omega0 = randn(n, m); Omega0 = qr(Omega0, 0); Y0 = A Omega0
  2. Omega = [Omega Omega0], Y = [Y Y0]            -- the earlier sketch is reused
  3. nu, Y_nu, C = chol(Omega^T Y_nu), B = Y_nu / C, [U, Sigma] = svd(B, 0),
     Lambda = max(0, Sigma^2 - nu)                  -- steps 4-9 of the base algorithm
  4. E = RandPowErrEst(A, U, Lambda, q)
  5. if the stopping criterion holds: return (U, Lambda)
  6. m <- l, target 2 l (the sketch size doubles); if 2 l > l_max the last block
     has m = l_max - l columns, steps 1-3 run once more and the result is
     returned (no estimate of it is made).

Readings where the pseudocode is loose:
  * the criterion is tested right after the estimate, so the doubling lines run
    only when it fails (their comment says they are for that case; run
    literally they would also extend a sketch that already meets it);
  * criterion "err": E <= tau mu (the pseudocode's Tol = tau mu); "err_lam":
    E <= tau mu and lam_l <= tau mu / 11 (the second condition of the text,
    used by the theorem on the final sketch size); "ratio": Strategy 2,
    lam_l <= tau mu, with no power estimate;
  * nu defaults to the base algorithm's eps(||Y||_F); shift="ada" selects the
    appendix's sqrt(n) eps(||Y||_2);
  * when l already equals l_max no block of zero columns is drawn;
  * random draws are inputs: draw_block(j, m) returns the j-th Gaussian block
    (n x m), draw_g(j) the start vector of the j-th estimate.
"""
from __future__ import annotations

import numpy as np

from .nystrom import nystrom_factor, orthonormalize
from .power import rand_pow_err_est


def ada_rand_nystrom(op, l0: int, lmax: int, q: int, tau: float, mu: float, draw_block, draw_g,
                     criterion: str = "err", shift: str = "fro") -> dict:
    """Returns U, lam, nu, ell, E (nan when the last approximation was not
    estimated), capped (l_max reached without the criterion holding) and the
    history [(l, E, lam_l), ...] of every factored stage."""
    if criterion not in ("err", "err_lam", "ratio"):
        raise ValueError(criterion)
    if not 1 <= l0 <= lmax:
        raise ValueError("need 1 <= l0 <= lmax")
    tol = tau * mu
    Omega = None
    Y = None
    m = l0
    j = 0
    history = []
    while True:
        # steps 1-2
        Om0 = orthonormalize(draw_block(j, m))
        Y0 = op.matmat(Om0)
        Omega = Om0 if Omega is None else np.hstack([Omega, Om0])
        Y = Y0 if Y is None else np.hstack([Y, Y0])
        # step 3
        r = nystrom_factor(Omega, Y, shift=shift)
        ell = Omega.shape[1]
        lam_l = float(r["lam"][-1])
        # steps 4-5
        if criterion == "ratio":
            E = float("nan")
            ok = lam_l <= tol
        else:
            E = rand_pow_err_est(op, r["U"], r["lam"], q, draw_g(j))
            ok = E <= tol and (criterion == "err" or lam_l <= tol / 11.0)
        history.append((ell, E, lam_l))
        j += 1
        if ok:
            return dict(U=r["U"], lam=r["lam"], nu=r["nu"], ell=ell, E=E, capped=False, history=history)
        # step 6
        m = ell
        if 2 * ell > lmax:
            m = lmax - ell
            if m > 0:
                Om0 = orthonormalize(draw_block(j, m))
                Y0 = op.matmat(Om0)
                Omega = np.hstack([Omega, Om0])
                Y = np.hstack([Y, Y0])
                r = nystrom_factor(Omega, Y, shift=shift)
                history.append((Omega.shape[1], float("nan"), float(r["lam"][-1])))
            return dict(U=r["U"], lam=r["lam"], nu=r["nu"], ell=Omega.shape[1], E=float("nan"), capped=True,
                        history=history)


def effective_dimension(eigs: np.ndarray, mu: float) -> float:
    """d_eff(mu) = tr(A (A + mu I)^{-1}) (definition of the effective
    dimension), written with the eigenvalues of A: sum_i lam_i / (lam_i + mu)."""
    eigs = np.asarray(eigs, dtype=np.float64)
    return float(np.sum(eigs / (eigs + mu)))
