"""Randomized Nystrom approximation (Algorithm "Randomized Nystrom Approximation",
Section 2.2) in float64.

Steps, in the algorithm's order and notation:
  1. Omega = randn(n, l)                     -- the Gaussian test matrix is an input
                                                 (``omega0``); random draws are passed in.
  2. Omega = qr(Omega, 0)                    -- keep the orthonormal factor Q.
  3. Y = A Omega                             -- l matvecs.
  4. nu = eps(norm(Y, 'fro'))                -- MATLAB eps: spacing of the number.
  5. Y_nu = Y + nu Omega                     -- shift for stability.
  6. C = chol(Omega^T Y_nu)                  -- upper factor, C^T C = Omega^T Y_nu.
  7. B = Y_nu / C                            -- B = Y_nu C^{-1}.
  8. [U, Sigma, ~] = svd(B, 0)               -- thin SVD, singular values descending.
  9. Lambda = max(0, Sigma^2 - nu)           -- remove the shift.

Readings where the paper is silent or ambiguous:
  * step 2 returns the Q factor (the approximation depends only on range(Omega),
    Lemma "Nystrom properties", item 2), so Q is the meaningful output;
  * the core matrix Omega^T Y_nu is symmetric in exact arithmetic; its upper
    triangle is used (as chol does), i.e. it is symmetrised first;
  * a failed Cholesky is retried with nu <- 10 nu, at most three times;
  * ``shift="ada"`` selects the shift of the adaptive variant (Appendix,
    algorithm "Adaptive Randomized Nystrom Approximation"):
    nu = sqrt(n) eps(norm(Y, 2)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def orthonormalize(omega0: np.ndarray) -> np.ndarray:
    """Thin QR of the test matrix; returns the n x l orthonormal factor."""
    q, _ = np.linalg.qr(np.asarray(omega0, dtype=np.float64), mode="reduced")
    return q


def matlab_eps(x: float) -> float:
    """Distance from |x| to the next larger float64 (MATLAB ``eps(x)``):
    2^(e - 52) where |x| = f 2^e with 1 <= f < 2."""
    x = abs(float(x))
    if x == 0.0:
        return 2.0 ** -1074
    _, e = np.frexp(x)          # x = m 2^e with 0.5 <= m < 1
    return float(np.ldexp(1.0, int(e) - 53))


class NotPSD(Exception):
    pass


def randomized_nystrom(op, omega0: np.ndarray, shift: str = "fro", use_qr: bool = True,
                       max_retry: int = 3, nu=None) -> dict:
    """Run the randomized Nystrom approximation.  Returns U (n x l, orthonormal
    columns), lam (l, descending, >= 0), nu, and the intermediates Omega, Y.
    ``nu`` fixes the shift instead of computing it (used by tests that make the
    shift large enough to observe)."""
    Omega = orthonormalize(omega0) if use_qr else np.asarray(omega0, dtype=np.float64)
    Y = op.matmat(Omega)
    return nystrom_factor(Omega, Y, shift=shift, max_retry=max_retry, nu=nu)


def nystrom_factor(Omega: np.ndarray, Y: np.ndarray, shift: str = "fro", max_retry: int = 3, nu=None) -> dict:
    """Steps 4-9 of the algorithm on a given test matrix Omega and sketch
    Y = A Omega (the adaptive variant calls them on concatenated sketches)."""
    n = Omega.shape[0]
    if nu is not None:
        nu = float(nu)
    elif shift == "fro":
        nu = matlab_eps(np.linalg.norm(Y, "fro"))
    elif shift == "ada":
        nu = np.sqrt(n) * matlab_eps(np.linalg.norm(Y, 2))
    else:
        raise ValueError(shift)
    for _ in range(max_retry + 1):
        Ynu = Y + nu * Omega
        M = Omega.T @ Ynu
        M = 0.5 * (M + M.T)
        try:
            C = sla.cholesky(M, lower=False)
            break
        except np.linalg.LinAlgError:
            nu *= 10.0
    else:
        raise NotPSD("Cholesky of Omega^T Y_nu failed after shift retries")
    # B = Y_nu C^{-1}  <=>  C^T B^T = Y_nu^T
    B = sla.solve_triangular(C, Ynu.T, trans="T", lower=False).T
    U, S, _ = np.linalg.svd(B, full_matrices=False)
    lam = np.maximum(0.0, S * S - nu)
    return dict(U=U, lam=lam, nu=nu, Omega=Omega, Y=Y, B=B, C=C)
