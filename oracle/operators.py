"""Operators A for the regularised system (A + mu I) x = b, in float64.

A is symmetric psd and is reached only through products A V (Section 1.1:
the method touches A through matvecs).  Three forms:

* DenseOp  -- an explicit symmetric n x n matrix.
* XtXOp    -- ridge normal equations, A = scale * X^T X for data X (m x n)
              (Section 1.3, eq. (RidgeRegression); scale absorbs the 1/n factor).
* XtDXOp   -- weighted normal equations, A = scale * X^T D X with D = diag(d),
              d >= 0: the data term of the Hessian of a regularised
              generalised linear model (logistic weights p (1 - p)), the
              operator of approximate leave-one-out cross-validation
              (Section 6.3, "Approximate cross-validation").
* RBFOp    -- Gaussian kernel matrix K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2))
              for points x_i (rows of X, n x d) (Section 6.5, kernel ridge
              regression).  K is never stored whole; row blocks are formed on
              demand.

Stored float32 data is promoted exactly to float64, so the oracle and a device
path reading the same float32 array define the identical matrix A.
"""
from __future__ import annotations

import numpy as np

_BLOCK = 2048


class DenseOp:
    def __init__(self, A: np.ndarray):
        self.A = np.asarray(A, dtype=np.float64)
        self.n = self.A.shape[0]

    def matmat(self, V: np.ndarray) -> np.ndarray:
        return self.A @ V

    def dense(self) -> np.ndarray:
        return self.A


class XtXOp:
    def __init__(self, X: np.ndarray, scale: float = 1.0):
        self.X = np.asarray(X, dtype=np.float64)
        self.scale = float(scale)
        self.n = self.X.shape[1]

    def matmat(self, V: np.ndarray) -> np.ndarray:
        # A V = scale * X^T (X V): two products, no n x n matrix is formed.
        return self.scale * (self.X.T @ (self.X @ V))

    def dense(self) -> np.ndarray:
        return self.scale * (self.X.T @ self.X)


class XtDXOp:
    def __init__(self, X: np.ndarray, d: np.ndarray, scale: float = 1.0):
        self.X = np.asarray(X, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)
        self.scale = float(scale)
        self.n = self.X.shape[1]

    def matmat(self, V: np.ndarray) -> np.ndarray:
        # A V = scale * X^T (D (X V)): the diagonal weights act between the
        # two products.
        XV = self.X @ V
        DXV = self.d[:, None] * XV if XV.ndim == 2 else self.d * XV
        return self.scale * (self.X.T @ DXV)

    def dense(self) -> np.ndarray:
        return self.scale * (self.X.T @ (self.d[:, None] * self.X))


def rbf_kernel_block(Xr: np.ndarray, Xc: np.ndarray, sigma: float) -> np.ndarray:
    """K(Xr, Xc) with entries exp(-||x - y||^2 / (2 sigma^2)).

    The squared distance is expanded as ||x||^2 + ||y||^2 - 2 x^T y (exact
    identity) and clipped at 0, since a squared distance is never negative.
    """
    Xr = np.asarray(Xr, dtype=np.float64)
    Xc = np.asarray(Xc, dtype=np.float64)
    d2 = (Xr * Xr).sum(1)[:, None] + (Xc * Xc).sum(1)[None, :] - 2.0 * (Xr @ Xc.T)
    np.maximum(d2, 0.0, out=d2)
    return np.exp(-d2 / (2.0 * sigma * sigma))


class RBFOp:
    def __init__(self, X: np.ndarray, sigma: float):
        self.X = np.asarray(X, dtype=np.float64)
        self.sigma = float(sigma)
        self.n = self.X.shape[0]

    def rows(self, idx) -> np.ndarray:
        return rbf_kernel_block(self.X[idx], self.X, self.sigma)

    def matmat(self, V: np.ndarray, workers: int = 1, block: int = _BLOCK) -> np.ndarray:
        """K V by row blocks.  workers > 1 evaluates the independent row blocks
        on that many threads: the same formula per block, with one BLAS thread
        per block (so sums inside a block may be ordered differently)."""
        V = np.asarray(V, dtype=np.float64)
        out = np.empty((self.n,) + V.shape[1:], dtype=np.float64)

        def one(i):
            out[i:i + block] = rbf_kernel_block(self.X[i:i + block], self.X, self.sigma) @ V

        starts = range(0, self.n, block)
        if workers <= 1:
            for i in starts:
                one(i)
        else:
            from concurrent.futures import ThreadPoolExecutor
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(workers) as ex:
                list(ex.map(one, starts))
        return out

    def dense(self) -> np.ndarray:
        return rbf_kernel_block(self.X, self.X, self.sigma)

    def dsigma_matmat(self, V: np.ndarray) -> np.ndarray:
        """(dK/dsigma) V with dK_ij/dsigma = K_ij ||x_i - x_j||^2 / sigma^3."""
        V = np.asarray(V, dtype=np.float64)
        out = np.empty((self.n,) + V.shape[1:], dtype=np.float64)
        s = self.sigma
        for i in range(0, self.n, _BLOCK):
            Xr = self.X[i:i + _BLOCK]
            d2 = (Xr * Xr).sum(1)[:, None] + (self.X * self.X).sum(1)[None, :] - 2.0 * (Xr @ self.X.T)
            np.maximum(d2, 0.0, out=d2)
            out[i:i + _BLOCK] = (np.exp(-d2 / (2 * s * s)) * d2 / s ** 3) @ V
        return out
