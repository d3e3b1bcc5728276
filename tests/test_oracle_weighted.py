"""Pins of the weighted operator A = scale X^T D X of the oracle against
definitions it does not share code with: the sum over rows of d_i x_i x_i^T
written as a loop, the unweighted operator for d = 1, and the rank-one
matrix x_k x_k^T for a one-hot weight vector."""
import numpy as np

from oracle import XtDXOp, XtXOp


def _data(seed=3, m=37, n=11):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, n))
    d = rng.uniform(0.0, 0.25, m)  # logistic weights p (1 - p) lie in [0, 1/4]
    return X, d


def test_weighted_matches_row_sum():
    X, d = _data()
    A = np.zeros((X.shape[1], X.shape[1]))
    for i in range(X.shape[0]):
        A += d[i] * np.outer(X[i], X[i])
    V = np.random.default_rng(4).standard_normal((X.shape[1], 3))
    op = XtDXOp(X, d, scale=0.5)
    np.testing.assert_allclose(op.matmat(V), 0.5 * A @ V, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(op.matmat(V[:, 0]), 0.5 * A @ V[:, 0], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(op.dense(), 0.5 * A, rtol=1e-13, atol=1e-13)


def test_unit_weights_reduce_to_normal_equations():
    X, _ = _data(5)
    V = np.random.default_rng(6).standard_normal((X.shape[1], 2))
    np.testing.assert_allclose(XtDXOp(X, np.ones(X.shape[0])).matmat(V), XtXOp(X).matmat(V), rtol=1e-14,
                               atol=1e-14)


def test_one_hot_weight_is_rank_one_and_psd():
    X, d = _data(7)
    e = np.zeros(X.shape[0])
    e[4] = 2.0
    np.testing.assert_allclose(XtDXOp(X, e).dense(), 2.0 * np.outer(X[4], X[4]), rtol=1e-14, atol=1e-14)
    w = np.linalg.eigvalsh(XtDXOp(X, d).dense())
    assert w.min() >= -1e-13 * w.max()
