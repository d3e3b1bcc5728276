"""Parity of the weighted operator A = X^T D X (the Hessian data term of
approximate cross-validation, logistic weights p (1 - p)) through the C ABI
against the CPU FP64 oracle: the X^T X operator with row weights applied
inside every product (float64 weights in the float64 products), its sketch,
whole Nystrom PCG solves (float64, and float32 data with float32 inner PCG and
float64 refinement), the ragged fallback, the refusals, and the separate
row-folding helper D^{1/2} X with its argument errors.

The oracle receives X and d as drawn.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from workloads import logistic_weights  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_02820_amd as nys  # noqa: E402

DEV = "cuda"


def h(t):
    return t.detach().double().cpu().numpy()


def _case(m=1203, n=301, seed=81, dtype=np.float64, decay=False):
    """Seeded data rows and logistic weights p (1 - p) in [0, 1/4], with every
    17th weight zero (rows that drop out of the Hessian).  decay: column j
    scaled by j^{-1/2}, so the spectrum decays as in the ridge workload."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, n)) / np.sqrt(m)
    if decay:
        X = X / np.sqrt(np.arange(1, n + 1))
    return X.astype(dtype), logistic_weights(m, seed + 1000)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [301, 64])
def test_weight_rows_folds_square_roots(dtype, n):
    """301 columns take the scalar kernel, 64 the 16-byte vector one."""
    X, d = _case(n=n, dtype=dtype)
    Xw = h(nys.nys_weight_rows(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV)))
    # one rounding of sqrt(d_i) to the data type, one of the product
    want = np.sqrt(d).astype(dtype)[:, None] * X
    np.testing.assert_allclose(Xw, want.astype(np.float64), rtol=2.0 ** -52 if dtype == np.float64 else 2.0 ** -23,
                               atol=0.0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [3, 8])
def test_weight_rows_more_rows_than_workgroups(dtype, n):
    """70001 rows: more than the 65536 workgroups the fold launches, so the
    grid strides over the rows; 3 columns take the scalar kernel, 8 the
    16-byte one.  Every row is checked."""
    X, d = _case(m=70001, n=n, seed=83, dtype=dtype)
    Xw = h(nys.nys_weight_rows(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV)))
    want = np.sqrt(d).astype(dtype)[:, None] * X
    np.testing.assert_allclose(Xw, want.astype(np.float64), rtol=2.0 ** -52 if dtype == np.float64 else 2.0 ** -23,
                               atol=0.0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("k", [1, 7])
def test_weighted_products(dtype, k):
    """float64 products: float32 data is promoted exactly and the float64
    weights act between the two products, so each entry is within float64
    rounding of X^T D X V (bound 1e-12 of |X|^T D |X| |V|).  float32 products
    (one vector): weights and sums in float32 (bound 2e-5 of the same)."""
    X, d = _case(dtype=dtype)
    Xd = X.astype(np.float64)
    op = nys.Operator.xtdx(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV), scale=0.5)
    V = np.random.default_rng(82).standard_normal((X.shape[1], k))
    mu = 1e-3
    out = h(nys.nys_op_apply(op, mu, torch.as_tensor(V, device=DEV)))
    ref = oracle.XtDXOp(X, d, 0.5).matmat(V) + mu * V
    scale = 0.5 * np.abs(Xd).T @ (d[:, None] * (np.abs(Xd) @ np.abs(V))) + mu * np.abs(V)
    assert (np.abs(out - ref) / scale).max() <= 1e-12
    if k == 1 and dtype == np.float32:
        v32 = V[:, 0].astype(np.float32)
        out32 = h(nys.nys_op_apply(op, mu, torch.as_tensor(v32, device=DEV)))
        ref32 = oracle.XtDXOp(X, d, 0.5).matmat(v32.astype(np.float64)) + mu * v32
        assert (np.abs(out32 - ref32) / scale[:, 0]).max() <= 2e-5


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_weighted_sketch_entries(prec):
    """Y = X^T D X Omega in float64, float32 and bf16x3 products, entry by entry
    against the oracle with the device's own test matrix (bound c |X|^T D |X|
    |Omega|, c = 1e-12, 5e-5, 1e-4)."""
    X, d = _case(m=1500, n=260, seed=87, dtype=np.float32)
    Xd = X.astype(np.float64)
    op = nys.Operator.xtdx(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV))
    Om, Y = nys.nys_sketch(op, 40, seed=88, prec=prec)
    Om, Y = h(Om), h(Y)
    err = np.abs(Y - oracle.XtDXOp(X, d).matmat(Om))
    scale = np.abs(Xd).T @ (d[:, None] * (np.abs(Xd) @ np.abs(Om)))
    assert (err / scale).max() < {0: 1e-12, 1: 5e-5, 3: 1e-4}[prec], (err / scale).max()


def test_weighted_solve_meets_tolerance_on_oracle_operator():
    """Sketch, factor and Nystrom PCG on float64 data; the oracle's float64
    true residual of X^T D X is below the tolerance."""
    X, d = _case(m=2400, n=520, seed=83, decay=True)
    op = nys.Operator.xtdx(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV))
    b = np.random.default_rng(84).standard_normal(520)
    mu = 1e-5
    Om, Y = nys.nys_sketch(op, 100, seed=85)
    P = nys.nys_factor(Om, Y)
    x, info = nys.nys_pcg_solve(op, P, mu, torch.as_tensor(b, device=DEV), tol=1e-10, maxit=500)
    assert info.status[0] == 0
    ref = oracle.XtDXOp(X, d)
    assert oracle.true_relres(ref, mu, h(x), b) <= 1.01e-10
    # the preconditioner did its work: the oracle's plain CG needs 154
    # iterations here, its Nystrom PCG with the same test matrix 61
    plain = oracle.nystrom_pcg(ref.matmat, b, mu, lambda v: v, tol=1e-10, maxit=2000)
    assert info.iters[0] * 2 <= plain["iters"]


@pytest.mark.parametrize("prec", [2, 3])
def test_weighted_float32_data_refinement_solve(prec):
    """float32 data, float64 weights: float32 (or bf16x3) sketch products,
    float32 inner PCG with the weights rounded to float32, float64 refinement
    residuals with the float64 weights, so the solution meets 1e-10 on the
    oracle's X^T D X itself (not on a rounded copy of it)."""
    X, d = _case(m=3000, n=600, seed=89, dtype=np.float32, decay=True)
    op = nys.Operator.xtdx(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV))
    b = oracle.XtDXOp(X, d).matmat(np.random.default_rng(90).standard_normal(600))
    mu = 1e-4
    Om, Y = nys.nys_sketch(op, 120, seed=91, prec=prec)
    P = nys.nys_factor(Om, Y, dtype=torch.float32, prec=prec)
    x, info = nys.nys_pcg_solve(op, P, mu, torch.as_tensor(b, device=DEV), tol=1e-10, maxit=1000, prec=prec,
                                inner_tol=3e-6)
    assert info.status[0] == 0
    true = oracle.true_relres(oracle.XtDXOp(X, d), mu, h(x), b)
    assert true <= 1.01e-10
    assert abs(true - info.relres[0]) <= 1e-12


def test_weighted_refusals_and_ragged_fallback():
    X, d = _case(m=900, n=150, seed=92)
    Xt = torch.as_tensor(X, device=DEV)
    dt = torch.as_tensor(d, device=DEV)
    op = nys.Operator.xtdx(Xt, dt)
    # column sampling and dL/dX are not formed for weighted operators
    with pytest.raises(nys.NysError) as e:
        nys.nys_sketch_columns(op, torch.arange(10, device=DEV, dtype=torch.int64))
    assert e.value.status == nys.NYS_ERR_ARG
    P = nys.nys_factor(*nys.nys_sketch(op, 30, seed=93))
    b = np.random.default_rng(94).standard_normal(150)
    x, _ = nys.nys_pcg_solve(op, P, 1e-3, torch.as_tensor(b, device=DEV), tol=1e-10, maxit=500)
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_backward(op, P, 1e-3, x, torch.as_tensor(b, device=DEV), want_X=True)
    assert e.value.status == nys.NYS_ERR_ARG
    # weights on a non-X^T X operator are refused
    rop = nys.Operator.rbf(torch.as_tensor(np.random.default_rng(95).standard_normal((150, 4)), device=DEV), 1.0)
    rop.weights = dt[:150].contiguous()
    with pytest.raises(nys.NysError) as e:
        nys.nys_op_apply(rop, 0.0, torch.as_tensor(b, device=DEV))
    assert e.value.status == nys.NYS_ERR_ARG
    # a ragged batch with a weighted problem is solved problem by problem
    X2, d2 = _case(m=700, n=120, seed=96)
    op2 = nys.Operator.xtx(torch.as_tensor(X2, device=DEV))
    P2 = nys.nys_factor(*nys.nys_sketch(op2, 24, seed=97))
    b2 = np.random.default_rng(98).standard_normal(120)
    Xs, info = nys.nys_pcg_solve_ragged([op, op2], [P, P2], [1e-3, 1e-3],
                                        [torch.as_tensor(b, device=DEV), torch.as_tensor(b2, device=DEV)],
                                        tol=1e-10, maxit=500)
    assert info.status == [0, 0]
    assert oracle.true_relres(oracle.XtDXOp(X, d), 1e-3, h(Xs[0]), b) <= 1.01e-10
    assert oracle.true_relres(oracle.XtXOp(X2), 1e-3, h(Xs[1]), b2) <= 1.01e-10


def test_weight_rows_in_place_and_errors():
    X, d = _case(m=300, n=40, seed=86)
    Xt = torch.as_tensor(X, device=DEV)
    dt = torch.as_tensor(d, device=DEV)
    out = nys.nys_weight_rows(Xt, dt, out=Xt)
    assert out.data_ptr() == Xt.data_ptr()
    np.testing.assert_allclose(h(Xt), np.sqrt(d)[:, None] * X, rtol=2.0 ** -52, atol=0.0)
    # a negative or non-finite weight is refused before anything is written
    Xt2 = torch.as_tensor(X, device=DEV)
    for bad in (-1e-3, float("nan"), float("inf")):
        db = d.copy()
        db[123] = bad
        with pytest.raises(nys.NysError) as e:
            nys.nys_weight_rows(Xt2, torch.as_tensor(db, device=DEV), out=Xt2)
        assert e.value.status == nys.NYS_ERR_ARG
        np.testing.assert_array_equal(h(Xt2), X)
    with pytest.raises(ValueError):
        nys.nys_weight_rows(Xt2, torch.as_tensor(d[:-1], device=DEV))
