"""Parity of the weighted operator A = X^T D X (the Hessian data term of
approximate cross-validation, logistic weights p (1 - p)) through the C ABI
against the CPU FP64 oracle: the folded data D^{1/2} X, products, a whole
Nystrom PCG solve, and the argument errors.

The oracle receives X and d as drawn; it never sees the folded data.
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


@pytest.mark.parametrize("dtype,bound", [(np.float64, 1e-12), (np.float32, 1e-6)])
@pytest.mark.parametrize("k", [1, 7])
def test_weighted_products(dtype, bound, k):
    """float64 data: rounding of the float64 products.  float32 data: the
    folded entries carry two float32 roundings (2^-23 relative), which bound
    the operator's relative difference from X^T D X by about 2.4e-7."""
    X, d = _case(dtype=dtype)
    op = nys.Operator.xtdx(torch.as_tensor(X, device=DEV), torch.as_tensor(d, device=DEV), scale=0.5)
    V = np.random.default_rng(82).standard_normal((X.shape[1], k))
    mu = 1e-3
    out = h(nys.nys_op_apply(op, mu, torch.as_tensor(V, device=DEV)))
    ref = oracle.XtDXOp(X, d, 0.5).matmat(V) + mu * V
    assert np.linalg.norm(out - ref) <= bound * np.linalg.norm(ref)


def test_weighted_solve_meets_tolerance_on_oracle_operator():
    """Sketch, factor and Nystrom PCG on the folded float64 data; the oracle's
    float64 true residual of X^T D X is below the tolerance."""
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
