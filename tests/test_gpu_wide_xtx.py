"""X^T X operators wider than the one-pass product keeps in registers: more
than 8192 columns (float32 16-byte rows) or 4096 (float64), and unaligned rows
past 8192 columns, take the two-pass product (row dots, then column partials);
aligned float64 rows with 4096 < n <= 8192 take the one-pass kernel with
scalar loads.  Products entry by entry against the oracle, and a solve judged
by the oracle's float64 residual."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_02820_amd as nys  # noqa: E402

DEV = "cuda"


def h(t):
    return t.detach().double().cpu().numpy()


def _data(m, n, seed, dtype):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((m, n)) / np.sqrt(m) / np.sqrt(np.arange(1, n + 1))).astype(dtype)
    return X


@pytest.mark.parametrize("m,n,dtype,ld_pad", [(3000, 10000, np.float32, 0), (2000, 6000, np.float64, 0),
                                             (2000, 10000, np.float64, 0), (2500, 9001, np.float32, 0),
                                             (1500, 8200, np.float32, 3)])
def test_wide_products(m, n, dtype, ld_pad):
    X = _data(m, n, 100 + n, dtype)
    Xt = torch.as_tensor(X, device=DEV)
    if ld_pad:  # a leading dimension larger than n (rows not 16-byte aligned)
        big = torch.zeros(m, n + ld_pad, dtype=Xt.dtype, device=DEV)
        big[:, :n] = Xt
        Xt = big[:, :n]
    op = nys.Operator(nys.NYS_OP_XTX, Xt, n) if ld_pad else nys.Operator.xtx(Xt)
    Xd = X.astype(np.float64)
    rng = np.random.default_rng(7)
    for k in (1, 3):
        V = rng.standard_normal((n, k))
        mu = 1e-3
        out = h(nys.nys_op_apply(op, mu, torch.as_tensor(V, device=DEV)))
        ref = oracle.XtXOp(Xd).matmat(V) + mu * V
        scale = np.abs(Xd).T @ (np.abs(Xd) @ np.abs(V)) + mu * np.abs(V)
        assert (np.abs(out - ref) / scale).max() <= 1e-12, (k, (np.abs(out - ref) / scale).max())
    if dtype == np.float32:  # float32 arithmetic, one vector
        v = rng.standard_normal(n).astype(np.float32)
        out = h(nys.nys_op_apply(op, 1e-3, torch.as_tensor(v, device=DEV)))
        vd = v.astype(np.float64)
        ref = oracle.XtXOp(Xd).matmat(vd) + 1e-3 * vd
        scale = np.abs(Xd).T @ (np.abs(Xd) @ np.abs(vd)) + 1e-3 * np.abs(vd)
        assert (np.abs(out - ref) / scale).max() <= 1e-4


def test_wide_refinement_solve():
    """float32 X with 10000 columns: bf16x3 sketch, float32 inner PCG on the
    two-pass product, float64 refinement; the oracle's residual meets 1e-10."""
    m, n = 12000, 10000
    X = _data(m, n, 7, np.float32)
    y = np.random.default_rng(8).standard_normal(m)
    Xd = X.astype(np.float64)
    b = Xd.T @ y
    mu = 1e-4
    op = nys.Operator.xtx(torch.as_tensor(X, device=DEV))
    prec = nys.NYS_PREC_BF16X3_REFINE64
    Om, Y = nys.nys_sketch(op, 300, seed=9, prec=prec)
    P = nys.nys_factor(Om, Y, dtype=torch.float32, prec=prec)
    x, info = nys.nys_pcg_solve(op, P, mu, torch.as_tensor(b, device=DEV), tol=1e-10, maxit=2000, prec=prec,
                                inner_tol=3e-6)
    assert info.status[0] == 0
    assert oracle.true_relres(oracle.XtXOp(Xd), mu, h(x), b) <= 1.02e-10
