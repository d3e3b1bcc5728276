"""Parity of the coupled block PCG (through the C ABI) against the CPU FP64
oracle: the block iterates after a fixed number of steps (the block Galerkin
solutions, identical in exact arithmetic whatever basis the QR picks), the
iteration count to a tolerance, and the converged solution."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from workloads import krr_small, ridge_dense  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_02820_amd as nys  # noqa: E402

DEV = "cuda"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _rbf_case(n=600, ell=40, seed=61, sigma=1.6):
    w = krr_small(n=n, d=6, ell=ell, seed=seed)
    ref = oracle.RBFOp(w["X"], sigma)
    r = oracle.randomized_nystrom(ref, w["omega0"])
    op = nys.Operator.rbf(dev(w["X"]), sigma)
    return ref, r, op


@pytest.mark.parametrize("s", [1, 3, 8])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_block_iterates_match_oracle(s, k):
    ref, r, op = _rbf_case()
    mu = 1e-3
    Pi = lambda R: oracle.precond_inv_apply(r["U"], r["lam"], mu, R)
    B = np.random.default_rng(62 + s).standard_normal((600, s))
    want = oracle.block_nystrom_pcg(ref.matmat, B, mu, Pi, tol=1e-300, maxit=k)
    P = nys.Precond(dev(r["U"]), dev(r["lam"]))
    X, info = nys.nys_block_pcg_solve(op, P, mu, dev(B), tol=1e-300, maxit=k)
    assert info.iters == [k] * s and info.code == nys.NYS_NOT_CONVERGED
    np.testing.assert_allclose(X.cpu().numpy(), want["X"], rtol=1e-8, atol=1e-9 * np.abs(want["X"]).max())


@pytest.mark.parametrize("udtype", [torch.float64, torch.float32])
def test_block_solve_converges_like_the_oracle(udtype):
    ref, r, op = _rbf_case(n=900, ell=60, seed=63, sigma=3.5)
    mu = 1e-3
    U = r["U"].astype(np.float32).astype(np.float64) if udtype == torch.float32 else r["U"]
    Pi = lambda R: oracle.precond_inv_apply(U, r["lam"], mu, R)
    B = np.random.default_rng(64).standard_normal((900, 6))
    want = oracle.block_nystrom_pcg(ref.matmat, B, mu, Pi, tol=1e-10, maxit=1000)
    assert want["converged"]
    P = nys.Precond(dev(U, udtype), dev(r["lam"]))
    X, info = nys.nys_block_pcg_solve(op, P, mu, dev(B), tol=1e-10, maxit=1000, check_every=1)
    assert info.code == nys.NYS_OK and all(st == 0 for st in info.status)
    # ~90 block steps: rounding may move the step that crosses 1e-10 by one or two
    assert abs(info.iters[0] - want["iters"]) <= 2
    Xh = X.cpu().numpy()
    for c in range(6):
        assert oracle.true_relres(ref, mu, Xh[:, c], B[:, c]) <= 1e-10
    # fewer block steps than the slowest independent column needs
    single = [oracle.nystrom_pcg(ref.matmat, B[:, c], mu, Pi, tol=1e-10, maxit=1000)["iters"] for c in range(6)]
    assert info.iters[0] < max(single)


def test_block_solve_xtx_operator():
    w = ridge_dense(m=1500, n=400, ell=30, seed=65, with_omega=True)
    ref = oracle.XtXOp(w["X"])
    r = oracle.randomized_nystrom(ref, w["omega0"])
    op = nys.Operator.xtx(dev(w["X"], torch.float32))
    mu = 1e-3
    B = np.random.default_rng(66).standard_normal((400, 4))
    P = nys.Precond(dev(r["U"]), dev(r["lam"]))
    X, info = nys.nys_block_pcg_solve(op, P, mu, dev(B), tol=1e-11, maxit=500)
    assert info.code == nys.NYS_OK
    Xh = X.cpu().numpy()
    for c in range(4):
        assert oracle.true_relres(ref, mu, Xh[:, c], B[:, c]) <= 1e-11


def test_block_solve_rejects_dependent_columns_and_bad_sizes():
    ref, r, op = _rbf_case(n=200, ell=20, seed=67)
    P = nys.Precond(dev(r["U"]), dev(r["lam"]))
    b = np.random.default_rng(68).standard_normal(200)
    with pytest.raises(nys.NysError):
        nys.nys_block_pcg_solve(op, P, 1e-3, dev(np.stack([b, 2 * b], axis=1)))
    with pytest.raises(nys.NysError):
        nys.nys_block_pcg_solve(op, P, 1e-3, dev(np.random.default_rng(69).standard_normal((200, 65))))
