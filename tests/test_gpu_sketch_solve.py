"""Parity of Nystrom sketch-and-solve (through the C ABI) against the CPU
FP64 oracle, on approximations the oracle builds from seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from workloads import krr_small, spectrum_psd  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_02820_amd as nys  # noqa: E402

DEV = "cuda"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.mark.parametrize("udtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("k", [1, 5, 70])
def test_sketch_solve_matches_oracle(udtype, k):
    n, ell, mu = 900, 60, 3e-3
    A = spectrum_psd(np.exp(-np.arange(n) / 25.0), 41)
    r = oracle.randomized_nystrom(oracle.DenseOp(A), np.random.default_rng(42).standard_normal((n, ell)))
    U = r["U"].astype(np.float32).astype(np.float64) if udtype == torch.float32 else r["U"]
    B = np.random.default_rng(43).standard_normal((n, k))
    P = nys.Precond(dev(U, udtype), dev(r["lam"]))
    X = nys.nys_sketch_solve(P, mu, dev(B)).cpu().numpy()
    want = oracle.nystrom_sketch_solve(U, r["lam"], mu, B)
    np.testing.assert_allclose(X, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_sketch_solve_on_a_kernel_problem_is_only_approximate():
    """The device pipeline (sketch, factor, sketch-and-solve) against the
    oracle's on the same Gaussian draw, and its error against the exact
    solution, which PCG removes."""
    w = krr_small(n=800, d=8, ell=60, seed=44)
    ref = oracle.RBFOp(w["X"], w["sigma"])
    op = nys.Operator.rbf(dev(w["X"]), w["sigma"])
    b = ref.matmat(w["w"]) + w["noise"] * w["eps"]
    mu = w["mu"]
    Om, Y = nys.nys_sketch(op, 60, omega0=dev(w["omega0"]))
    P = nys.nys_factor(Om, Y)
    x = nys.nys_sketch_solve(P, mu, dev(b)).cpu().numpy()
    r = oracle.randomized_nystrom(ref, w["omega0"])
    want = oracle.nystrom_sketch_solve(r["U"], r["lam"], mu, b)
    # the two approximations agree to float64 roundoff of K, amplified by 1/mu
    assert np.linalg.norm(x - want) <= 1e-7 * np.linalg.norm(want)
    xs = oracle.dense_solve(ref.dense(), mu, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) > 1e-3
    xp, info = nys.nys_pcg_solve(op, P, mu, dev(b), tol=1e-10, maxit=3000)
    assert info.status[0] == 0 and oracle.true_relres(ref, mu, xp.cpu().numpy(), b) <= 1e-10


def test_sketch_solve_argument_errors():
    P = nys.Precond(dev(np.eye(30)[:, :3]), dev(np.ones(3)))
    with pytest.raises(nys.NysError):
        nys.nys_sketch_solve(P, 0.0, dev(np.ones(30)))
