"""Parity of the HIP path (through the C ABI) against the CPU FP64 oracle.

Inputs come from the seeded generators in ``workloads``; the oracle never
receives a value computed by the device.  Where a result is unique only up to
signs/rotations (Omega after QR, U), the test compares invariant quantities
(A Omega Omega^T, U Lambda U^T, P^{-1} r).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from workloads import krr_small, lowrank_psd, ridge_dense, spectrum_psd  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_02820_amd as nys  # noqa: E402

DEV = "cuda"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def h(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_library_loaded():
    assert nys.lib().nys_version().startswith(b"nyspcg")


@pytest.mark.parametrize("n,ell,seed", [(37, 13, 7), (1000, 64, 20211001), (3, 1, 5)])
def test_gaussian_matches_philox_oracle(n, ell, seed):
    dev = h(nys.nys_gaussian(seed, n, ell))
    ref = oracle.gaussian_philox(seed, n, ell)
    np.testing.assert_allclose(dev, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind", ["dense", "xtx32", "xtx64", "rbf64", "rbf32"])
@pytest.mark.parametrize("k", [1, 3, 70])
def test_op_apply(kind, k):
    rng = np.random.default_rng(100 + k)
    if kind == "dense":
        A = spectrum_psd(1.0 / np.arange(1, 302), 3)
        op, ref = nys.Operator.dense(t64(A)), oracle.DenseOp(A)
    elif kind.startswith("xtx"):
        X = rng.standard_normal((517, 301)).astype(np.float32 if kind == "xtx32" else np.float64)
        op = nys.Operator.xtx(t32(X) if kind == "xtx32" else t64(X), scale=0.5)
        ref = oracle.XtXOp(X, 0.5)
    else:
        X = rng.standard_normal((301, 17)).astype(np.float32 if kind == "rbf32" else np.float64)
        op = nys.Operator.rbf(t32(X) if kind == "rbf32" else t64(X), 2.3)
        ref = oracle.RBFOp(X, 2.3)
    V = rng.standard_normal((301, k))
    mu = 0.37
    out = h(nys.nys_op_apply(op, mu, t64(V)))
    np.testing.assert_allclose(out, ref.matmat(V) + mu * V, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", ["dense64", "xtx32_f64", "xtx32_sketch_f32", "xtx32_sketch_bf16x3",
                                  "xtx32_sketch_bf16x3_rounds"])
def test_large_tile_products(case):
    """Products of at least 1e9 multiply-adds with 16-byte aligned operands take
    the 128 x 128 tile GEMM (split-K when the output has few tiles); the sizes
    leave ragged tiles in every dimension.  The last case's X Omega has
    between one and two rounds of tiles (157 x 4 = 628 on 512 slots), so its
    rows are done in two parts, the second split over k."""
    rng = np.random.default_rng(7)
    if case == "dense64":
        n, k = 2050, 250
        A = rng.standard_normal((n, n))
        A = A + A.T
        V = rng.standard_normal((n, k))
        out = h(nys.nys_op_apply(nys.Operator.dense(t64(A)), 0.25, t64(V)))
        assert rel(out, A @ V + 0.25 * V) < 1e-13
    elif case == "xtx32_f64":
        X = rng.standard_normal((4001, 1204)).astype(np.float32)
        V = rng.standard_normal((1204, 210))
        out = h(nys.nys_op_apply(nys.Operator.xtx(t32(X), scale=0.5), 0.25, t64(V)))
        ref = oracle.XtXOp(X.astype(np.float64), 0.5).matmat(V) + 0.25 * V
        assert rel(out, ref) < 1e-13
    else:
        m, n, ell = (20000, 1100, 400) if case.endswith("rounds") else (4001, 1204, 212)
        X = rng.standard_normal((m, n)).astype(np.float32)
        om0 = rng.standard_normal((n, ell))
        op = nys.Operator.xtx(t32(X))
        bf = "bf16x3" in case
        prec = nys.NYS_PREC_BF16X3_REFINE64 if bf else nys.NYS_PREC_FP32_REFINE64
        Om, Y = nys.nys_sketch(op, ell, omega0=t64(om0), prec=prec)
        Om, Y = h(Om), h(Y)
        Q = oracle.orthonormalize(om0)
        Xd = X.astype(np.float64)
        ref = oracle.XtXOp(Xd).matmat(Q)
        # float32 products over K = 4001 and 1204 terms: relative error ~1e-6;
        # bf16x3 products (hi/lo split, lo*lo dropped): ~3 * 2^-18 per product
        assert rel(Y @ Om.T, ref @ Q.T) < (1e-4 if bf else 2e-5)
        # entry by entry against X^T X times the device's own test matrix, each
        # entry bounded by c |X|^T |X| |Omega| (c: the per-product relative error
        # of the two roundings with margin), ragged tail tiles included
        err = np.abs(Y - oracle.XtXOp(Xd).matmat(Om))
        scale = np.abs(Xd).T @ (np.abs(Xd) @ np.abs(Om))
        assert (err / scale).max() < (1e-4 if bf else 5e-5), (err / scale).max()


@pytest.mark.parametrize("d", [1, 8, 33])
def test_rbf_single_vector_dims(d):
    rng = np.random.default_rng(200 + d)
    X = rng.standard_normal((777, d)) * 1.5
    v = rng.standard_normal(777)
    op = nys.Operator.rbf(t64(X), 1.9)
    out = h(nys.nys_op_apply(op, 0.0, t64(v)))
    np.testing.assert_allclose(out, oracle.RBFOp(X, 1.9).matmat(v), rtol=1e-12, atol=1e-12)


def test_xtx_single_vector_f32_arith():
    """float32 arithmetic over float32 data: within float32 rounding of the oracle."""
    w = ridge_dense(m=3000, n=1000, ell=50, seed=5)
    X = w["X"]
    v = np.random.default_rng(6).standard_normal(1000)
    op = nys.Operator.xtx(t32(X))
    out = h(nys.nys_op_apply(op, 1e-4, t32(v).to(torch.float32)))
    ref = oracle.XtXOp(X).matmat(v) + 1e-4 * v
    assert rel(out, ref) < 1e-5


def _sketch_case(n=300, ell=23, seed=41):
    A = spectrum_psd(1.0 / np.arange(1, n + 1) ** 1.5, seed)
    om0 = np.random.default_rng(seed + 1).standard_normal((n, ell))
    return A, om0


def test_sketch_is_range_invariant_match():
    A, om0 = _sketch_case()
    op = nys.Operator.dense(t64(A))
    Om, Y = nys.nys_sketch(op, om0.shape[1], omega0=t64(om0))
    Om, Y = h(Om), h(Y)
    np.testing.assert_allclose(Om.T @ Om, np.eye(om0.shape[1]), atol=1e-13)
    Q = oracle.orthonormalize(om0)
    np.testing.assert_allclose(Om @ Om.T, Q @ Q.T, atol=1e-12)
    np.testing.assert_allclose(Y @ Om.T, A @ Q @ Q.T, atol=1e-12)


@pytest.mark.parametrize("n,ell", [(300, 23), (517, 64), (200, 1), (130, 130)])
def test_factor_matches_oracle(n, ell):
    A, om0 = _sketch_case(n, ell, seed=n + ell)
    op = nys.Operator.dense(t64(A))
    Om, Y = nys.nys_sketch(op, ell, omega0=t64(om0))
    P = nys.nys_factor(Om, Y)
    ref = oracle.randomized_nystrom(oracle.DenseOp(A), om0)
    U, lam = h(P.U), h(P.lam)
    # U = B W S^{-1/2} from the eigenpairs (W, S) of B^T B: an off-diagonal e_ij
    # left by the eigensolver shows in U^T U as e_ij / sqrt(s_i s_j); entries
    # below 1e-14 max(s) are not rotated, so the bound grows for tiny s.
    s2 = lam + P.nu
    bound = 1e-13 + 4e-14 * s2.max() / np.sqrt(np.outer(s2, s2))
    assert np.all(np.abs(U.T @ U - np.eye(ell)) <= bound)
    assert np.all(np.diff(lam) <= 0)
    # the shift nu = eps(||Y||_F): the same float64 number as the oracle's, unless
    # ||Y||_F lies within rounding of a power of two (then eps may differ by 2x)
    yf = np.linalg.norm(ref["Y"], "fro")
    if abs(np.log2(yf) - np.round(np.log2(yf))) > 1e-12:
        assert P.nu == ref["nu"], (P.nu, ref["nu"])
    else:
        assert P.nu in (ref["nu"], 2 * ref["nu"], 0.5 * ref["nu"])
    np.testing.assert_allclose(lam, ref["lam"], rtol=1e-9, atol=1e-12 * ref["lam"][0])
    Ah = (U * lam) @ U.T
    Ar = (ref["U"] * ref["lam"]) @ ref["U"].T
    assert rel(Ah, Ar) < 1e-10
    r = np.random.default_rng(1).standard_normal(n)
    mu = 1e-3
    z_dev = h(nys.nys_precond_apply(P, mu, t64(r)))
    z_ref = oracle.precond_inv_apply(ref["U"], ref["lam"], mu, r)
    assert rel(z_dev, z_ref) < 1e-9


def test_factor_low_rank_exact_recovery():
    A = lowrank_psd(400, 30, seed=9)
    om0 = np.random.default_rng(10).standard_normal((400, 48))
    op = nys.Operator.dense(t64(A))
    Om, Y = nys.nys_sketch(op, 48, omega0=t64(om0))
    P = nys.nys_factor(Om, Y)
    U, lam = h(P.U), h(P.lam)
    assert np.linalg.norm(A - (U * lam) @ U.T, 2) <= 1e-11 * np.linalg.norm(A, 2)


def test_device_preconditioner_spectrum_rank_deficient():
    """Rank-30 A sketched with l = 48 (so lam_l = 0): the device factor's
    P^{-1}, formed column by column through the device apply, equals the
    oracle's P^{-1} entrywise (the I - U U^T part included, which depends on
    the orthonormality of U's columns with tiny eigenvalues); its eigenvalues
    lie in [(lam_l + mu)/(lam_1 + mu), 1] (eq. (NysPre)), and
    P^{-1/2} (A + mu I) P^{-1/2} has no eigenvalue below mu (the preconditioned
    spectrum bound, read as >= mu)."""
    n, ell = 300, 48
    A = lowrank_psd(n, 30, seed=19)
    om0 = np.random.default_rng(20).standard_normal((n, ell))
    op = nys.Operator.dense(t64(A))
    P = nys.nys_factor(*nys.nys_sketch(op, ell, omega0=t64(om0)))
    ref = oracle.randomized_nystrom(oracle.DenseOp(A), om0)
    lam = h(P.lam)
    assert lam[-1] <= 1e-12 * lam[0]
    for mu in (1e-3, 1.0):
        E = np.eye(n)
        Pinv = np.concatenate([h(nys.nys_precond_apply(P, mu, t64(E[:, j:j + 150]))) for j in range(0, n, 150)],
                              axis=1)
        Pref = oracle.precond_inv_matrix(ref["U"], ref["lam"], mu)
        assert np.abs(Pinv - Pref).max() <= 1e-10, (mu, np.abs(Pinv - Pref).max())
        ev, V = np.linalg.eigh(0.5 * (Pinv + Pinv.T))
        lo = (lam[-1] + mu) / (lam[0] + mu)
        assert ev.min() >= lo * (1 - 1e-8) and ev.max() <= 1 + 1e-10, (mu, ev.min(), lo, ev.max())
        S = (V * np.sqrt(ev)) @ V.T
        pre = np.linalg.eigvalsh(S @ (A + mu * np.eye(n)) @ S)
        assert pre.min() >= mu * (1 - 1e-8), (mu, pre.min())


def test_float32_factor_orthonormality_and_spectrum():
    """The float32-U factor (the mixed-precision modes' storage, eigensolver
    stopped at ratio 1e-3): U's columns orthonormal to 2e-5 in the 2-norm, so
    P^{-1} = I + U F U^T keeps its eigenvalues in [(lam_l + mu)/(lam_1 + mu), 1]
    up to that departure, far inside positive definiteness here; and the
    approximation equals the oracle's to float32 accuracy."""
    w = ridge_dense(m=3000, n=800, ell=160, seed=21)
    X = w["X"]
    op = nys.Operator.xtx(t32(X))
    prec = nys.NYS_PREC_FP32_REFINE64
    P = nys.nys_factor(*nys.nys_sketch(op, 160, omega0=t64(w["omega0"]), prec=prec), dtype=torch.float32,
                       prec=prec)
    U, lam = h(P.U), h(P.lam)
    dev = np.linalg.norm(U.T @ U - np.eye(160), 2)
    assert dev <= 2e-5, dev
    mu = w["mu"]
    E = np.eye(800)
    Pinv = np.concatenate([h(nys.nys_precond_apply(P, mu, t64(E[:, j:j + 200]))) for j in range(0, 800, 200)],
                          axis=1)
    ev = np.linalg.eigvalsh(0.5 * (Pinv + Pinv.T))
    lo = (lam[-1] + mu) / (lam[0] + mu)
    assert ev.min() >= lo - 2 * dev and ev.max() <= 1 + 2 * dev, (ev.min(), lo, ev.max())
    assert lo > 10 * dev
    ref = oracle.randomized_nystrom(oracle.XtXOp(X), w["omega0"])
    Ah = (U * lam) @ U.T
    Ar = (ref["U"] * ref["lam"]) @ ref["U"].T
    assert rel(Ah, Ar) < 1e-4


@pytest.mark.parametrize("k", [1, 5])
def test_precond_apply_with_oracle_factors(k):
    """Oracle U, lam passed in: P^{-1} R agrees to rounding (eq. (NysPre))."""
    A, om0 = _sketch_case(411, 37, seed=77)
    ref = oracle.randomized_nystrom(oracle.DenseOp(A), om0)
    P = nys.Precond(t64(ref["U"]), t64(ref["lam"]))
    R = np.random.default_rng(3).standard_normal((411, k))
    for mu in (1e-1, 1e-4, 0.0):
        z = h(nys.nys_precond_apply(P, mu, t64(R)))
        np.testing.assert_allclose(z, oracle.precond_inv_apply(ref["U"], ref["lam"], mu, R), rtol=1e-12,
                                   atol=1e-12)


def _krr(n, ell, seed):
    w = krr_small(n=n, d=8, ell=ell, seed=seed)
    op_ref = oracle.RBFOp(w["X"], w["sigma"])
    b = op_ref.matmat(w["w"]) + w["noise"] * w["eps"]
    return w, op_ref, b


@pytest.mark.parametrize("n,ell", [(700, 50), (2048, 100)])
def test_pcg_solve_fp64_rbf(n, ell):
    w, op_ref, b = _krr(n, ell, 20211001 if n == 2048 else 11)
    op = nys.Operator.rbf(t64(w["X"]), w["sigma"])
    Om, Y = nys.nys_sketch(op, ell, omega0=t64(w["omega0"]))
    P = nys.nys_factor(Om, Y)
    x, info = nys.nys_pcg_solve(op, P, w["mu"], t64(b), tol=1e-10, maxit=2000)
    x = h(x)
    assert info.status[0] == 0
    rr = oracle.true_relres(op_ref, w["mu"], x, b)
    assert rr <= 1e-10
    assert abs(info.relres[0] - rr) <= 1e-12
    ref = oracle.randomized_nystrom(op_ref, w["omega0"])
    out = oracle.nystrom_pcg(op_ref.matmat, b, w["mu"],
                             lambda v: oracle.precond_inv_apply(ref["U"], ref["lam"], w["mu"], v),
                             tol=1e-10, maxit=2000)
    # Same Omega, same algorithm: the iteration counts agree up to the drift of
    # finite-precision CG over a few hundred steps (loss of orthogonality).
    assert abs(info.iters[0] - out["iters"]) <= max(2, 0.05 * out["iters"])
    xs = oracle.dense_solve(op_ref.dense(), w["mu"], b)
    ev = np.linalg.eigvalsh(op_ref.dense())
    kappa = (ev.max() + w["mu"]) / w["mu"]
    assert rel(x, xs) <= kappa * 1e-10


def test_pcg_mu_grid_and_rhs_block():
    w, op_ref, b = _krr(600, 40, 12)
    rng = np.random.default_rng(13)
    B = np.stack([b, rng.standard_normal(600)], axis=1)
    mus = [1e-4, 1e-2, 1.0]
    op = nys.Operator.rbf(t64(w["X"]), w["sigma"])
    Om, Y = nys.nys_sketch(op, 40, omega0=t64(w["omega0"]))
    P = nys.nys_factor(Om, Y)
    X, info = nys.nys_pcg_solve(op, P, mus, t64(B), tol=1e-10, maxit=3000)
    X = h(X)
    K = op_ref.dense()
    for m, mu in enumerate(mus):
        for r in range(2):
            c = m * 2 + r
            assert info.status[c] == 0
            assert oracle.true_relres(op_ref, mu, X[:, c], B[:, r]) <= 1e-10
            xs = oracle.dense_solve(K, mu, B[:, r])
            assert rel(X[:, c], xs) <= 1e-10 * (np.linalg.eigvalsh(K).max() + mu) / mu


def test_pcg_xtx_refinement_small():
    w = ridge_dense(m=4000, n=800, ell=100, seed=14)
    X = w["X"]
    op_ref = oracle.XtXOp(X)
    b = X.astype(np.float64).T @ w["y"]
    op = nys.Operator.xtx(t32(X))
    Om, Y = nys.nys_sketch(op, 100, omega0=t64(w["omega0"]), prec=nys.NYS_PREC_FP32_REFINE64)
    P = nys.nys_factor(Om, Y, dtype=torch.float32, prec=nys.NYS_PREC_FP32_REFINE64)
    x, info = nys.nys_pcg_solve(op, P, w["mu"], t64(b), tol=1e-10, maxit=500, prec=nys.NYS_PREC_FP32_REFINE64)
    assert info.status[0] == 0 and info.refine_steps >= 1
    assert oracle.true_relres(op_ref, w["mu"], h(x), b) <= 1e-10
    # plain float64 path on the same operator reaches the same solution
    P64 = nys.nys_factor(*nys.nys_sketch(op, 100, omega0=t64(w["omega0"])))
    x64, info64 = nys.nys_pcg_solve(op, P64, w["mu"], t64(b), tol=1e-10, maxit=500)
    assert oracle.true_relres(op_ref, w["mu"], h(x64), b) <= 1e-10
    xs = oracle.dense_solve(op_ref.dense(), w["mu"], b)
    assert rel(h(x), xs) < 1e-7 and rel(h(x64), xs) < 1e-7


def test_pcg_fp32_only_path():
    w = ridge_dense(m=3000, n=600, ell=80, seed=15)
    X = w["X"]
    b = X.astype(np.float64).T @ w["y"]
    op = nys.Operator.xtx(t32(X))
    P = nys.nys_factor(*nys.nys_sketch(op, 80, omega0=t64(w["omega0"]), prec=nys.NYS_PREC_FP32),
                       dtype=torch.float32, prec=nys.NYS_PREC_FP32)
    x, info = nys.nys_pcg_solve(op, P, w["mu"], t64(b), tol=1e-5, maxit=500, prec=nys.NYS_PREC_FP32)
    assert oracle.true_relres(oracle.XtXOp(X), w["mu"], h(x), b) <= 1e-5


def test_backward_rbf_against_oracle():
    w, op_ref, b = _krr(400, 40, 16)
    mu = w["mu"] * 10
    c = np.random.default_rng(17).standard_normal(400)
    op = nys.Operator.rbf(t64(w["X"]), w["sigma"])
    P = nys.nys_factor(*nys.nys_sketch(op, 40, omega0=t64(w["omega0"])))
    x, _ = nys.nys_pcg_solve(op, P, mu, t64(b), tol=1e-12, maxit=3000)
    gx = c  # L = c^T x
    r = nys.nys_pcg_backward(op, P, mu, x, t64(gx), want_sigma=True, tol=1e-12, maxit=3000)
    K = op_ref.dense()
    xs = oracle.dense_solve(K, mu, b)
    g = oracle.adjoint_gradients(op_ref, mu, xs, gx, lambda v: oracle.dense_solve(K, mu, v))
    assert rel(h(r["gb"]), g["gb"]) < 1e-8
    assert r["gmu"] == pytest.approx(g["gmu"], rel=1e-7)
    assert r["gsigma"] == pytest.approx(g["gsigma"], rel=1e-7)


def test_backward_xtx_data_gradient():
    w = ridge_dense(m=500, n=120, ell=30, seed=18)
    X = w["X"].astype(np.float64)
    b = X.T @ w["y"]
    mu = 1e-2
    c = np.random.default_rng(19).standard_normal(120)
    op = nys.Operator.xtx(t64(X))
    P = nys.nys_factor(*nys.nys_sketch(op, 30, omega0=t64(w["omega0"])))
    x, _ = nys.nys_pcg_solve(op, P, mu, t64(b), tol=1e-12, maxit=2000)
    r = nys.nys_pcg_backward(op, P, mu, x, t64(c), want_X=True, tol=1e-12, maxit=2000)
    A = X.T @ X
    xs = oracle.dense_solve(A, mu, b)
    g = oracle.adjoint_gradients(oracle.XtXOp(X), mu, xs, c, lambda v: oracle.dense_solve(A, mu, v))
    assert rel(h(r["gX"]), g["gX"]) < 1e-7


def test_rbf_cross_products():
    rng = np.random.default_rng(21)
    Xtr = rng.standard_normal((500, 16))
    Xv = rng.standard_normal((130, 16))
    v = rng.standard_normal(130)
    u = rng.standard_normal(500)
    op = nys.Operator.rbf(t64(Xtr), 4.0)
    Kv = oracle.rbf_kernel_block(Xv, Xtr, 4.0)
    out = h(nys.nys_rbf_cross(op, t64(Xv), t64(u)))
    np.testing.assert_allclose(out, Kv @ u, rtol=1e-12, atol=1e-12)
    out_t = h(nys.nys_rbf_cross(op, t64(Xv), t64(v), transpose=True))
    np.testing.assert_allclose(out_t, Kv.T @ v, rtol=1e-12, atol=1e-12)
    # dK/dsigma form: v has nv entries, wvec n entries (a regression case: the
    # call must not read v as an n-vector)
    dv, ds = nys.nys_rbf_cross(op, t64(Xv), t64(v), wvec=t64(u))
    d2 = ((Xv[:, None, :] - Xtr[None, :, :]) ** 2).sum(-1)
    np.testing.assert_allclose(h(dv), (Kv * d2 / 4.0 ** 3) @ u, rtol=1e-11, atol=1e-13)
    assert ds == pytest.approx(float(v @ ((Kv * d2 / 4.0 ** 3) @ u)), rel=1e-11)
    with pytest.raises(ValueError):
        nys.nys_rbf_cross(op, t64(Xv), t64(u), wvec=t64(u))


def test_determinism_bitwise():
    w, op_ref, b = _krr(900, 60, 22)
    op = nys.Operator.rbf(t64(w["X"]), w["sigma"])
    xs = []
    for _ in range(2):
        P = nys.nys_factor(*nys.nys_sketch(op, 60, omega0=t64(w["omega0"])))
        x, _ = nys.nys_pcg_solve(op, P, w["mu"], t64(b), tol=1e-10, maxit=2000)
        xs.append(h(x))
    assert np.array_equal(xs[0], xs[1])


def test_error_paths_on_device():
    w, op_ref, b = _krr(200, 20, 23)
    op = nys.Operator.rbf(t64(w["X"]), w["sigma"])
    P = nys.nys_factor(*nys.nys_sketch(op, 20, omega0=t64(w["omega0"])))
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve(op, P, -1.0, t64(b))
    assert e.value.status == nys.NYS_ERR_ARG
    x, info = nys.nys_pcg_solve(op, P, w["mu"], t64(b), tol=1e-14, maxit=3)
    assert info.code == nys.NYS_NOT_CONVERGED and info.iters[0] == 3
    # indefinite dense operator: breakdown
    Aneg = -np.eye(50)
    opn = nys.Operator.dense(t64(Aneg))
    Pn = nys.Precond(t64(np.eye(50)[:, :2]), t64(np.array([1.0, 1.0])))
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve(opn, Pn, 0.5, t64(np.ones(50)), maxit=10)
    assert e.value.status == nys.NYS_ERR_BREAKDOWN
    # rank-deficient test matrix is reported by the sketch
    with pytest.raises(nys.NysError) as e:
        nys.nys_sketch(op, 20, omega0=t64(np.zeros((200, 20))))
    assert e.value.status == nys.NYS_ERR_NOT_PSD
    # sketch sizes and preconditioner ranks above 2048 are refused up front
    big = nys.Operator.dense(t64(np.eye(2100)))
    with pytest.raises(nys.NysError) as e:
        nys.nys_sketch(big, 2049, seed=1)
    assert e.value.status == nys.NYS_ERR_ARG
    Pbig = nys.Precond(t64(np.eye(2100)[:, :2049]), t64(np.ones(2049)))
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve(big, Pbig, 0.5, t64(np.ones(2100)), maxit=5)
    assert e.value.status == nys.NYS_ERR_ARG
    # zero columns past the first 32 x 32 block: the zero pivot (column 40) is
    # met by a later step of the blocked Cholesky, not by its first block
    om_bad = np.random.default_rng(5).standard_normal((200, 70))
    om_bad[:, 40:] = 0.0
    with pytest.raises(nys.NysError) as e:
        nys.nys_sketch(op, 70, omega0=t64(om_bad))
    assert e.value.status == nys.NYS_ERR_NOT_PSD


# ---------------------------------------------------------------- reduced-precision RBF

def _mixture_case(n, d, ell, seed):
    from workloads import krr_mixture
    w = krr_mixture(n=n, d=d, ell=ell, seed=seed)
    op_ref = oracle.RBFOp(w["X"], w["sigma"])
    b = op_ref.matmat(w["w"]) + w["noise"] * w["eps"]
    return w, op_ref, b


@pytest.mark.parametrize("prec,tol", [(1, 2e-5), (3, 2e-4)])
@pytest.mark.parametrize("k", [1, 5, 20, 40, 70, 150])
def test_rbf_lowp_products(prec, tol, k):
    """float32 Gram (prec 1) and bf16x3 Gram (prec 3) against the float64 oracle.
    Bounds: float32 exp and accumulation over ~1e3 terms (~1e-6 .. 1e-5);
    bf16x3 keeps ~16 bits of each coordinate (~1e-4).  k covers the one-vector
    kernel, the register kernel's 16, 32 and 64 column blocks (ragged) and the
    LDS kernel's 128 and (bf16x3 mode) 256 column blocks."""
    w, op_ref, _ = _mixture_case(1111, 32, 10, 40 + k)
    op = nys.Operator.rbf(t32(w["X"]), w["sigma"])
    V = np.random.default_rng(k).standard_normal((1111, k)).astype(np.float32).astype(np.float64)
    out = h(nys.nys_op_apply(op, 0.25, t32(V), prec=prec))
    ref = op_ref.matmat(V) + 0.25 * V
    assert rel(out, ref) < tol
    # entry by entry: |error| <= c (|K| |V| + 0.25 |V|), c = 2e-5 (float32 Gram and
    # accumulation) or 5e-4 (bf16x3 Gram: ~2^-16 of each product in the exponent)
    scale = op_ref.matmat(np.abs(V)) + 0.25 * np.abs(V)
    assert (np.abs(out - ref) / scale).max() < (2e-5 if prec == 1 else 5e-4)


@pytest.mark.parametrize("d", [3, 16])
def test_rbf_lowp_small_dims(d):
    rng = np.random.default_rng(60 + d)
    X = rng.standard_normal((517, d)).astype(np.float32)
    op = nys.Operator.rbf(t32(X), 1.7)
    v = rng.standard_normal(517)
    ref = oracle.RBFOp(X, 1.7).matmat(v)
    assert rel(h(nys.nys_op_apply(op, 0.0, t32(v), prec=3)), ref) < 2e-4
    assert rel(h(nys.nys_op_apply(op, 0.0, t32(v), prec=1)), ref) < 2e-5
    V = rng.standard_normal((517, 3))
    ref = oracle.RBFOp(X, 1.7).matmat(V)
    assert rel(h(nys.nys_op_apply(op, 0.0, t32(V), prec=3)), ref) < 2e-4
    assert rel(h(nys.nys_op_apply(op, 0.0, t32(V), prec=1)), ref) < 2e-5


@pytest.mark.parametrize("prec", [2, 3])
def test_rbf_mixed_precision_solve_reaches_fp64_tolerance(prec):
    """Reduced-precision inner PCG + float64 refinement: true float64 relative
    residual <= 1e-10 (the precision form is judged by the float64 oracle)."""
    n = 3000
    w, op_ref, b = _mixture_case(n, 32, 200, 41)
    mu = 1e-6 * n
    op = nys.Operator.rbf(t32(w["X"]), w["sigma"])
    Om, Y = nys.nys_sketch(op, 200, omega0=t64(w["omega0"]), prec=prec)
    P = nys.nys_factor(Om, Y, dtype=torch.float32, prec=prec)
    x, info = nys.nys_pcg_solve(op, P, mu, t64(b), tol=1e-10, maxit=2000, prec=prec, max_refine=20,
                                inner_tol=1e-3)
    assert info.status[0] == 0, info
    assert oracle.true_relres(op_ref, mu, h(x), b) <= 1e-10
    xs = oracle.dense_solve(op_ref.dense(), mu, b)
    assert rel(h(x), xs) < 1e-6


def test_rbf_lowp_sketch_close_to_oracle():
    w, op_ref, _ = _mixture_case(1500, 32, 64, 42)
    op = nys.Operator.rbf(t32(w["X"]), w["sigma"])
    for prec, tol in ((1, 1e-5), (3, 1e-3)):
        Om, Y = nys.nys_sketch(op, 64, omega0=t64(w["omega0"]), prec=prec)
        Om, Y = h(Om), h(Y)
        Q = oracle.orthonormalize(w["omega0"])
        assert rel(Y @ Om.T, op_ref.matmat(Q) @ Q.T) < tol
        # entry by entry against K times the device's own test matrix, bounded
        # by c |K| |Omega| (c as in the product test; Omega is rounded to
        # float32 for the reduced-precision products)
        Om32 = Om.astype(np.float32).astype(np.float64)
        err = np.abs(Y - op_ref.matmat(Om32))
        scale = op_ref.matmat(np.abs(Om32))
        assert (err / scale).max() < (2e-5 if prec == 1 else 5e-4), (prec, (err / scale).max())


def test_rbf_block_mu_grid_float_refine():
    """mu grid x right-hand sides in one block solve with float32 block products."""
    n = 1200
    w, op_ref, b = _mixture_case(n, 16, 100, 43)
    B = np.stack([b, np.random.default_rng(44).standard_normal(n)], axis=1)
    mus = [1e-3 * n, 1e-5 * n]
    op = nys.Operator.rbf(t32(w["X"]), w["sigma"])
    Om, Y = nys.nys_sketch(op, 100, omega0=t64(w["omega0"]), prec=2)
    P = nys.nys_factor(Om, Y, dtype=torch.float32, prec=2)
    X, info = nys.nys_pcg_solve(op, P, mus, t64(B), tol=1e-10, maxit=3000, prec=2, max_refine=20,
                                inner_tol=1e-3)
    X = h(X)
    for m, mu in enumerate(mus):
        for r in range(2):
            assert oracle.true_relres(op_ref, mu, X[:, m * 2 + r], B[:, r]) <= 1e-10


@pytest.mark.parametrize("kind,check_every", [("rbf", 1), ("rbf", 8), ("xtx", 4)])
def test_block_column_compaction(kind, check_every):
    """A wide mu grid makes columns finish at very different iterations; the
    block solve drops finished columns from the products at each poll.  Every
    column must still reach the tolerance (oracle residual) in the iteration
    count of its own single-column solve, and land at that solve's x."""
    if kind == "rbf":
        w, op_ref, b = _krr(500, 30, 45)
        op = nys.Operator.rbf(t64(w["X"]), w["sigma"])
        ell, om0 = 30, w["omega0"]
    else:
        w = ridge_dense(m=1500, n=400, ell=40, seed=46)
        op_ref = oracle.XtXOp(w["X"])
        b = w["X"].astype(np.float64).T @ w["y"]
        op = nys.Operator.xtx(t64(w["X"].astype(np.float64)))
        ell, om0 = 40, w["omega0"]
    n = op_ref.n
    rng = np.random.default_rng(47)
    B = np.stack([b] + [rng.standard_normal(n) for _ in range(3)], axis=1)
    mus = list(np.logspace(-5, 0, 10))
    P = nys.nys_factor(*nys.nys_sketch(op, ell, omega0=t64(om0)))
    X, info = nys.nys_pcg_solve(op, P, mus, t64(B), tol=1e-10, maxit=4000, check_every=check_every)
    X = h(X)
    assert len(set(info.iters)) > 3  # columns really finish at different points
    for m, mu in enumerate(mus):
        for r in range(B.shape[1]):
            c = m * B.shape[1] + r
            assert info.status[c] == 0 and info.relres[c] <= 1e-10
            # the oracle re-evaluates the residual; at mu = 1e-5 the product
            # K x carries rounding of order eps ||K|| ||x|| (~1e-12 of ||b||),
            # so the two float64 evaluations may straddle 1e-10 by that much
            assert oracle.true_relres(op_ref, mu, X[:, c], B[:, r]) <= 1.02e-10
            if (m + r) % 7 == 0:  # a spread of single-column comparisons
                x1, i1 = nys.nys_pcg_solve(op, P, mu, t64(B[:, r]), tol=1e-10, maxit=4000)
                assert abs(i1.iters[0] - info.iters[c]) <= max(2, info.iters[c] // 20)
                kappa = 1.0 + 10.0 / mu
                assert rel(X[:, c], h(x1)) <= 1e-9 * kappa


def _ragged_problems(sizes, seed, dtype=np.float32):
    """Independent ridge problems X_k (m_k x n_k, unaligned n_k included) as in
    the batched workload, with their float64 right-hand sides."""
    probs = []
    for q, (m, n) in enumerate(sizes):
        w = ridge_dense(m=m, n=n, ell=max(8, 16 * -(-n // 128)), seed=seed + q)
        X = w["X"].astype(dtype)
        probs.append(dict(X=X, b=X.astype(np.float64).T @ w["y"], mu=w["mu"] * (1 + q), ell=w["ell"],
                          omega0=w["omega0"]))
    return probs


@pytest.mark.parametrize("prec", [0, 2])
def test_ragged_batched_solve(prec):
    """All problems advance in the same launches; each must reach the float64
    tolerance on its own operator (oracle residual) with the iteration count of
    its own single solve."""
    sizes = [(1200, 301), (800, 200), (2000, 513), (600, 150), (1500, 387), (900, 64)]
    probs = _ragged_problems(sizes, 60, np.float32 if prec else np.float64)
    tdev = t32 if prec else t64
    udt = torch.float32 if prec else torch.float64
    ops, Ps = [], []
    for p in probs:
        op = nys.Operator.xtx(tdev(p["X"]))
        Om, Y = nys.nys_sketch(op, p["ell"], omega0=t64(p["omega0"]), prec=prec)
        ops.append(op)
        Ps.append(nys.nys_factor(Om, Y, dtype=udt, prec=prec))
    Xs, info = nys.nys_pcg_solve_ragged(ops, Ps, [p["mu"] for p in probs], [t64(p["b"]) for p in probs],
                                        tol=1e-10, maxit=2000, prec=prec)
    for q, p in enumerate(probs):
        opr = oracle.XtXOp(p["X"])
        assert info.status[q] == 0 and info.relres[q] <= 1e-10
        assert oracle.true_relres(opr, p["mu"], h(Xs[q]), p["b"]) <= 1.02e-10
        xs = oracle.dense_solve(opr.dense(), p["mu"], p["b"])
        assert rel(h(Xs[q]), xs) < 1e-5  # kappa(A + mu I) <= 1e4 times 1e-10
        if prec == 0:
            x1, i1 = nys.nys_pcg_solve(ops[q], Ps[q], p["mu"], t64(p["b"]), tol=1e-10, maxit=2000)
            assert abs(i1.iters[0] - info.iters[q]) <= max(2, i1.iters[0] // 20)


def test_ragged_mixed_operators_fall_back():
    """A batch that mixes operator kinds is solved problem by problem."""
    probs = _ragged_problems([(700, 180), (500, 90)], 70, np.float64)
    w, op_ref, b = _krr(300, 20, 71)
    ops = [nys.Operator.xtx(t64(p["X"])) for p in probs] + [nys.Operator.rbf(t64(w["X"]), w["sigma"])]
    oms = [p["omega0"] for p in probs] + [w["omega0"]]
    ells = [p["ell"] for p in probs] + [20]
    Ps = [nys.nys_factor(*nys.nys_sketch(o, l, omega0=t64(om))) for o, l, om in zip(ops, ells, oms)]
    mus = [p["mu"] for p in probs] + [1e-2]
    bs = [p["b"] for p in probs] + [b]
    Xs, info = nys.nys_pcg_solve_ragged(ops, Ps, mus, [t64(x) for x in bs], tol=1e-10, maxit=2000)
    refs = [oracle.XtXOp(p["X"]) for p in probs] + [op_ref]
    for q in range(3):
        assert info.status[q] == 0
        assert oracle.true_relres(refs[q], mus[q], h(Xs[q]), bs[q]) <= 1.02e-10


@pytest.mark.parametrize("n,ell", [(1500, 500), (1400, 500), (200, 64)])
def test_sketch_device_gaussian_orthonormal(n, ell):
    """The device test matrix is orthonormalised by one CholeskyQR pass when
    n >= 3 l (Gaussian, well conditioned) and by two otherwise; either way
    Omega^T Omega = I and Y = A Omega."""
    A = spectrum_psd(1.0 / np.arange(1, n + 1) ** 2, 80 + n)
    op = nys.Operator.dense(t64(A))
    Om, Y = nys.nys_sketch(op, ell, seed=17)
    Om, Y = h(Om), h(Y)
    assert np.linalg.norm(Om.T @ Om - np.eye(ell), 2) < 1e-13
    assert np.linalg.norm(Y - A @ Om) <= 1e-12 * np.linalg.norm(Y)
