"""nys_pcg_solve_noalloc: the device-info solve without a workspace argument
(its scratch is the library's static per-GPU array).  Two calls in a row,
the second on a smaller problem, each compared with the workspace form of
nys_pcg_solve on the same inputs (same kernels: bit-identical results) and
judged by the float64 oracle's true residual; a solve too large for the
static scratch is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from workloads import krr_small  # noqa: E402

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


def _info(k):
    return (torch.zeros(k, dtype=torch.int32, device=DEV), torch.zeros(k, dtype=torch.float64, device=DEV),
            torch.full((k,), 99, dtype=torch.int32, device=DEV))


def _case(n, ell, seed, nrhs):
    w = krr_small(n=n, d=8, ell=ell, seed=seed)
    opr = oracle.RBFOp(w["X"], w["sigma"])
    b = opr.matmat(w["w"]) + w["noise"] * w["eps"]
    cols = [b] + [np.random.default_rng(seed + j).standard_normal(n) for j in range(1, nrhs)]
    return w, np.stack(cols, axis=1)


@pytest.mark.parametrize("n,ell,nrhs,mus,prec,seed", [
    (700, 40, 2, [1e-3, 1e-2, 1e-1], 0, 71),   # first call: 6 columns, float64
    (300, 20, 1, [1e-2], 2, 72),               # second call: smaller, float32 inner + float64 refinement
])
def test_noalloc_matches_workspace_form(n, ell, nrhs, mus, prec, seed):
    w, B = _case(n, ell, seed, nrhs)
    data = t64(w["X"]) if prec == 0 else t32(w["X"])
    op = nys.Operator.rbf(data, w["sigma"])
    udt = torch.float64 if prec == 0 else torch.float32
    P = nys.nys_factor(*nys.nys_sketch(op, ell, omega0=t64(w["omega0"]), prec=prec), dtype=udt, prec=prec)
    k = len(mus) * nrhs
    kw = dict(tol=1e-10, maxit=700 if prec == 0 else 200, prec=prec, max_refine=6, inner_tol=1e-3)
    Bt = t64(B)
    Xs = torch.zeros(n, k, dtype=torch.float64, device=DEV)
    i_s, r_s, s_s = _info(k)
    steps_s = nys.nys_pcg_solve_noalloc(op, P, mus, Bt, Xs, i_s, r_s, s_s, **kw)
    Xw = torch.zeros(n, k, dtype=torch.float64, device=DEV)
    i_w, r_w, s_w = _info(k)
    steps_w = nys.nys_pcg_solve_device(op, P, mus, Bt, Xw, i_w, r_w, s_w, **kw)
    torch.cuda.synchronize()
    assert steps_s == steps_w
    assert np.array_equal(h(Xs), h(Xw))
    assert torch.equal(i_s, i_w) and torch.equal(r_s, r_w) and torch.equal(s_s, s_w)
    opr_d = oracle.RBFOp(np.asarray(w["X"], dtype=np.float32) if prec else w["X"], w["sigma"])
    Xh = h(Xs)
    for m, mu in enumerate(mus):
        for r in range(nrhs):
            c = m * nrhs + r
            true = oracle.true_relres(opr_d, mu, Xh[:, c], B[:, r])
            assert int(s_s[c]) == nys.NYS_OK and true <= 1.02e-10, (c, int(s_s[c]), true)
            assert abs(float(r_s[c]) - true) <= 1e-12


def test_noalloc_refuses_oversized_and_host_polled_calls():
    n = 60000
    X = torch.zeros(n, 2, dtype=torch.float64, device=DEV)
    op = nys.Operator.rbf(X, 1.0)
    U = torch.zeros(n, 1, dtype=torch.float64, device=DEV)
    lam = torch.ones(1, dtype=torch.float64, device=DEV)
    P = nys.Precond(U, lam, 0.0)
    mus = [0.1 * (j + 1) for j in range(256)]
    B = torch.zeros(n, 1, dtype=torch.float64, device=DEV)
    Xo = torch.zeros(n, 256, dtype=torch.float64, device=DEV)
    i_, r_, s_ = _info(256)
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve_noalloc(op, P, mus, B, Xo, i_, r_, s_)
    assert e.value.status == nys.NYS_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int(s_[0]) == 99  # nothing was enqueued
    # the host-polled form is not offered without a workspace
    o = nys._opts(1e-10, 10, 0, 10, 1, 1e-4, device_info=0)
    info = nys._Info(None, None, None, 0, 0)
    mu_arr = (ctypes.c_double * 1)(0.1)
    Xs = torch.zeros(n, 1, dtype=torch.float64, device=DEV)
    code = nys.lib().nys_pcg_solve_noalloc(ctypes.byref(op.c()), ctypes.byref(P.c()), mu_arr, 1, nys._ptr(B), 1, 1,
                                           nys._ptr(Xs), 1, ctypes.byref(o), ctypes.byref(info), nys._stream())
    assert code == nys.NYS_ERR_ARG
    assert nys.lib().nys_noalloc_scratch_bytes() == 64 << 20
