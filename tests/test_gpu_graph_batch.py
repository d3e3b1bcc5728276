"""Batched solves in one captured graph: the device-info forms of the block
solve (a mu grid x right-hand sides sharing one RBF preconditioner; stopped
column blocks skip their kernel products) and of the ragged batch of ridge
problems, captured together with torch.cuda.graph and replayed.

Every replay must equal the eager device-info calls on the same inputs bit
for bit, and every column / problem must meet the tolerance on the float64
oracle's residual.  The ragged device-info form is also checked on its own
(float64 and float32 + float64 refinement) against the oracle."""
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


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def h(t):
    return t.detach().double().cpu().numpy()


def _info(k):
    return (torch.zeros(k, dtype=torch.int32, device=DEV), torch.zeros(k, dtype=torch.float64, device=DEV),
            torch.full((k,), 99, dtype=torch.int32, device=DEV))


def _ragged(sizes, seed, prec):
    probs, ops, Ps = [], [], []
    for q, (m, n) in enumerate(sizes):
        w = ridge_dense(m=m, n=n, ell=max(8, 16 * -(-n // 128)), seed=seed + q)
        X = w["X"] if prec else w["X"].astype(np.float64)
        p = dict(X=X, b=X.astype(np.float64).T @ w["y"], mu=w["mu"] * (1 + q), ell=w["ell"])
        op = nys.Operator.xtx(t32(X) if prec else t64(X))
        Om, Y = nys.nys_sketch(op, p["ell"], omega0=t64(w["omega0"]), prec=prec)
        Ps.append(nys.nys_factor(Om, Y, dtype=torch.float32 if prec else torch.float64, prec=prec))
        ops.append(op)
        probs.append(p)
    return probs, ops, Ps


@pytest.mark.parametrize("prec", [0, 2])
def test_ragged_device_info_meets_oracle(prec):
    sizes = [(1200, 301), (800, 200), (2000, 513), (600, 150), (900, 64)]
    probs, ops, Ps = _ragged(sizes, 80, prec)
    Bs = [t64(p["b"]) for p in probs]
    Xs = [torch.zeros_like(b) for b in Bs]
    it, rr, st = _info(len(probs))
    maxit = 400 if prec == 0 else 120
    steps, total = nys.nys_pcg_solve_ragged_device(ops, Ps, [p["mu"] for p in probs], Bs, Xs, it, rr, st,
                                                   tol=1e-10, maxit=maxit, prec=prec, max_refine=5, inner_tol=1e-5)
    torch.cuda.synchronize()
    assert (steps, total) == ((0, maxit) if prec == 0 else (5, 5 * maxit))
    for q, p in enumerate(probs):
        true = oracle.true_relres(oracle.XtXOp(p["X"]), p["mu"], h(Xs[q]), p["b"])
        assert int(st[q]) == nys.NYS_OK and true <= 1.02e-10, (q, int(st[q]), true)
        assert abs(float(rr[q]) - true) <= 1e-12
        assert 0 < int(it[q]) <= maxit * max(steps, 1)
    if prec == 0:  # same iteration counts as the host-polled batch (within 5%)
        _, info = nys.nys_pcg_solve_ragged(ops, Ps, [p["mu"] for p in probs], Bs, tol=1e-10, maxit=maxit)
        for q in range(len(probs)):
            assert abs(int(it[q]) - info.iters[q]) <= max(2, info.iters[q] // 20)


def test_block_and_ragged_in_one_graph():
    prec = nys.NYS_PREC_FP32_REFINE64
    # block part: RBF operator, 4 mu x 2 right-hand sides = 8 columns
    w = krr_small(n=700, d=8, ell=40, seed=81)
    opr = oracle.RBFOp(np.asarray(w["X"], dtype=np.float32), w["sigma"])
    b0 = opr.matmat(w["w"]) + w["noise"] * w["eps"]
    B0 = np.stack([b0, np.random.default_rng(82).standard_normal(700)], axis=1)
    mus = [1e-3, 1e-2, 1e-1, 1.0]
    op = nys.Operator.rbf(t32(w["X"]), w["sigma"])
    P = nys.nys_factor(*nys.nys_sketch(op, 40, omega0=t64(w["omega0"]), prec=prec), dtype=torch.float32, prec=prec)
    k = len(mus) * 2
    kwb = dict(tol=1e-10, maxit=150, prec=prec, max_refine=6, inner_tol=1e-3, ws=nys.workspace(op, 40, k, prec))
    Bc = t64(B0)
    Xc = torch.zeros(700, k, dtype=torch.float64, device=DEV)
    ib, rb, sb = _info(k)
    # ragged part: 4 ridge problems
    probs, rops, rPs = _ragged([(1000, 250), (700, 180), (1500, 400), (600, 96)], 83, prec)
    rmus = [p["mu"] for p in probs]
    Brs = [t64(p["b"]) for p in probs]
    Xrs = [torch.zeros_like(b) for b in Brs]
    ir, rr, sr = _info(len(probs))
    cops = [o for o in rops]
    wsr = torch.empty(nys.lib().nys_workspace_size_ragged(
        (nys._Operator * 4)(*[o.c() for o in cops]), (nys._Precond * 4)(*[p.c() for p in rPs]), 4, prec),
        dtype=torch.uint8, device=DEV)
    kwr = dict(tol=1e-10, maxit=120, prec=prec, max_refine=5, inner_tol=1e-5, ws=wsr)

    def body():
        Xc.zero_()
        for x in Xrs:
            x.zero_()
        nys.nys_pcg_solve_device(op, P, mus, Bc, Xc, ib, rb, sb, **kwb)
        nys.nys_pcg_solve_ragged_device(rops, rPs, rmus, Brs, Xrs, ir, rr, sr, **kwr)

    body()  # eager warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    rng = np.random.default_rng(84)
    for rep in range(3):
        Bn = B0 * (1.0 + rep) + (rep > 0) * rng.standard_normal(B0.shape)
        bns = [p["b"] * (1.0 + 0.5 * rep) for p in probs]
        Bc.copy_(t64(Bn))
        for x, bn in zip(Brs, bns):
            x.copy_(t64(bn))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Xg, Xrg = h(Xc), [h(x) for x in Xrs]
        infos = [t.clone() for t in (ib, rb, sb, ir, rr, sr)]
        # eager references on their own buffers
        Xe = torch.zeros(700, k, dtype=torch.float64, device=DEV)
        ie = _info(k)
        nys.nys_pcg_solve_device(op, P, mus, t64(Bn), Xe, *ie, **kwb)
        Xre = [torch.zeros(len(bn), dtype=torch.float64, device=DEV) for bn in bns]
        ire = _info(4)
        nys.nys_pcg_solve_ragged_device(rops, rPs, rmus, [t64(bn) for bn in bns], Xre, *ire, **kwr)
        torch.cuda.synchronize()
        assert np.array_equal(Xg, h(Xe))
        for a, e in zip(Xrg, Xre):
            assert np.array_equal(a, h(e))
        for got, ref in zip(infos, list(ie) + list(ire)):
            assert torch.equal(got, ref)
        for m, mu in enumerate(mus):
            for r in range(2):
                c = m * 2 + r
                assert int(infos[2][c]) == nys.NYS_OK
                assert oracle.true_relres(opr, mu, Xg[:, c], Bn[:, r]) <= 1.02e-10
        for q, p in enumerate(probs):
            assert int(infos[5][q]) == nys.NYS_OK
            assert oracle.true_relres(oracle.XtXOp(p["X"]), p["mu"], Xrg[q], bns[q]) <= 1.02e-10
