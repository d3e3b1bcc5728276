"""Benchmark: Nystrom PCG solves/s on one MI355X at a true float64 relative
residual of 1e-10 for the chosen form next to the plain float64 GPU path,
with the roofline of the dominant kernel and the CPU oracle as a baseline.

Default workload ("ridge"): dense ridge regression, X = G diag(j^-1/2) stored
in float32 (20000 x 4000, G ~ N(0, 1/20000)), A = X^T X, b = X^T y, mu = 1e-4,
l = 500; chosen form = float32 inner PCG + float64 residual refinement.  One
step = one whole solve: Gaussian test matrix, sketch Y = A Omega, shifted
Cholesky + SVD factorisation, PCG to 1e-10.

Other workloads (--workload): krr_small (n = 2048, d = 8, l = 100, float64),
krr (n = 1e5, d = 32, l = 1000, bf16x3 Gram tiles + refinement), batched
(one RBF sketch, 32 mu x 8 right-hand sides, plus 64 ragged ridge problems),
diff (validation-loss gradient through the RBF solve), adaptive (the ridge
system with the sketch size chosen by adaptive rank selection), sketch_solve
(Nystrom sketch-and-solve on the krr_small system: its accuracy and rate
against PCG's), block (coupled block PCG on 8 right-hand sides of the
krr_small system against the independent-column solve).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                [--no-plain] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG solves/s + matvec %roofline at rel-res 1e-10, chosen vs plain FP64 GPU"
HBM_PEAK_GBS = 8000.0
# v_exp_f32 issue rate: 256 CUs x 4 SIMDs x 4 lanes/clk (quarter rate) x 2.4 GHz
EXP_PEAK_GPS = 256 * 4 * 4 * 2.4


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xtx_fused_ridge_20000x4000_pmc.txt")
XTX_SOURCE = os.path.join(ROOT, "paper_2110_02820_amd", "csrc", "xtx.hip")


def measured_traffic():
    """HBM bytes per launch of the float32 X^T X product kernel (xtx_fused),
    from the committed FETCH_SIZE / WRITE_SIZE counter summary; None when the
    summary is missing or the kernel source has changed since the counters
    were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
        with open(XTX_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if kv.get("kernel_source_sha256", "").strip() != sha:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ridge",
                    choices=["ridge", "krr_small", "krr", "krr_cols", "batched", "diff", "adaptive",
                             "sketch_solve", "block", "weighted"])
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=30)
    ap.add_argument("--n", type=int, default=0, help="override the system size (reduced runs)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="relative tolerance of each float32 inner solve (0: the workload's default)")
    ap.add_argument("--prec", default="", choices=["", "fp32_refine64", "bf16x3_refine64"],
                    help="ridge: precision mode of the chosen form (empty: the workload's default)")
    ap.add_argument("--graph", action="store_true",
                    help="batched: every PCG solve of a step (block + ragged, device-info forms) replayed as one "
                         "captured graph; sketches and factors stay eager")
    ap.add_argument("--graph-maxit", type=int, default=400, help="batched --graph: block iterations per step")
    ap.add_argument("--graph-refine", type=int, default=8, help="batched --graph: block refinement steps")
    ap.add_argument("--autotune", action="store_true",
                    help="batched / krr: run the block-product autotuner before the timed region")
    ap.add_argument("--kernel-only", action="store_true",
                    help="ridge: only the X^T X product (and a 256 MiB device copy as the counter "
                         "calibration), for hardware-counter runs")
    return ap.parse_args()


class Timer:
    """Phase times from events recorded on the current stream at the end of
    each phase: nothing synchronises inside the timed region, so the host
    enqueues the next phase while the device still runs the last one.  A
    phase runs from the previous event (or the timer's creation) to its own;
    reading .t synchronises once and returns seconds per phase."""

    def __init__(self, torch):
        self.torch = torch
        self.ev = []
        self.last = self._event()

    def _event(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def lap(self, key, t0):
        e = self._event()
        self.ev.append((key, self.last, e))
        self.last = e
        return time.perf_counter()

    @property
    def t(self):
        self.torch.cuda.synchronize()
        out = {}
        for key, a, b in self.ev:
            out[key] = out.get(key, 0.0) + 1e-3 * a.elapsed_time(b)
        return out


def full_solve(nys, torch, op, ell, seed, prec, udtype, mus, B, ws, tol, timer, cols=None, **kw):
    """cols = (device index tensor, workspace): column-sampling sketch instead
    of the Gaussian one (its Y is float64, so the factor takes the float64 shift)."""
    t = time.perf_counter()
    if cols is None:
        Om, Y = nys.nys_sketch(op, ell, seed=seed, prec=prec, ws=ws)
        fprec = prec
    else:
        Om, Y = nys.nys_sketch_columns(op, cols[0], ws=cols[1])
        fprec = nys.NYS_PREC_FP64
    t = timer.lap("sketch", t)
    P = nys.nys_factor(Om, Y, dtype=udtype, ws=ws, prec=fprec)
    del Om, Y
    t = timer.lap("factor", t)
    X, info = nys.nys_pcg_solve(op, P, mus, B, tol=tol, prec=prec, ws=ws, **kw)
    timer.lap("pcg", t)
    return X, info, P


def kernel_avg_ms(torch, fn, reps):
    for _ in range(2):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cores_used():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return os.cpu_count()


def base_record(args, value, ms, dtype, config, extra):
    out = {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    return out


# --------------------------------------------------------------------------- ridge (default)

def run_ridge(args, nys, torch):
    from workloads import ridge_dense
    dev = "cuda:0"
    m, n, ell = 20000, (args.n or 4000), 500
    w = ridge_dense(m=m, n=n, ell=ell, with_omega=False)
    X32h = w["X"]
    b_h = X32h.astype(np.float64).T @ w["y"]  # input synthesis (host, float64)
    mu, tol = w["mu"], 1e-10
    X32 = torch.as_tensor(X32h, device=dev)
    b = torch.as_tensor(b_h, device=dev)
    op = nys.Operator.xtx(X32)
    # default: sketch products on bf16 MFMA (hi/lo split; the preconditioner
    # needs no more), float32 inner PCG, float64 refinement and factorisation
    bf = args.prec != "fp32_refine64"
    prec = nys.NYS_PREC_BF16X3_REFINE64 if bf else nys.NYS_PREC_FP32_REFINE64
    ws = nys.workspace(op, ell, 1, prec)
    # each float32 inner solve to about sqrt(tol) / 3: two refinement steps
    # reach tol with margin (float32 PCG gets to ~1e-6 here before rounding)
    kw = dict(maxit=1000, inner_tol=args.inner_tol or 3e-6)

    def timed(opx, precx, wsx, udtype, steps, warmup, label):
        for i in range(warmup):
            full_solve(nys, torch, opx, ell, 1000 + i, precx, udtype, mu, b, wsx, tol, Timer(torch), **kw)
        tm = Timer(torch)
        infos = []
        t = time.perf_counter()
        for i in range(steps):
            a = time.perf_counter()
            _, info, P = full_solve(nys, torch, opx, ell, 20211002 + i, precx, udtype, mu, b, wsx, tol, tm, **kw)
            infos.append(info)
            log("%s step %d: %.2f ms, iters %d, refine %d, relres %.2e" %
                (label, i, 1e3 * (time.perf_counter() - a), info.iters[0], info.refine_steps, info.relres[0]))
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        return el, {k: 1e3 * v / steps for k, v in tm.t.items()}, infos, P

    el, phases, infos, P_last = timed(op, prec, ws, torch.float32, args.steps, args.warmup, "chosen")
    # the regime where one preconditioner serves many solves (a mu path or new
    # right-hand sides): PCG solves alone, reusing the last step's factor
    torch.cuda.synchronize()
    t = time.perf_counter()
    pinfos = [nys.nys_pcg_solve(op, P_last, mu, b, tol=tol, prec=prec, ws=ws, **kw)[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    el_pcg = time.perf_counter() - t
    del P_last
    v32 = torch.randn(n, dtype=torch.float32, device=dev)
    wsm = nys.workspace(op, 1, 1, nys.NYS_PREC_FP64)
    # the dominant kernel's launch duration from HIP events the library records
    # on its stream around each launch; the whole product (with its column
    # reduction and launch gaps) is timed alongside
    nys.timing_begin()
    prod_ms = kernel_avg_ms(torch, lambda: nys.nys_op_apply(op, mu, v32, ws=wsm), args.matvec_reps)
    mv_ms, launches = nys.timing_end()
    alg_bytes = m * n * 4 + 2 * n * 4  # X once + p in + v out
    achieved = alg_bytes / (mv_ms * 1e-3) / 1e9
    out = base_record(
        args, args.steps / el, 1e3 * el / args.steps, "bf16x3+f32+f64" if bf else "f32+f64",
        {"workload": "ridge regression A = X^T X, X %dx%d float32 = G diag(j^-1/2), mu=1e-4, l=%d, b = X^T y, "
                     "tol 1e-10 (true float64 residual)" % (m, n, ell),
         "precision": ("sketch products on bf16 MFMA (hi/lo split), " if bf else "float32 sketch products, ") +
                      "float32 inner PCG + float64 residual refinement; float64 core factorisation",
         "step": "Gaussian Omega + sketch + factor + PCG solve"},
        {"correct": all(i.relres[0] <= tol and i.status[0] == 0 for i in infos),
         "relres": max(i.relres[0] for i in infos), "iters": infos[-1].iters[0],
         "refine_steps": infos[-1].refine_steps, "phase_ms": phases,
         "pcg_only": {"value": args.steps / el_pcg, "unit": "solves/s", "ms_per_solve": 1e3 * el_pcg / args.steps,
                      "note": "PCG solves to 1e-10 reusing one factor (sketch and factor not repeated)",
                      "correct": all(i.relres[0] <= tol and i.status[0] == 0 for i in pinfos)},
         "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                      "kernel": "xtx_fused<float,float> (one pass over X: X^T (X p) partial sums)",
                      "avg_ms": mv_ms, "launches_timed": launches, "alg_bytes": alg_bytes,
                      "product_avg_ms": prod_ms,
                      "product_note": "the whole product (xtx_fused + reduce_cols, launch gaps included)"}})
    if not args.no_plain:
        X64 = X32.double()
        op64 = nys.Operator.xtx(X64)
        ws64 = nys.workspace(op64, ell, 1, nys.NYS_PREC_FP64)
        n64 = max(1, min(args.steps, 3))
        el64, ph64, inf64, _ = timed(op64, nys.NYS_PREC_FP64, ws64, torch.float64, n64, 1, "plain")
        out["plain_fp64"] = {"value": n64 / el64, "unit": "solves/s", "ms_per_step": 1e3 * el64 / n64,
                             "phase_ms": ph64, "iters": inf64[-1].iters[0], "relres": inf64[-1].relres[0],
                             "correct": all(i.relres[0] <= tol for i in inf64)}
        out["speedup_vs_plain_fp64"] = out["value"] / out["plain_fp64"]["value"]
        del X64, op64, ws64
    if not args.no_cpu_baseline:
        import oracle
        from workloads import gaussian_test_matrix
        opr = oracle.XtXOp(X32h)
        om0 = gaussian_test_matrix(n, ell, 7)
        # whole solves, repeated until about 10 s of host time have been spent
        reps = 0
        t = time.perf_counter()
        while True:
            r = oracle.randomized_nystrom(opr, om0)
            o = oracle.nystrom_pcg(opr.matmat, b_h, mu,
                                   lambda v: oracle.precond_inv_apply(r["U"], r["lam"], mu, v), tol=tol, maxit=1000)
            reps += 1
            el = time.perf_counter() - t
            if el >= 10.0 or reps >= 30:
                break
        out["cpu_baseline"] = {"value": reps / el, "unit": "solves/s", "cores": cores_used(), "kind": "oracle",
                               "sample": "%d full solves of the same workload (sketch + factor + PCG to 1e-10), "
                                         "numpy float64" % reps, "seconds": el, "iters": o["iters"]}
    return out


def run_ridge_kernel(args, nys, torch):
    """The dominant kernel alone: float32 (X^T X + mu I) p on the ridge workload, then a
    plain device copy of 256 MiB whose counter readings calibrate FETCH_SIZE / WRITE_SIZE."""
    from workloads import ridge_dense
    dev = "cuda:0"
    m, n = 20000, (args.n or 4000)
    w = ridge_dense(m=m, n=n, ell=8, with_omega=False)
    op = nys.Operator.xtx(torch.as_tensor(w["X"], device=dev))
    v32 = torch.randn(n, dtype=torch.float32, device=dev)
    wsm = nys.workspace(op, 1, 1, nys.NYS_PREC_FP64)
    mv_ms = kernel_avg_ms(torch, lambda: nys.nys_op_apply(op, w["mu"], v32, ws=wsm), args.matvec_reps)
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    cp_ms = kernel_avg_ms(torch, lambda: dst.copy_(src), 10)
    return {"kernel": "xtx_fused<float,float> + reduce_cols", "avg_ms": mv_ms, "reps": args.matvec_reps + 2,
            "alg_bytes": m * n * 4 + 2 * n * 4, "copy_bytes_each_way": src.numel() * 4, "copy_avg_ms": cp_ms,
            "copy_reps": 12}


# --------------------------------------------------------------------------- adaptive rank

def run_adaptive(args, nys, torch):
    """The ridge system with l chosen by adaptive rank selection (Strategy 1
    with the theorem's two conditions, tau = 44 as in its corollary, q = 10
    power steps), l0 = 64 doubling up to l_max = 2048, then the PCG solve."""
    from workloads import ridge_dense
    dev = "cuda:0"
    m, n = 20000, (args.n or 4000)
    l0, lmax, tau, q = 64, min(2048, n), 44.0, 10
    w = ridge_dense(m=m, n=n, ell=8, with_omega=False)
    X32h = w["X"]
    b_h = X32h.astype(np.float64).T @ w["y"]
    mu, tol = w["mu"], 1e-10
    op = nys.Operator.xtx(torch.as_tensor(X32h, device=dev))
    b = torch.as_tensor(b_h, device=dev)
    prec = nys.NYS_PREC_BF16X3_REFINE64
    wsa = nys.workspace_adaptive(op, lmax, prec)
    kw = dict(maxit=1000, inner_tol=args.inner_tol or 3e-6)
    wss = {}

    def step(seed):
        tm = Timer(torch)
        t = time.perf_counter()
        P, info = nys.nys_nystrom_adaptive(op, l0, lmax, mu, tau=tau, q=q, criterion=nys.NYS_ADA_ERR_LAM,
                                           seed=seed, prec=prec, dtype=torch.float32, ws=wsa)
        t = tm.lap("adaptive_nystrom", t)
        ell = info["ell"]
        if ell not in wss:
            wss[ell] = nys.workspace(op, ell, 1, prec)
        X, sinfo = nys.nys_pcg_solve(op, P, mu, b, tol=tol, prec=prec, ws=wss[ell], **kw)
        tm.lap("pcg", t)
        return info, sinfo, tm

    for i in range(args.warmup):
        step(1000 + i)
    t = time.perf_counter()
    runs = []
    for i in range(args.steps):
        info, sinfo, tm = step(20211002 + i)
        runs.append((info, sinfo, tm))
        log("adaptive step %d: l=%d E=%.3e capped=%s iters %d relres %.2e %s" %
            (i, info["ell"], info["err"], info["capped"], sinfo.iters[0], sinfo.relres[0],
             {k: round(1e3 * v, 2) for k, v in tm.t.items()}))
    el = time.perf_counter() - t
    out = base_record(
        args, args.steps / el, 1e3 * el / args.steps, "bf16x3+f32+f64",
        {"workload": "ridge regression A = X^T X, X %dx%d float32 = G diag(j^-1/2), mu=1e-4, b = X^T y, tol 1e-10; "
                     "l by adaptive rank selection: l0=%d doubling to l_max=%d until ||E|| <= tau mu and "
                     "lam_l <= tau mu / 11, tau=%g, q=%d power steps" % (m, n, l0, lmax, tau, q),
         "precision": "sketch products on bf16 MFMA (hi/lo split), float32 power-step products and inner PCG, "
                      "float64 refinement and core factorisations",
         "step": "adaptive sketch/factor/estimate stages + PCG solve"},
        {"correct": all(s.relres[0] <= tol and s.status[0] == 0 for _, s, _ in runs),
         "ell": runs[-1][0]["ell"], "err_estimate": runs[-1][0]["err"], "capped": runs[-1][0]["capped"],
         "iters": runs[-1][1].iters[0], "refine_steps": runs[-1][1].refine_steps,
         "phase_ms": {k: 1e3 * sum(r[2].t.get(k, 0.0) for r in runs) / args.steps for k in runs[0][2].t}})
    if not args.no_cpu_baseline:
        import oracle
        opr = oracle.XtXOp(X32h)
        db = lambda j, mm: oracle.gaussian_philox(7 + 2 * j, n, mm)
        dg = lambda j: oracle.gaussian_philox(8 + 2 * j, n, 1)[:, 0]
        t = time.perf_counter()
        r = oracle.ada_rand_nystrom(opr, l0, lmax, q, tau, mu, db, dg, criterion="err_lam")
        o = oracle.nystrom_pcg(opr.matmat, b_h, mu, lambda v: oracle.precond_inv_apply(r["U"], r["lam"], mu, v),
                               tol=tol, maxit=1000)
        el = time.perf_counter() - t
        out["cpu_baseline"] = {"value": 1.0 / el, "unit": "solves/s", "cores": cores_used(), "kind": "oracle",
                               "sample": "one full adaptive solve of the same workload (stages + PCG to 1e-10), "
                                         "numpy float64", "seconds": el, "ell": r["ell"], "iters": o["iters"]}
    return out


# --------------------------------------------------------------------------- sketch-and-solve

def run_sketch_solve(args, nys, torch):
    """Nystrom sketch-and-solve on the krr_small system (n = 2048, d = 8,
    mu = 1e-3) at l = 100, 400, 1600: time per solve (sketch + factor +
    Woodbury solve) and the true float64 relative residual it reaches, next to
    Nystrom PCG at l = 100.  Sketch-and-solve never reaches 1e-10 here (the
    paper's point), so its rate is not a solve rate at the metric's tolerance:
    `value` is PCG's."""
    from workloads import krr_small
    dev = "cuda:0"
    n = args.n or 2048
    w = krr_small(n=n, d=8, ell=100)
    X = torch.as_tensor(w["X"], dtype=torch.float64, device=dev)
    op = nys.Operator.rbf(X, w["sigma"])
    b = rbf_rhs(nys, torch, op, w, dev)
    mu, tol = w["mu"], 1e-10
    bn = float(torch.linalg.norm(b))
    res = {}
    for ell in (100, 400, 1600):
        ws = nys.workspace(op, ell, 1, nys.NYS_PREC_FP64)
        for i in range(args.warmup):
            Om, Y = nys.nys_sketch(op, ell, seed=1000 + i, ws=ws)
            nys.nys_sketch_solve(nys.nys_factor(Om, Y, ws=ws), mu, b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(args.steps):
            Om, Y = nys.nys_sketch(op, ell, seed=20211001 + i, ws=ws)
            P = nys.nys_factor(Om, Y, ws=ws)
            x = nys.nys_sketch_solve(P, mu, b)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / args.steps
        r = b - nys.nys_op_apply(op, mu, x)
        res[ell] = {"ms_per_solve": 1e3 * el, "solves_per_s": 1.0 / el, "relres": float(torch.linalg.norm(r)) / bn}
        log("sketch-and-solve l=%d: %.2f ms, relres %.2e" % (ell, 1e3 * el, res[ell]["relres"]))
    ws = nys.workspace(op, 100, 1, nys.NYS_PREC_FP64)
    tm = Timer(torch)
    t = time.perf_counter()
    for i in range(args.steps):
        _, info, _ = full_solve(nys, torch, op, 100, 20211001 + i, nys.NYS_PREC_FP64, torch.float64, mu, b, ws, tol,
                                tm, maxit=5000)
    el = time.perf_counter() - t
    return base_record(
        args, args.steps / el, 1e3 * el / args.steps, "f64",
        {"workload": "kernel ridge regression, RBF n=%d d=8 sigma=sqrt(8), mu=1e-3: Nystrom sketch-and-solve at "
                     "l = 100, 400, 1600 against Nystrom PCG at l = 100 (value: PCG to 1e-10)" % n,
         "precision": "float64",
         "step": "Gaussian Omega + sketch + factor + (Woodbury solve | PCG solve)"},
        {"correct": info.relres[0] <= tol, "pcg_relres": info.relres[0], "pcg_iters": info.iters[0],
         "sketch_and_solve": {str(k): v for k, v in res.items()},
         "sketch_and_solve_reaches_tol": any(v["relres"] <= tol for v in res.values())})


# --------------------------------------------------------------------------- weighted (ALOOCV operator)

def run_weighted(args, nys, torch):
    """The ALOOCV operator X^T D X + mu I on the ridge data (X 20000 x 4000
    float32, l = 500, mu = 1e-4) with seeded logistic Hessian weights
    d = p (1 - p): the X^T X operator with float64 row weights applied inside
    every product, whole solves in the ridge line's chosen form; the float64
    refinement residuals use the float64 weights, so the tolerance holds for
    X^T D X itself (checked by the oracle after the timed region)."""
    from workloads import logistic_weights, ridge_dense
    dev = "cuda:0"
    m, n, ell = 20000, (args.n or 4000), 500
    w = ridge_dense(m=m, n=n, ell=ell, with_omega=False)
    d_h = logistic_weights(m)
    X = torch.as_tensor(w["X"], device=dev)
    d = torch.as_tensor(d_h, device=dev)
    # right-hand side X^T D y (input synthesis on the host, float64)
    b_h = w["X"].astype(np.float64).T @ (d_h * w["y"])
    b = torch.as_tensor(b_h, device=dev)
    mu, tol = w["mu"], 1e-10
    op = nys.Operator.xtdx(X, d)
    prec = nys.NYS_PREC_BF16X3_REFINE64
    ws = nys.workspace(op, ell, 1, prec)
    kw = dict(maxit=1000, inner_tol=3e-6)
    for i in range(args.warmup):
        full_solve(nys, torch, op, ell, 1000 + i, prec, torch.float32, mu, b, ws, tol, Timer(torch), **kw)
    tm = Timer(torch)
    infos = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        x, info, _ = full_solve(nys, torch, op, ell, 20211002 + i, prec, torch.float32, mu, b, ws, tol, tm, **kw)
        infos.append(info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    # the oracle's float64 residual of the last solution on X^T D X (outside the timed region)
    import oracle
    rr_or = oracle.true_relres(oracle.XtDXOp(w["X"], d_h), mu, x.cpu().numpy().reshape(-1), b_h)
    return base_record(
        args, args.steps / el, 1e3 * el / args.steps, "bf16x3+f32+f64",
        {"workload": "ALOOCV operator X^T D X + mu I, X %dx%d float32 (ridge data), d = p(1-p) logistic weights "
                     "(float64), mu=1e-4, l=%d, tol 1e-10 (true float64 residual of X^T D X)" % (m, n, ell),
         "precision": "row weights inside every product (float64 in the refinement residuals, float32 in the "
                      "inner products); then the ridge line's chosen form",
         "step": "Gaussian Omega + sketch + factor + PCG solve"},
        {"correct": all(i.relres[0] <= tol and i.status[0] == 0 for i in infos) and rr_or <= 1.01 * tol,
         "relres": max(i.relres[0] for i in infos), "oracle_relres_last": rr_or, "iters": infos[-1].iters[0],
         "refine_steps": infos[-1].refine_steps, "phase_ms": {k: 1e3 * v / args.steps for k, v in tm.t.items()}})


# --------------------------------------------------------------------------- block PCG

def run_block(args, nys, torch):
    """Coupled block Nystrom PCG (O'Leary) for 8 right-hand sides sharing mu
    on the krr_small system (n = 2048, d = 8, l = 100, mu = 1e-3), float64,
    next to the same 8 columns solved independently (nys_pcg_solve)."""
    from workloads import krr_small
    dev = "cuda:0"
    n, s, ell = (args.n or 2048), 8, 100
    w = krr_small(n=n, d=8, ell=ell)
    X = torch.as_tensor(w["X"], dtype=torch.float64, device=dev)
    op = nys.Operator.rbf(X, w["sigma"])
    mu, tol = w["mu"], 1e-10
    B = torch.as_tensor(np.random.default_rng(20211006).standard_normal((n, s)), device=dev)
    ws = nys.workspace(op, ell, s, nys.NYS_PREC_FP64)
    import ctypes
    wsb = torch.empty(nys.lib().nys_workspace_size_block(ctypes.byref(op.c()), ell, s), dtype=torch.uint8,
                      device=dev)

    def one(seed, block, tm):
        t = time.perf_counter()
        Om, Y = nys.nys_sketch(op, ell, seed=seed, ws=ws)
        P = nys.nys_factor(Om, Y, ws=ws)
        t = tm.lap("sketch_factor", t)
        if block:
            Xs, info = nys.nys_block_pcg_solve(op, P, mu, B, tol=tol, maxit=5000, ws=wsb)
        else:
            Xs, info = nys.nys_pcg_solve(op, P, mu, B, tol=tol, maxit=5000, ws=ws)
        tm.lap("pcg", t)
        return Xs, info

    out = {}
    for block in (True, False):
        for i in range(args.warmup):
            one(1000 + i, block, Timer(torch))
        tm = Timer(torch)
        t = time.perf_counter()
        for i in range(args.steps):
            Xs, info = one(20211001 + i, block, tm)
        el = time.perf_counter() - t
        R = B - nys.nys_op_apply(op, mu, Xs)
        rel = (torch.linalg.norm(R, dim=0) / torch.linalg.norm(B, dim=0)).max().item()
        out[block] = {"solves_per_s": s * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                      "iters": max(info.iters), "true_relres_max": rel,
                      "phase_ms": {k: 1e3 * v / args.steps for k, v in tm.t.items()}}
        log("%s: %.2f ms per 8 solves, iters %d, relres %.2e" % ("block" if block else "independent",
                                                                  1e3 * el / args.steps, max(info.iters), rel))
    b = out[True]
    return base_record(
        args, b["solves_per_s"], b["ms_per_step"], "f64",
        {"workload": "coupled block PCG: RBF n=%d d=8 sigma=sqrt(8), mu=1e-3, l=%d, 8 right-hand sides N(0,1), "
                     "tol 1e-10" % (n, ell),
         "precision": "float64",
         "step": "Gaussian Omega + sketch + factor + block PCG for all 8 columns"},
        {"correct": b["true_relres_max"] <= 1.01 * tol, "block": b, "independent_columns": out[False]})


# --------------------------------------------------------------------------- RBF helpers

def rbf_rhs(nys, torch, op, w, dev):
    """b = K w + 0.01 eps on the device (float64 product of the stored points)."""
    wv = torch.as_tensor(w["w"], device=dev)
    Kw = nys.nys_op_apply(op, 0.0, wv)
    return Kw + w["noise"] * torch.as_tensor(w["eps"], device=dev)


def rbf_cpu_sample(w, ell, nvec=1):
    """The float64 CPU oracle on a bounded sample of the RBF products: one
    2048-row block of K (the oracle's own block size) times l columns and
    times nvec columns.  Returns the extrapolated whole-matrix times
    (n / 2048 blocks) for the sketch product and for one PCG product."""
    import oracle
    opr = oracle.RBFOp(w["X"], w["sigma"])
    n = opr.n
    blk = min(2048, n)
    rng = np.random.default_rng(3)
    V = rng.standard_normal((n, ell))
    v = rng.standard_normal((n, nvec))
    idx = np.arange(blk)
    t = time.perf_counter()
    opr.rows(idx) @ V
    t_sk = (time.perf_counter() - t) * n / blk
    t = time.perf_counter()
    opr.rows(idx) @ v
    t_mv = (time.perf_counter() - t) * n / blk
    return t_sk, t_mv


def run_krr(args, nys, torch, small=False, columns=False):
    from workloads import column_sample, krr_mixture, krr_small
    dev = "cuda:0"
    if small:
        n, d, ell = (args.n or 2048), 8, 100
        w = krr_small(n=n, d=d, ell=ell)
        X = torch.as_tensor(w["X"], dtype=torch.float64, device=dev)
        prec, udtype, label = nys.NYS_PREC_FP64, torch.float64, "f64"
        mu = w["mu"]
        kw = dict(maxit=5000)
    else:
        n, d, ell = (args.n or 100000), 32, 1000
        w = krr_mixture(n=n, d=d, ell=ell, with_omega=False)
        X = torch.as_tensor(w["X"], device=dev)
        prec, udtype, label = nys.NYS_PREC_BF16X3_REFINE64, torch.float32, "bf16x3+f32+f64"
        mu = w["mu"]
        kw = dict(maxit=5000, max_refine=40, inner_tol=args.inner_tol or 3e-3)
    tol = 1e-10
    op = nys.Operator.rbf(X, w["sigma"])
    b = rbf_rhs(nys, torch, op, w, dev)
    ws = nys.workspace(op, ell, 1, prec)
    tuned = None
    if args.autotune and not small:
        t = time.perf_counter()
        nys.nys_autotune(op, prec, [ell])  # the sketch's block product (ell columns)
        tuned = {"seconds": time.perf_counter() - t, "choices": {ell: nys.nys_autotune_query(op, prec, ell)[:4]}}
        log("autotune: %s" % tuned)
    # column sampling: the index sets are inputs, drawn and uploaded before the timed steps
    cols = {}
    if columns:
        import ctypes
        wsc = torch.empty(nys.lib().nys_workspace_size_columns(ctypes.byref(op.c()), ell), dtype=torch.uint8,
                          device=dev)
        for sd in [1000 + i for i in range(args.warmup)] + [20211003 + i for i in range(args.steps)]:
            cols[sd] = (torch.as_tensor(column_sample(n, ell, sd), device=dev), wsc)
    for i in range(args.warmup):
        full_solve(nys, torch, op, ell, 1000 + i, prec, udtype, mu, b, ws, tol, Timer(torch),
                   cols=cols.get(1000 + i), **kw)
    tm = Timer(torch)
    infos = []
    t = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        _, info, _ = full_solve(nys, torch, op, ell, 20211003 + i, prec, udtype, mu, b, ws, tol, tm,
                                cols=cols.get(20211003 + i), **kw)
        infos.append(info)
        log("krr step %d: %.1f ms iters %d refine %d relres %.2e" % (i, 1e3 * (time.perf_counter() - a),
                                                                     info.iters[0], info.refine_steps,
                                                                     info.relres[0]))
    el = time.perf_counter() - t
    # dominant kernel: one single-vector product in the chosen arithmetic
    if small:
        v = torch.randn(n, dtype=torch.float64, device=dev)
        mv_ms = kernel_avg_ms(torch, lambda: nys.nys_op_apply(op, mu, v), args.matvec_reps)
        ev = n * n / (mv_ms * 1e-3) / 1e9
        # Gram on f64 MFMA; per entry the vector units spend ~32 float64
        # operations (exp, distance, compensated sum): 78.6 TFLOP/s / 64
        roof = {"bound": "alu", "achieved": ev, "peak": 78.6e3 / 64, "unit": "G kernel entries/s",
                "frac": ev / (78.6e3 / 64), "traffic": None,
                "kernel": "rbf_mv_f64m (f64 MFMA Gram; float64 exp + compensated sum, ~32 float64 ops "
                          "per entry)", "avg_ms": mv_ms}
    else:
        v = torch.randn(n, dtype=torch.float32, device=dev)
        mv_ms = kernel_avg_ms(torch, lambda: nys.nys_op_apply(op, mu, v, prec=prec), args.matvec_reps)
        # K is symmetric: the product evaluates each of its n (n + 1) / 2
        # distinct entries once, one v_exp_f32 each
        ev = n * (n + 1) / 2 / (mv_ms * 1e-3) / 1e9
        roof = {"bound": "alu", "achieved": ev, "peak": EXP_PEAK_GPS, "unit": "G exp/s",
                "frac": ev / EXP_PEAK_GPS, "traffic": None,
                "kernel": "rbf_mv_lowp_sym<bf16x3>: one v_exp_f32 per distinct kernel entry (n(n+1)/2 per product)",
                "entries_per_s": n * n / (mv_ms * 1e-3), "avg_ms": mv_ms}
    out = base_record(
        args, args.steps / el, 1e3 * el / args.steps, label,
        {"workload": ("kernel ridge regression, RBF n=%d d=%d sigma=sqrt(d), mu=%g, l=%d, tol 1e-10%s"
                      % (n, d, mu, ell, "; sketch from l uniformly sampled kernel columns" if columns else "")),
         "precision": "float64" if small else "bf16x3 Gram tiles on MFMA, float32 inner PCG, float64 refinement",
         "step": ("sampled kernel columns" if columns else "Gaussian Omega + sketch") +
                 " + factor + PCG solve"},
        {"correct": all(i.relres[0] <= tol and i.status[0] == 0 for i in infos),
         "relres": max(i.relres[0] for i in infos), "iters": infos[-1].iters[0],
         "refine_steps": infos[-1].refine_steps,
         "phase_ms": {k: 1e3 * v / args.steps for k, v in tm.t.items()}, "roofline": roof})
    if tuned is not None:
        out["autotune"] = tuned
    if not args.no_plain and not small and not columns:
        ws64 = nys.workspace(op, ell, 1, nys.NYS_PREC_FP64)
        tm64 = Timer(torch)
        t = time.perf_counter()
        _, inf64, _ = full_solve(nys, torch, op, ell, 7, nys.NYS_PREC_FP64, torch.float64, mu, b, ws64, tol, tm64,
                                 maxit=5000)
        el64 = time.perf_counter() - t
        out["plain_fp64"] = {"value": 1.0 / el64, "unit": "solves/s", "ms_per_step": 1e3 * el64,
                             "phase_ms": {k: 1e3 * v for k, v in tm64.t.items()}, "iters": inf64.iters[0],
                             "relres": inf64.relres[0], "correct": inf64.relres[0] <= tol}
        out["speedup_vs_plain_fp64"] = out["value"] / out["plain_fp64"]["value"]
    if not args.no_cpu_baseline:
        t_sk, t_mv = rbf_cpu_sample(w, ell)
        it = infos[-1].total_iters or infos[-1].iters[0]
        if columns:
            import oracle
            t = time.perf_counter()
            oracle.RBFOp(w["X"], w["sigma"]).rows(column_sample(n, ell, 5))
            t_sk = time.perf_counter() - t
        est = t_sk + it * t_mv
        out["cpu_baseline"] = {"value": 1.0 / est, "unit": "solves/s", "cores": cores_used(), "kind": "oracle",
                               "sample": ("oracle kernel rows at the l sampled points (the column sketch)"
                                          if columns else "oracle RBF row block (2048 rows of K) times l columns") +
                                         " and a 2048-row block times one column, scaled by n/2048; solve = sketch "
                                         "+ %d PCG products (the GPU run's count); factorisation not counted, so "
                                         "the CPU figure is an upper bound" % it,
                               "seconds_est": est}
    return out


# --------------------------------------------------------------------------- batched

def run_batched(args, nys, torch):
    from workloads import batched_cv
    dev = "cuda:0"
    n = args.n or 50000
    log("generating the batched workload (n=%d, 64 ragged problems)" % n)
    w = batched_cv(n=n, with_omega=False, with_ragged=True)
    log("inputs ready")
    tol = 1e-10
    X = torch.as_tensor(w["X"], device=dev)
    op = nys.Operator.rbf(X, w["sigma"])
    B = torch.as_tensor(w["B"], device=dev)
    mus = [float(m) for m in w["mus"]]
    ell = w["ell"]
    # float32 Gram tiles: at the smallest mu of the grid (n 1e-8) the bf16x3
    # perturbation of K exceeds mu and K + mu I is no longer definite
    prec = nys.NYS_PREC_FP32_REFINE64
    ws = nys.workspace(op, ell, len(mus) * B.shape[1], prec)
    rag = w["ragged"]
    rops, rbs = [], []
    for p in rag:
        Xk = torch.as_tensor(p["X"], device=dev)
        rops.append(nys.Operator.xtx(Xk))
        rbs.append(torch.as_tensor(p["X"].astype(np.float64).T @ p["y"], device=dev))

    tuned = None
    if args.autotune:
        t = time.perf_counter()
        ks = [8, 16, 32, 64, 128, 192, 256, ell]
        nys.nys_autotune(op, prec, ks)
        tuned = {"seconds": time.perf_counter() - t,
                 "choices": {k: nys.nys_autotune_query(op, prec, k)[:4] for k in ks}}
        log("autotune: %s" % tuned)
    if args.graph:
        return run_batched_graph(args, nys, torch, w, op, B, mus, ell, prec, ws, rops, rbs, rag, tol, tuned)

    def step(seed):
        tm = Timer(torch)
        t = time.perf_counter()
        Xs, info, _ = full_solve(nys, torch, op, ell, seed, prec, torch.float32, mus, B, ws, tol, tm, maxit=5000,
                                 max_refine=40, inner_tol=args.inner_tol or 3e-2)
        log("block solve: %s, iters max %d, refine %d" % ({k: round(1e3 * v, 1) for k, v in tm.t.items()},
                                                          max(info.iters), info.refine_steps))
        t = time.perf_counter()
        Ps = []
        for k, (o, p) in enumerate(zip(rops, rag)):
            Om, Y = nys.nys_sketch(o, p["ell"], seed=seed + k, prec=prec)
            Ps.append(nys.nys_factor(Om, Y, dtype=torch.float32, prec=prec))
        tm.lap("ragged_factor", t)
        log("ragged sketches + factors: %.1f ms" % (1e3 * tm.t["ragged_factor"]))
        t = time.perf_counter()
        Xr, rinfo = nys.nys_pcg_solve_ragged(rops, Ps, [p["mu"] for p in rag], rbs, tol=tol, prec=prec,
                                             maxit=1000)
        tm.lap("ragged_pcg", t)
        return info, rinfo, tm

    for i in range(args.warmup):
        step(100 + i)
    t = time.perf_counter()
    infos = []
    tms = []
    for i in range(args.steps):
        info, rinfo, tm = step(20211004 + i)
        infos.append((info, rinfo))
        tms.append(tm)
        log("batched step %d: %s; block iters max %d; ragged relres max %.2e" %
            (i, {k: round(1e3 * v, 1) for k, v in tm.t.items()}, max(info.iters), max(rinfo.relres)))
    el = time.perf_counter() - t
    nsolves = len(mus) * B.shape[1] + len(rag)
    ok = all(max(a.relres) <= tol and max(r.relres) <= tol for a, r in infos)
    phases = {k: 1e3 * sum(tm.t.get(k, 0.0) for tm in tms) / args.steps for k in tms[0].t}
    plain = None if args.no_plain else batched_plain_fp64(nys, torch, w, X, B, mus, rops, rbs, rag, tol)
    extra = {} if tuned is None else {"autotune": tuned}
    if plain is not None:
        extra.update({"plain_fp64": plain, "speedup_vs_plain_fp64": (nsolves * args.steps / el) / plain["value"]})
    return base_record(
        args, nsolves * args.steps / el, 1e3 * el / args.steps, "f32+f64",
        {"workload": "batched cross-validation: RBF n=%d d=16 l=%d, 32 mu x 8 rhs in one block solve, plus 64 "
                     "ragged ridge problems (n_k = m_k/4, m_k in [1000, 20000])" % (n, ell),
         "precision": "float32 Gram tiles (RBF) / float32 data (ridge), float32 inner PCG, float64 refinement",
         "step": "all 320 solves incl. sketches"},
        dict({"correct": ok, "phase_ms": phases, "solves_per_step": nsolves,
              "block_iters_max": max(infos[-1][0].iters), "block_refine": infos[-1][0].refine_steps}, **extra))


def run_batched_graph(args, nys, torch, w, op, B, mus, ell, prec, ws, rops, rbs, rag, tol, tuned):
    """The batched step with every PCG solve in one captured graph: the block
    solve (32 mu x 8 right-hand sides, device-info form: fixed iteration
    counts, stopped column blocks skip their products) and the ragged batch
    (device-info form) are captured once on buffers that hold the current
    preconditioners; each step sketches and factors eagerly, copies the
    factors into those buffers and replays the graph."""
    dev = B.device
    n, k = B.shape[0], len(mus) * B.shape[1]
    Ub = torch.empty(n, ell, dtype=torch.float32, device=dev)
    lb = torch.empty(ell, dtype=torch.float64, device=dev)
    Pb = nys.Precond(Ub, lb, 0.0)
    rUs = [torch.empty(o.n, p["ell"], dtype=torch.float32, device=dev) for o, p in zip(rops, rag)]
    rls = [torch.empty(p["ell"], dtype=torch.float64, device=dev) for p in rag]
    rPb = [nys.Precond(u, l, 0.0) for u, l in zip(rUs, rls)]
    rmus = [p["mu"] for p in rag]
    X = torch.zeros(n, k, dtype=torch.float64, device=dev)
    Xr = [torch.zeros_like(b) for b in rbs]
    ib = [torch.zeros(k, dtype=torch.int32, device=dev), torch.zeros(k, dtype=torch.float64, device=dev),
          torch.zeros(k, dtype=torch.int32, device=dev)]
    ir = [torch.zeros(len(rag), dtype=torch.int32, device=dev), torch.zeros(len(rag), dtype=torch.float64, device=dev),
          torch.zeros(len(rag), dtype=torch.int32, device=dev)]
    wsr = torch.empty(nys.lib().nys_workspace_size_ragged(
        (nys._Operator * len(rops))(*[o.c() for o in rops]), (nys._Precond * len(rPb))(*[p.c() for p in rPb]),
        len(rops), prec), dtype=torch.uint8, device=dev)
    kwb = dict(tol=tol, maxit=args.graph_maxit, prec=prec, max_refine=args.graph_refine,
               inner_tol=args.inner_tol or 3e-2, ws=ws)
    kwr = dict(tol=tol, maxit=150, prec=prec, max_refine=4, inner_tol=1e-5, ws=wsr)

    def factors(seed, tm):
        t = time.perf_counter()
        Om, Y = nys.nys_sketch(op, ell, seed=seed, prec=prec, ws=ws)
        P = nys.nys_factor(Om, Y, dtype=torch.float32, ws=ws, prec=prec)
        del Om, Y
        Ub.copy_(P.U)
        lb.copy_(P.lam)
        t = tm.lap("block_factor", t)
        for q, (o, p) in enumerate(zip(rops, rag)):
            Om, Y = nys.nys_sketch(o, p["ell"], seed=seed + q, prec=prec)
            Pq = nys.nys_factor(Om, Y, dtype=torch.float32, prec=prec)
            rUs[q].copy_(Pq.U)
            rls[q].copy_(Pq.lam)
        tm.lap("ragged_factor", t)

    def body():
        X.zero_()
        for x in Xr:
            x.zero_()
        nys.nys_pcg_solve_device(op, Pb, mus, B, X, *ib, **kwb)
        nys.nys_pcg_solve_ragged_device(rops, rPb, rmus, rbs, Xr, *ir, **kwr)

    tm0 = Timer(torch)
    factors(99, tm0)
    t = time.perf_counter()
    body()  # eager run outside the capture (one-time set-up, warm-up)
    torch.cuda.synchronize()
    log("eager device-info solves: %.1f ms" % (1e3 * (time.perf_counter() - t)))
    t = time.perf_counter()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    torch.cuda.synchronize()
    t_capture = time.perf_counter() - t
    log("graph captured in %.1f ms" % (1e3 * t_capture))

    def step(seed):
        tm = Timer(torch)
        factors(seed, tm)
        t = time.perf_counter()
        g.replay()
        tm.lap("graph_pcg", t)
        return tm

    for i in range(args.warmup):
        step(100 + i)
    t = time.perf_counter()
    tms, oks = [], []
    for i in range(args.steps):
        tm = step(20211004 + i)
        tms.append(tm)
        rb, sb, rr, sr = ib[1].cpu(), ib[2].cpu(), ir[1].cpu(), ir[2].cpu()
        oks.append(bool((sb == 0).all()) and bool((sr == 0).all()) and float(rb.max()) <= tol and
                   float(rr.max()) <= tol)
        log("graph step %d: %s; block relres max %.2e, iters max %d; ragged relres max %.2e" %
            (i, {kk: round(1e3 * v, 1) for kk, v in tm.t.items()}, float(rb.max()), int(ib[0].max()),
             float(rr.max())))
    el = time.perf_counter() - t
    nsolves = k + len(rag)
    phases = {kk: 1e3 * sum(tm.t.get(kk, 0.0) for tm in tms) / args.steps for kk in tms[0].t}
    extra = {"correct": all(oks), "phase_ms": phases, "solves_per_step": nsolves, "capture_ms": 1e3 * t_capture,
             "graph": {"block_maxit": args.graph_maxit, "block_refine": args.graph_refine, "ragged_maxit": 150,
                       "ragged_refine": 4}}
    if tuned is not None:
        extra["autotune"] = tuned
    return base_record(
        args, nsolves * args.steps / el, 1e3 * el / args.steps, "f32+f64",
        {"workload": "batched cross-validation: RBF n=%d d=16 l=%d, 32 mu x 8 rhs in one block solve, plus 64 "
                     "ragged ridge problems (n_k = m_k/4, m_k in [1000, 20000]); every PCG solve of the step in one "
                     "captured graph" % (n, ell),
         "precision": "float32 Gram tiles (RBF) / float32 data (ridge), float32 inner PCG, float64 refinement",
         "step": "all 320 solves incl. sketches (sketches and factors eager, PCG as one graph replay)"},
        extra)


def batched_plain_fp64(nys, torch, w, X, B, mus, rops, rbs, rag, tol):
    """The plain float64 GPU path on a documented subset of the batched
    workload, one system at a time: the RBF data upcast to float64 in HBM, a
    float64 sketch and factor (the preconditioner does not depend on mu, so the
    plain path also builds it once), then 8 columns spanning the mu grid (mu
    indices 0, 4, ..., 28 with right-hand side m mod 8), each solved alone in
    float64; and 4 ragged problems (every 16th) each with its own float64
    sketch, factor and solve.  The per-solve rate extrapolates the subset to
    the whole batch: 320 / (t_setup + 256 mean(t_column) + 64 mean(t_ragged))."""
    dev = X.device
    f64 = nys.NYS_PREC_FP64
    X64 = X.double()
    op64 = nys.Operator.rbf(X64, w["sigma"])
    ell = w["ell"]
    ws = nys.workspace(op64, ell, 1, f64)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Om, Y = nys.nys_sketch(op64, ell, seed=5, prec=f64, ws=ws)
    P = nys.nys_factor(Om, Y, dtype=torch.float64, ws=ws, prec=f64)
    del Om, Y
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    cols = list(range(0, len(mus), 4))
    t_cols, it_cols, ok = [], [], True
    for m in cols:
        b = B[:, m % B.shape[1]].contiguous()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = nys.nys_pcg_solve(op64, P, mus[m], b, tol=tol, maxit=5000, prec=f64, ws=ws)
        torch.cuda.synchronize()
        t_cols.append(time.perf_counter() - t)
        it_cols.append(info.iters[0])
        ok = ok and info.relres[0] <= tol
        log("plain fp64 column mu=%.3g: %.1f ms, %d iters" % (mus[m], 1e3 * t_cols[-1], info.iters[0]))
    del P, ws, op64, X64
    t_rag = []
    for k in range(0, len(rag), 16):
        Xk64 = rops[k].data.double()
        o64 = nys.Operator.xtx(Xk64)
        wsk = nys.workspace(o64, rag[k]["ell"], 1, f64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        Om, Y = nys.nys_sketch(o64, rag[k]["ell"], seed=11 + k, prec=f64, ws=wsk)
        Pk = nys.nys_factor(Om, Y, dtype=torch.float64, ws=wsk, prec=f64)
        _, info = nys.nys_pcg_solve(o64, Pk, rag[k]["mu"], rbs[k], tol=tol, maxit=1000, prec=f64, ws=wsk)
        torch.cuda.synchronize()
        t_rag.append(time.perf_counter() - t)
        ok = ok and info.relres[0] <= tol
        log("plain fp64 ragged problem %d (%dx%d): %.1f ms" % (k, Xk64.shape[0], Xk64.shape[1], 1e3 * t_rag[-1]))
        del Xk64, o64, wsk, Pk
    ncol, nrag = len(mus) * B.shape[1], len(rag)
    total = t_setup + ncol * float(np.mean(t_cols)) + nrag * float(np.mean(t_rag))
    return {"value": (ncol + nrag) / total, "unit": "solves/s", "seconds_extrapolated": total,
            "setup_ms": 1e3 * t_setup, "column_ms": [1e3 * v for v in t_cols], "column_iters": it_cols,
            "ragged_ms": [1e3 * v for v in t_rag], "correct": bool(ok),
            "sample": "float64 sketch + factor once, 8 of 256 columns (mu indices 0, 4, ..., 28) solved one at "
                      "a time, 4 of 64 ragged problems (sketch + factor + solve each); extrapolated to 320 solves"}


# --------------------------------------------------------------------------- differentiation

def run_diff(args, nys, torch):
    from workloads import differentiation
    dev = "cuda:0"
    n = args.n or 100000
    w = differentiation(n=n, nval=max(1000, n // 10), with_omega=False)
    log("inputs ready")
    X = torch.as_tensor(w["X"], device=dev)
    Xv = torch.as_tensor(w["Xval"], device=dev)
    op = nys.Operator.rbf(X, w["sigma"])
    b = rbf_rhs(nys, torch, op, w, dev)
    wv = torch.as_tensor(w["w"], device=dev)
    yv = nys.nys_rbf_cross(op, Xv, wv) + w["noise"] * torch.as_tensor(w["eps_val"], device=dev)
    ell, mu, sigma, tol = w["ell"], w["mu"], w["sigma"], 1e-10
    prec = nys.NYS_PREC_BF16X3_REFINE64
    ws = nys.workspace(op, ell, 1, prec)
    itol = args.inner_tol or 3e-2

    def step(seed):
        """Forward solve, loss and its gradients through torch.autograd: the
        adjoint solve reuses the forward preconditioner."""
        tm = Timer(torch)
        t = time.perf_counter()
        Om, Y = nys.nys_sketch(op, ell, seed=seed, prec=prec, ws=ws)
        P = nys.nys_factor(Om, Y, dtype=torch.float32, ws=ws, prec=prec)
        del Om, Y
        t = tm.lap("sketch_factor", t)
        bt = b.clone().requires_grad_(True)
        mut = torch.tensor(mu, dtype=torch.float64, device=dev, requires_grad=True)
        sgt = torch.tensor(sigma, dtype=torch.float64, device=dev, requires_grad=True)
        x = nys.nystrom_solve(bt, mut, P, X=X, sigma=sgt, tol=tol, maxit=5000, prec=prec, inner_tol=itol)
        rv = nys.rbf_cross(x, sgt, X, Xv) - yv
        L = (rv * rv).sum()
        t = tm.lap("forward", t)
        gb, gmu, gsig = torch.autograd.grad(L, [bt, mut, sgt])
        tm.lap("backward", t)
        return float(L), gb, float(gmu), float(gsig), x.detach(), tm

    for i in range(args.warmup):
        step(200 + i)
    t = time.perf_counter()
    tms = []
    for i in range(args.steps):
        L, gb, gmu, gs, x, tm = step(20211005 + i)
        tms.append(tm)
        log("diff step %d: L=%.6e dL/dmu=%.6e dL/dsigma=%.6e %s" % (i, L, gmu, gs,
                                                                   {k: round(1e3 * v, 1) for k, v in tm.t.items()}))
    el = time.perf_counter() - t
    # correctness, outside the timed region: the oracle's float64 kernel rows
    # at sampled points check the forward residual b - (K + mu I) x and the
    # validation residual K_val x - y_val that the loss and its gradients use
    import oracle
    rng = np.random.default_rng(75)
    Xd = w["X"].astype(np.float64)
    xh = x.cpu().numpy()
    bh = b.cpu().numpy()
    ridx = rng.choice(n, size=48, replace=False)
    rows = oracle.rbf_kernel_block(Xd[ridx], Xd, sigma)
    r_fwd = np.abs(bh[ridx] - (rows @ xh + mu * xh[ridx])).max() / np.linalg.norm(bh)
    vidx = rng.choice(Xv.shape[0], size=32, replace=False)
    yvh = yv.cpu().numpy()
    rv_or = oracle.rbf_kernel_block(w["Xval"].astype(np.float64)[vidx], Xd, sigma) @ xh - yvh[vidx]
    rv_dev = (nys.nys_rbf_cross(op, Xv, x) - yv).cpu().numpy()[vidx]
    rv_err = np.abs(rv_dev - rv_or).max() / max(np.abs(rv_or).max(), 1e-300)
    ok = r_fwd <= tol and rv_err <= 1e-10
    extra = {}
    if not args.no_plain:
        # plain float64 GPU path: data upcast to float64 in HBM, float64 sketch,
        # factor, forward and adjoint solves, one evaluation; its loss and
        # gradients also cross-check the chosen form's (relative agreement)
        X64, Xv64 = X.double(), Xv.double()
        op64 = nys.Operator.rbf(X64, sigma)
        ws64 = nys.workspace(op64, ell, 1, nys.NYS_PREC_FP64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        Om, Y = nys.nys_sketch(op64, ell, seed=20211005, prec=nys.NYS_PREC_FP64, ws=ws64)
        P64 = nys.nys_factor(Om, Y, dtype=torch.float64, ws=ws64, prec=nys.NYS_PREC_FP64)
        del Om, Y
        bt = b.clone().requires_grad_(True)
        mut = torch.tensor(mu, dtype=torch.float64, device=dev, requires_grad=True)
        sgt = torch.tensor(sigma, dtype=torch.float64, device=dev, requires_grad=True)
        x64 = nys.nystrom_solve(bt, mut, P64, X=X64, sigma=sgt, tol=tol, maxit=5000, prec=nys.NYS_PREC_FP64)
        rv64 = nys.rbf_cross(x64, sgt, X64, Xv64) - yv
        L64 = (rv64 * rv64).sum()
        gb64, gmu64, gs64 = torch.autograd.grad(L64, [bt, mut, sgt])
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t
        rel = lambda a, c: abs(a - c) / max(abs(c), 1e-300)
        agree = {"L": rel(L, float(L64)), "dL_dmu": rel(gmu, float(gmu64)), "dL_dsigma": rel(gs, float(gs64)),
                 "dL_db": float((gb - gb64).norm() / gb64.norm())}
        log("plain fp64 evaluation: %.1f ms; relative agreement %s" % (1e3 * el64, agree))
        extra = {"plain_fp64": {"value": 1.0 / el64, "unit": "evaluations/s", "ms_per_step": 1e3 * el64,
                                "agreement_with_chosen": agree},
                 "speedup_vs_plain_fp64": (args.steps / el) * el64}
        ok = ok and max(agree.values()) <= 1e-5
        del X64, Xv64, op64, ws64, P64
    return base_record(
        args, args.steps / el, 1e3 * el / args.steps, "bf16x3+f32+f64",
        {"workload": "validation loss L = ||K_val x - y_val||^2 through the RBF solve, n=%d, nval=%d, d=16, l=%d"
                     % (n, Xv.shape[0], ell),
         "precision": "bf16x3 Gram tiles, float32 inner PCG, float64 refinement and gradient reductions",
         "step": "sketch + factor + forward solve + loss + torch.autograd.grad (adjoint solve with the same "
                 "preconditioner, dL/dmu, dL/dsigma, dL/db)"},
        {"unit_note": "value = loss-and-gradient evaluations per second",
         "correct": bool(ok), "check": {"forward_residual_rows_max_over_bnorm": r_fwd,
                                        "val_residual_rows_rel_err": rv_err, "rows": 48, "val_rows": 32},
         "phase_ms": {k: 1e3 * sum(tm.t.get(k, 0.0) for tm in tms) / args.steps for k in tms[0].t},
         "L": L, "dL_dmu": gmu, "dL_dsigma": gs, **extra})


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; the figure is one "
              "GPU's throughput (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2110_02820_amd as nys
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    fn = {"ridge": run_ridge_kernel if args.kernel_only else run_ridge,
          "krr_small": lambda a, n, t: run_krr(a, n, t, small=True), "krr": run_krr,
          "krr_cols": lambda a, n, t: run_krr(a, n, t, columns=True),
          "batched": run_batched, "diff": run_diff, "adaptive": run_adaptive,
          "sketch_solve": run_sketch_solve, "block": run_block, "weighted": run_weighted}[args.workload]
    out = fn(args, nys, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
