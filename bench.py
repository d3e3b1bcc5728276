"""Benchmark: Nystrom PCG solves/s on one MI355X at a true float64 relative
residual of 1e-10, chosen form (float32 inner PCG + float64 refinement) next
to the plain float64 GPU path, plus the roofline of the dominant kernel (the
one-pass X^T X matvec) and the CPU oracle as a baseline.

Workload (default): dense ridge regression, X = G diag(j^-1/2) in float32
(20000 x 4000, G ~ N(0, 1/20000)), A = X^T X, b = X^T y, mu = 1e-4, l = 500.
One step = one whole solve: Gaussian test matrix, sketch Y = A Omega, shifted
Cholesky + SVD factorisation, and PCG with refinement to 1e-10.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-plain] [--no-cpu-baseline]
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=20000)
    ap.add_argument("--n", type=int, default=4000)
    ap.add_argument("--ell", type=int, default=500)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=30)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2110_02820_amd as nys
    from workloads import ridge_dense

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    t0 = time.time()
    w = ridge_dense(m=args.m, n=args.n, ell=args.ell, with_omega=False)
    X32h = w["X"]
    # b = X^T y (input synthesis on the host, float64)
    b_h = X32h.astype(np.float64).T @ w["y"]
    mu, ell, tol = w["mu"], args.ell, 1e-10
    X32 = torch.as_tensor(X32h, device=dev)
    b = torch.as_tensor(b_h, device=dev)
    op = nys.Operator.xtx(X32)
    prec = nys.NYS_PREC_FP32_REFINE64
    ws = nys.workspace(op, ell, 1, prec)
    print("# inputs ready in %.1fs" % (time.time() - t0), file=sys.stderr, flush=True)

    def step(seed, opx, precx, wsx, udtype):
        Om, Y = nys.nys_sketch(opx, ell, seed=seed, prec=precx, ws=wsx)
        P = nys.nys_factor(Om, Y, dtype=udtype, ws=wsx, prec=precx)
        x, info = nys.nys_pcg_solve(opx, P, mu, b, tol=tol, maxit=1000, prec=precx, ws=wsx, inner_tol=1e-4)
        return x, info

    def timed(opx, precx, wsx, udtype, steps, warmup, label):
        for i in range(warmup):
            step(1000 + i, opx, precx, wsx, udtype)
        torch.cuda.synchronize()
        ph = {"sketch": 0.0, "factor": 0.0, "pcg": 0.0}
        infos = []
        t = time.perf_counter()
        for i in range(steps):
            a = time.perf_counter()
            Om, Y = nys.nys_sketch(opx, ell, seed=20211002 + i, prec=precx, ws=wsx)
            torch.cuda.synchronize()
            bb = time.perf_counter()
            P = nys.nys_factor(Om, Y, dtype=udtype, ws=wsx, prec=precx)
            torch.cuda.synchronize()
            c = time.perf_counter()
            x, info = nys.nys_pcg_solve(opx, P, mu, b, tol=tol, maxit=1000, prec=precx, ws=wsx, inner_tol=1e-4)
            torch.cuda.synchronize()
            d = time.perf_counter()
            ph["sketch"] += bb - a
            ph["factor"] += c - bb
            ph["pcg"] += d - c
            infos.append(info)
            print("# %s step %d: %.2f ms, iters %d, refine %d, relres %.2e" %
                  (label, i, 1e3 * (d - a), info.iters[0], info.refine_steps, info.relres[0]),
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        return el, {k: 1e3 * v / steps for k, v in ph.items()}, infos

    el, phases, infos = timed(op, prec, ws, torch.float32, args.steps, args.warmup, "chosen")
    ok = all(i.relres[0] <= tol and i.status[0] == 0 for i in infos)
    ms = 1e3 * el / args.steps

    # roofline of the dominant kernel: the one-pass float32 X^T X matvec
    v32 = torch.randn(args.n, dtype=torch.float32, device=dev)
    wsm = nys.workspace(op, 1, 1, nys.NYS_PREC_FP64)
    for _ in range(3):
        nys.nys_op_apply(op, mu, v32, ws=wsm)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.matvec_reps):
        nys.nys_op_apply(op, mu, v32, ws=wsm)
    e1.record()
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / args.matvec_reps
    alg_bytes = args.m * args.n * 4 + 2 * args.n * 4  # X once + p in + v out
    achieved = alg_bytes / (mv_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": args.steps / el, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "ridge regression A = X^T X, X %dx%d float32 = G diag(j^-1/2), mu=1e-4, "
                               "l=%d, b = X^T y, tol 1e-10 (true float64 residual)" % (args.m, args.n, ell),
                   "precision": "float32 inner PCG + float64 residual refinement; float64 core factorisation",
                   "step": "Gaussian Omega + sketch + factor + PCG solve"},
        "correct": ok,
        "relres": max(i.relres[0] for i in infos),
        "iters": infos[-1].iters[0], "refine_steps": infos[-1].refine_steps,
        "phase_ms": phases,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "xtx_fused<float,float> + reduce_cols (one X^T X matvec)",
                     "avg_ms": mv_ms, "alg_bytes": alg_bytes},
    }

    if not args.no_plain:
        X64 = X32.double()
        op64 = nys.Operator.xtx(X64)
        ws64 = nys.workspace(op64, ell, 1, nys.NYS_PREC_FP64)
        el64, ph64, inf64 = timed(op64, nys.NYS_PREC_FP64, ws64, torch.float64, max(1, min(args.steps, 3)), 1,
                                  "plain")
        n64 = max(1, min(args.steps, 3))
        out["plain_fp64"] = {"value": n64 / el64, "unit": "solves/s", "ms_per_step": 1e3 * el64 / n64,
                             "phase_ms": ph64, "iters": inf64[-1].iters[0], "relres": inf64[-1].relres[0],
                             "correct": all(i.relres[0] <= tol for i in inf64)}
        out["speedup_vs_plain_fp64"] = out["value"] / out["plain_fp64"]["value"]
        del X64, op64, ws64

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, b_h, mu, ell, tol)
    print(json.dumps(out), flush=True)


def cpu_baseline(w, b_h, mu, ell, tol):
    """The float64 CPU oracle, unchanged, on one full solve of the same workload."""
    import oracle
    from workloads import gaussian_test_matrix
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    X = w["X"]
    opr = oracle.XtXOp(X)
    om0 = gaussian_test_matrix(X.shape[1], ell, 7)
    t = time.perf_counter()
    r = oracle.randomized_nystrom(opr, om0)
    out = oracle.nystrom_pcg(opr.matmat, b_h, mu, lambda v: oracle.precond_inv_apply(r["U"], r["lam"], mu, v),
                             tol=tol, maxit=1000)
    el = time.perf_counter() - t
    return {"value": 1.0 / el, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": "one full solve of the same workload (sketch + factor + PCG to 1e-10), numpy float64",
            "seconds": el, "iters": out["iters"]}


if __name__ == "__main__":
    main()
