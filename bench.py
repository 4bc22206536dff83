#!/usr/bin/env python3
"""Throughput of the Cholesky factor + reverse-mode adjoint hot path on one MI355X.

One step = restore the covariance and the adjoint seed from pristine device
copies, factor (in place), solve z = L^-1 y and alpha = L^-T z, log-det, then the
adjoint Abar of the factor.  The workload is the n = 16384 Matern-3/2 covariance
on 2-D points (x ~ U([0,50]^2), lengthscale 3, noise 0.01 I, Lbar ~ N(0,1)).
Inputs are generated once on the host, copied to the device before timing and
stay resident.  value = (n^3/3 + n^2/2 + n/6 + 2 n^3/3) / (seconds per step),
in GFLOP/s; the solves and copies are inside the timed step but add no flops.

Prints ONE JSON line (rank 0).  ``--gpus N`` with N > 1 exits: this build runs
on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X dense matrix peaks
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n_sample: int, threads: int | None):
    """Oracle factor + adjoint on a same-density sample of the workload."""
    import oracle
    import workloads as W
    case = W.c3(n=n_sample)
    t0 = time.perf_counter()
    L, info = oracle.potrf(case["A"])
    Ab = oracle.potrf_adjoint(L, case["Lbar"])
    dt = time.perf_counter() - t0
    F = W.flops_factor(n_sample) + W.flops_adjoint(n_sample)
    return {"value": F / dt / 1e9, "unit": "GFLOP/s",
            "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": f"factor+adjoint of the same-density Matern-3/2 matrix at n={n_sample} "
                      f"(1 run, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--form", choices=["fp64"], default="fp64")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=5120)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1907_01063_amd import Handle

    n = args.n
    log(f"generating workload n={n}")
    case = W.c3(n=n)
    dev = "cuda"
    A0 = torch.from_numpy(case["A"]).to(dev)
    Lb0 = torch.from_numpy(case["Lbar"]).to(dev)
    y0 = torch.from_numpy(case["y"]).to(dev)
    del case
    L = torch.empty_like(A0)
    Lb = torch.empty_like(Lb0)
    z = torch.empty_like(y0)
    a = torch.empty_like(y0)
    info = torch.zeros((), dtype=torch.int32, device=dev)
    ld = torch.zeros((), dtype=torch.float64, device=dev)
    H = Handle()
    H.set_options(block=args.block)

    def step():
        L.copy_(A0)
        H.factor(L, info)
        z.copy_(y0)
        H.trsm(L, z)
        a.copy_(z)
        H.trsm(L, a, trans=True)
        H.logdet(L, ld)
        Lb.copy_(Lb0)
        H.adjoint(L, Lb)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    if int(info.item()) != 0:
        raise SystemExit(f"factor reported info={int(info.item())}")

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log(f"timed {args.steps} steps: {ms:.2f} ms/step")
    F = W.flops_factor(n) + W.flops_adjoint(n)
    value = F / (ms * 1e-3) / 1e9

    # residuals of the last step (checks, not part of the timing)
    rows = torch.randperm(n, generator=torch.Generator().manual_seed(0))[:64].to(dev)
    Asym = A0
    res_fact = (torch.linalg.norm(L[rows] @ L.T - Asym[rows]) / torch.linalg.norm(Asym[rows])).item()
    r = y0 - Asym @ a
    eta = (r.abs().max() / (Asym.abs().sum(1).max() * a.abs().max() + y0.abs().max())).item()
    log(f"sampled ||LL^T-A||/||A|| = {res_fact:.2e}, solve eta_inf = {eta:.2e}")

    roof = None
    if not args.no_trace:
        H.trace_enable(True)
        H.trace_reset()
        step()
        tr = H.trace_read()
        H.trace_enable(False)
        mfma = {k: v for k, v in tr.items()
                if k in ("trailing_update", "adj_left_update", "adj_row_update", "panel_solve",
                         "adj_panel_solve", "adj_diag_product")}
        dom = max(mfma, key=lambda k: mfma[k][1])
        cnt, kms, kfl, kby = tr[dom]
        achieved = kfl / (kms * 1e-3) / 1e12
        peak = PEAK_TFLOPS["f64"]
        roof = {"bound": "mfma", "kernel": dom, "launches": cnt, "achieved": round(achieved, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "avg_launch_ms": round(kms / max(cnt, 1), 4),
                "classes_ms": {k: round(v[1], 3) for k, v in tr.items()}}
        log(f"trace: {json.dumps(roof)}")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle) at n={args.cpu_sample}")
        cpu = cpu_baseline(args.cpu_sample, int(os.environ.get("OMP_NUM_THREADS", "0")) or None)

    out = {
        "metric": "Cholesky factor+adjoint GFLOP/s @ n=16384, FP64 vs mixed, at stated residual",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"matern32-2d-n{n} factor+solves+logdet+adjoint", "n": n,
                   "form": args.form, "block": args.block or 128,
                   "frac_of_fp64_peak": round(value / 1e3 / PEAK_TFLOPS["f64"], 4),
                   "factor_residual_sampled": res_fact, "solve_eta_inf": eta},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
