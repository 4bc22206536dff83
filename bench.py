#!/usr/bin/env python3
"""Throughput of the Cholesky factor + reverse-mode adjoint hot path on one MI355X.

Headline (``value``): FP64, n = 16384 Matern-3/2 covariance on 2-D points
(x ~ U([0,50]^2), lengthscale 3, noise 0.01 I, Lbar ~ N(0,1), y ~ N(0,1)).
One step = restore the covariance and the adjoint seed from pristine device
copies, factor (in place), z = L^-1 y, alpha = L^-T z, log-det, adjoint Abar.
value = (n^3/3 + n^2/2 + n/6 + 2 n^3/3) / (seconds per step) in GFLOP/s; the
solves and copies are inside the timed step but add no flops.

Also measured (under ``config``), each on its own workload:
  mixed    the same step with FP32-MFMA trailing updates and the FP64 solve
           replaced by the FP64-refined solve of K alpha = y (eta <= 1e-12),
           with its error against the FP64 path;
  batched  512 SE covariances of order U{32..1024} (3-D inputs), factor +
           adjoint of all in one persistent graph-replayed launch;
  gp       GP marginal log-likelihood gradient at n = 30000 (SE-ARD, 8-D
           inputs) through the autograd.Function, FP64 and mixed.
Inputs are generated on the host with fixed seeds, copied to the device before
timing and stay resident.  Prints ONE JSON line.  ``--gpus N`` with N > 1
exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X dense matrix peaks
METRIC = "Cholesky factor+adjoint GFLOP/s @ n=16384, FP64 vs mixed, at stated residual"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_time(case) -> float:
    """Seconds of the oracle's factor + adjoint of one case."""
    import oracle
    t0 = time.perf_counter()
    L, _ = oracle.potrf(case["A"])
    oracle.potrf_adjoint(L, case["Lbar"])
    return time.perf_counter() - t0


def cpu_baseline(n_sample: int, per_config: bool):
    """The oracle's factor + adjoint on a same-density sample of the workload
    (the headline line), and, per workload, the oracle's times with the
    paper's repetition protocol where they fit in a bounded run."""
    import statistics
    import oracle
    import workloads as W
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    threads = oracle.threads()
    case = W.c3(n=n_sample)
    dt = oracle_time(case)
    F = W.flops_factor(n_sample) + W.flops_adjoint(n_sample)
    out = {"value": round(F / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"factor+adjoint of the same-density Matern-3/2 matrix at n={n_sample}, 1 run, "
                     f"{dt:.1f} s (GFLOP/s with the same flop count)",
           "cpu_model": cpu_model(), "host_cpus_available": cores, "omp_threads": threads}
    del case
    if not per_config:
        return out
    pc = {}
    c1 = W.c1()
    F1 = W.flops_factor(256) + W.flops_adjoint(256)
    for t in (1, cores):
        oracle.set_threads(t)
        ts = sorted(oracle_time(c1) for _ in range(9))
        pc[f"se1d-n256 threads={t}"] = {"median_s": statistics.median(ts), "min_s": ts[0],
                                        "gflops_median": round(F1 / statistics.median(ts) / 1e9, 3),
                                        "protocol": "median of 9"}
        log(f"oracle se1d-n256 threads={t}: median {statistics.median(ts) * 1e3:.2f} ms")
    oracle.set_threads(cores)
    c2 = W.c2()
    F2 = W.flops_factor(4096) + W.flops_adjoint(4096)
    ts = sorted(oracle_time(c2) for _ in range(3))
    pc[f"se4d-n4096 threads={cores}"] = {"median_s": statistics.median(ts), "min_s": ts[0],
                                         "gflops_median": round(F2 / statistics.median(ts) / 1e9, 3),
                                         "protocol": "median of 3"}
    log(f"oracle se4d-n4096: median {statistics.median(ts):.2f} s")
    del c2
    bc = W.c4()
    t0 = time.perf_counter()
    Fb = 0.0
    for nb, off in zip(bc["n"], bc["off"]):
        nb = int(nb)
        A = bc["base"][off:off + nb * nb].reshape(nb, nb)
        Lb = bc["Lbar"][off:off + nb * nb].reshape(nb, nb)
        L, _ = oracle.potrf(A)
        oracle.potrf_adjoint(L, Lb)
        Fb += W.flops_factor(nb) + W.flops_adjoint(nb)
    tb = time.perf_counter() - t0
    pc[f"se3d-batch512 threads={cores}"] = {"s": tb, "gflops": round(Fb / tb / 1e9, 3), "protocol": "1 run"}
    log(f"oracle se3d-batch512: {tb:.2f} s")
    out["per_config"] = pc
    return out


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed PMC record
    (profiles/traffic.json), or None if the record is for another kernel or
    the kernel's sources changed since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(root, src), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return round(rec["traffic_bytes_per_launch"])


PROGRESS = False   # --progress: one line per step (each step then waits for the GPU)


def ops_bench(reps: int = 5):
    """The operations beside the factor (lower-triangular inverse and the
    reverse modes of the solve and the inverse, products and their split-K
    form, A A^T, the Bernoulli-logit GLM), each on seeded synthetic inputs
    of a stated shape: median of `reps` launches after one warm-up, as
    GFLOP/s against the FP64 matrix peak (contractions) or GB/s of
    algorithmic bytes against 8 TB/s (the GLM)."""
    import statistics
    import numpy as np
    import torch
    import workloads as W
    from paper_1907_01063_amd import Handle
    from paper_1907_01063_amd import ops as O
    dev = "cuda"
    H = Handle()

    def med_ms(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    out = {}

    def rec(name, ms, flops=None, nbytes=None, note=""):
        r = {"ms": round(ms, 4)}
        if flops is not None:
            tf = flops / (ms * 1e-3) / 1e12
            r.update({"flops": flops, "TFLOP/s": round(tf, 2), "frac_fp64_peak": round(tf / PEAK_TFLOPS["f64"], 4)})
        if nbytes is not None:
            gbs = nbytes / (ms * 1e-3) / 1e9
            r.update({"bytes": nbytes, "GB/s": round(gbs, 1), "frac_hbm": round(gbs / 8000.0, 4)})
        if note:
            r["flop_count"] = note
        out[name] = r
        log(f"ops {name}: {json.dumps(r)}")

    n = 16384
    c = W.tri(n)
    L = torch.from_numpy(c["L"]).to(dev)
    del c
    X = torch.empty_like(L)
    rec(f"trtri-n{n}", med_ms(lambda: O.trtri(H, L, X)), n ** 3 / 3.0, note="n^3/3")
    n2 = 8192
    L2 = L[:n2, :n2].contiguous()
    X2 = O.trtri(H, L2)
    Xb2 = torch.tril(torch.randn(n2, n2, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(7)))
    Lb2 = torch.empty_like(L2)
    rec(f"trtri_adjoint-n{n2}", med_ms(lambda: O.trtri_adjoint(H, X2, Xb2, Lb2)), float(n2) ** 3,
        note="n^3 (two triangular-by-triangular products)")
    del X2, Xb2, Lb2, L2
    r = 64
    Bm = torch.randn(n, r, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(8))
    C = Bm.clone()
    H.trsm(L, C)
    Cb0 = torch.randn(n, r, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(9))
    Cb = Cb0.clone()
    Lb = torch.empty_like(L)

    def tadj():
        Cb.copy_(Cb0)
        O.trsm_adjoint(H, L, C, Cb, False, Lb)
    rec(f"trsm_adjoint-n{n}-r{r}", med_ms(tadj), 2.0 * n * n * r, note="2 n^2 r (solve n^2 r + tril(Bbar C^T) n^2 r)")
    del L, X, Bm, C, Cb0, Cb, Lb
    torch.cuda.empty_cache()
    m = 8192
    g = torch.Generator(dev).manual_seed(10)
    A = torch.randn(m, m, dtype=torch.float64, device=dev, generator=g)
    B = torch.randn(m, m, dtype=torch.float64, device=dev, generator=g)
    Cm = torch.empty_like(A)
    rec(f"gemm-{m}x{m}x{m}", med_ms(lambda: O.gemm(H, A, B, C=Cm)), 2.0 * m ** 3, note="2MNK")
    Ab, Bb = torch.empty_like(A), torch.empty_like(B)
    rec(f"gemm_adjoint-{m}x{m}x{m}", med_ms(lambda: O.gemm_adjoint(H, A, B, Cm, Abar=Ab, Bbar=Bb)),
        4.0 * m ** 3, note="4MNK (Abar and Bbar)")
    del Ab, Bb
    rec(f"multiply_transpose-{m}x{m}", med_ms(lambda: O.multiply_transpose(H, A, Cm)), float(m) * (m + 1) * m,
        note="M(M+1)K (lower tiles, mirrored)")
    del A, B, Cm
    torch.cuda.empty_cache()
    Ms, Ks = 256, 262144
    As = torch.randn(Ms, Ks, dtype=torch.float64, device=dev, generator=g)
    Bs = torch.randn(Ks, Ms, dtype=torch.float64, device=dev, generator=g)
    Cs = torch.empty(Ms, Ms, dtype=torch.float64, device=dev)
    ms_s = med_ms(lambda: O.gemm(H, As, Bs, C=Cs))
    rec(f"gemm_splitk-{Ms}x{Ms}x{Ks}", ms_s, 2.0 * Ms * Ms * Ks, note=f"2MNK, {O.last_splits(H)} k-slices")
    del As, Bs, Cs
    torch.cuda.empty_cache()
    for (nn, kk) in ((1000000, 100), (100000, 1000)):
        gl = W.glm(nn, kk)
        Xg = torch.from_numpy(gl["X"]).to(dev)
        yg = torch.from_numpy(gl["y"]).to(dev)
        al = torch.tensor(gl["alpha"], dtype=torch.float64, device=dev)
        be = torch.from_numpy(gl["beta"]).to(dev)
        del gl
        by = 8.0 * nn * kk + 4.0 * nn
        rec(f"glm_bernoulli_logit-n{nn}-k{kk}", med_ms(lambda: O.glm_bernoulli_logit(H, Xg, yg, al, be)),
            nbytes=by)
        rec(f"glm_bernoulli_logit-n{nn}-k{kk}-with-dX",
            med_ms(lambda: O.glm_bernoulli_logit(H, Xg, yg, al, be, with_dX=True)), nbytes=by + 8.0 * nn * kk)
        del Xg, yg, al, be
        torch.cuda.empty_cache()
    del H
    return out


def timed(fn, steps, warmup, what=""):
    import torch
    for i in range(warmup):
        fn()
        if PROGRESS:
            torch.cuda.synchronize()
            log(f"{what} warmup step {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn()
        if PROGRESS:
            torch.cuda.synchronize()
            log(f"{what} step {i + 1}/{steps} done")
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def mixed_step(args, A0, Lb0, y0, info, ld):
    """The mixed-form step on the headline workload: restore the covariance,
    factor with FP32 trailing updates, FP64-refined solve of K alpha = y,
    log-det, restore the adjoint seed, adjoint.  Returns (step, L, Abar, x,
    handle, out) with out holding the last refinement's (x, iters, eta)."""
    import torch
    from paper_1907_01063_amd import GPC_MIXED, Handle
    Lm, Lbm = torch.empty_like(A0), torch.empty_like(Lb0)
    xr = torch.empty_like(y0)
    Hm = Handle()
    Hm.set_options(block=args.block, precision=GPC_MIXED, lookahead=args.lookahead, adjoint_group=args.adjoint_group)
    out = {}

    def stepmix():
        Lm.copy_(A0)
        Hm.factor(Lm, info)
        out["x"], out["it"], out["eta"] = Hm.solve_refined(A0, Lm, y0, x=xr, check=False)
        Hm.logdet(Lm, ld)
        Lbm.copy_(Lb0)
        Hm.adjoint(Lm, Lbm)

    return stepmix, Lm, Lbm, xr, Hm, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--lookahead", type=int, default=1)
    ap.add_argument("--adjoint-group", type=int, default=0, choices=range(0, 9),
                    help="reverse-sweep steps whose B-bar updates are applied together (0 = library default)")
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--gp-evals", type=int, default=10,
                    help="GP gradient evaluations timed per form (of the workload's 100 jittered thetas)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-configs", action="store_true",
                    help="skip the oracle's per-workload timings (the cpu_baseline sample only)")
    ap.add_argument("--progress", action="store_true",
                    help="log every step after waiting for it (for profiler runs; timing is then not meaningful)")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--serial-classes", action="store_true",
                    help="also trace one step with lookahead off (per-class kernel times, each kernel alone)")
    ap.add_argument("--headline-only", action="store_true")
    ap.add_argument("--no-ops", action="store_true", help="skip the operations beside the factor")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 512-matrix batch (for profiler runs; prints its own JSON line)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="run only the mixed-form step (for profiler runs; prints its own JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    global PROGRESS
    PROGRESS = args.progress

    import numpy as np
    import torch
    import workloads as W
    from paper_1907_01063_amd import GPC_FP64, GPC_MIXED, Handle, gp_mll

    n = args.n
    dev = "cuda"
    log(f"generating matern32-2d n={n}")
    case = W.c3(n=n)
    A0 = torch.from_numpy(case["A"]).to(dev)
    Lb0 = torch.from_numpy(case["Lbar"]).to(dev)
    y0 = torch.from_numpy(case["y"]).to(dev)
    del case
    L, Lb = torch.empty_like(A0), torch.empty_like(Lb0)
    z, a = torch.empty_like(y0), torch.empty_like(y0)
    info = torch.zeros((), dtype=torch.int32, device=dev)
    ld = torch.zeros((), dtype=torch.float64, device=dev)
    H = Handle()
    H.set_options(block=args.block, precision=GPC_FP64, lookahead=args.lookahead, adjoint_group=args.adjoint_group)
    F = W.flops_factor(n) + W.flops_adjoint(n)

    if args.batched_only:
        # the batch alone, for profiler runs of its kernels (no headline)
        del A0, Lb0, y0, L, Lb
        torch.cuda.empty_cache()
        bc = W.c4()
        base0 = torch.from_numpy(bc["base"]).to(dev)
        lbar0 = torch.from_numpy(bc["Lbar"]).to(dev)
        bw, lw = torch.empty_like(base0), torch.empty_like(lbar0)
        binfo = torch.zeros(len(bc["n"]), dtype=torch.int32, device=dev)
        Hb = Handle()

        def stepb():
            bw.copy_(base0)
            lw.copy_(lbar0)
            Hb.factor_adjoint_batched(bc["n"], bc["off"], bw, lw, binfo)
        msb = timed(stepb, args.steps, args.warmup, "batched")
        print(json.dumps({"form": "batched", "workload": "se3d-batch512", "ms_per_step_with_copies": round(msb, 3)}),
              flush=True)
        return

    if args.mixed_only:
        # the mixed step alone, for profiler runs of its kernels (no headline)
        stepmix = mixed_step(args, A0, Lb0, y0, info, ld)[0]
        msm = timed(stepmix, args.steps, args.warmup, "mixed")
        print(json.dumps({"form": "mixed", "workload": f"matern32-2d-n{n}", "ms_per_step": round(msm, 3),
                          "GFLOP/s": round(F / (msm * 1e-3) / 1e9, 2)}), flush=True)
        return

    def step64():
        L.copy_(A0)
        H.factor(L, info)
        z.copy_(y0)
        H.trsm(L, z)
        a.copy_(z)
        H.trsm(L, a, trans=True)
        H.logdet(L, ld)
        Lb.copy_(Lb0)
        H.adjoint(L, Lb)

    log(f"fp64: {args.warmup} warmup + {args.steps} timed steps")
    ms = timed(step64, args.steps, args.warmup, "fp64")
    H.check()   # raises if a one-launch solve sweep ran out of time
    tr_timed = None
    if not args.no_trace:
        # the same number of steps again, same schedule, with the library's
        # launch trace on: every kernel launch bracketed by HIP events on the
        # stream it runs on (the events cost about 4 % of a step, so the
        # step time above is taken without them)
        log("fp64: traced steps")
        H.trace_reset()
        H.trace_enable(True)
        timed(step64, args.steps, 0, "fp64 traced")
        tr_timed = H.trace_read()
        H.trace_enable(False)
    if int(info.item()) != 0:
        raise SystemExit(f"factor reported info={int(info.item())}")
    value = F / (ms * 1e-3) / 1e9
    log(f"fp64: {ms:.2f} ms/step, {value:.0f} GFLOP/s")
    rows = torch.randperm(n, generator=torch.Generator().manual_seed(0))[:64].to(dev)
    res_fact = (torch.linalg.norm(L[rows] @ L.T - A0[rows]) / torch.linalg.norm(A0[rows])).item()
    r = y0 - A0 @ a
    eta64 = (r.abs().max() / (A0.abs().sum(1).max() * a.abs().max() + y0.abs().max())).item()
    log(f"fp64: sampled |LL^T-A|/|A| = {res_fact:.2e}, direct-solve eta_inf = {eta64:.2e}")

    roof = None
    if not args.no_trace:
        tr = tr_timed
        # roofline kernel: the adjoint's row update Rbar -= [M; Cbar]^T [R; B]
        # (split-K slices), the class with the most time in the step's trace
        # (33 ms against 31.5 for the left update Bbar -= Cbar R with
        # 512-blocks); its launches overlap the diagonal chain of the next
        # block on the other stream, as in every timed step
        dom = "adj_row_update"
        cnt, kms, kfl, kby = tr[dom]
        achieved = kfl / (kms * 1e-3) / 1e12
        serial = None
        if args.serial_classes:
            # one more step with lookahead off: every kernel then runs alone
            H.set_options(lookahead=0)
            H.trace_reset()
            H.trace_enable(True)
            step64()
            torch.cuda.synchronize()
            serial = {k: round(v[1], 3) for k, v in H.trace_read().items() if v[0]}
            H.trace_enable(False)
            H.set_options(lookahead=args.lookahead)
            log(f"serial classes (ms per step): {serial}")
        # wall clock of each phase of the step (main stream), for the breakdown
        def phase(fn, reps=2):
            return round(timed(fn, reps, 0), 3)
        phases = {"copy_A": phase(lambda: L.copy_(A0)),
                  "factor": phase(lambda: (L.copy_(A0), H.factor(L, info))) ,
                  "solves": phase(lambda: (z.copy_(y0), H.trsm(L, z), a.copy_(z), H.trsm(L, a, trans=True))),
                  "logdet": phase(lambda: H.logdet(L, ld)),
                  "adjoint": phase(lambda: (Lb.copy_(Lb0), H.adjoint(L, Lb)))}
        phases["factor"] = round(phases["factor"] - phases["copy_A"], 3)
        phases["adjoint"] = round(phases["adjoint"] - phases["copy_A"], 3)
        log(f"phases (ms, copies of the inputs removed): {phases}")
        roof = {"bound": "mfma", "kernel": dom,
                "schedule": f"{args.steps} traced steps after the timed ones (lookahead {args.lookahead}), HIP events per launch",
                "launches": cnt, "achieved": round(achieved, 3),
                "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f64"], 4),
                "traffic": measured_traffic(dom), "avg_launch_ms": round(kms / max(cnt, 1), 4),
                "algorithmic_flops_per_launch": round(kfl / max(cnt, 1)),
                "algorithmic_bytes_per_launch": round(kby / max(cnt, 1)),
                "classes_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in tr.items() if v[0]},
                "serial_classes_ms": serial, "phases_ms": phases}
        log(f"trace: {json.dumps(roof)}")

    # the library's defaults (include/gpchol.h, gpc_options.block and adjoint_group)
    adj_block = min(args.block, 512) if args.block else (512 if n >= 8192 else 256)
    adj_group = args.adjoint_group or (1 if adj_block >= 512 else 2)
    cfg = {"workload": f"matern32-2d-n{n} factor+solves+logdet+adjoint", "n": n, "form": "fp64",
           "factor_block": args.block or (512 if n >= 8192 else 256), "adjoint_block": adj_block,
           "lookahead": args.lookahead, "adjoint_group": adj_group, "frac_of_fp64_peak": round(value / 1e3 / PEAK_TFLOPS["f64"], 4),
           "factor_residual_sampled": res_fact, "solve_eta_inf": eta64}

    if not args.headline_only:
        # ---- mixed form with the FP64-refined solve
        stepmix, Lm, Lbm, xr, Hm, out = mixed_step(args, A0, Lb0, y0, info, ld)
        log(f"mixed: {args.warmup} warmup + {args.steps} timed steps")
        msm = timed(stepmix, args.steps, args.warmup, "mixed")
        Hm.check()
        trm = None
        if not args.no_trace:
            Hm.trace_reset()
            Hm.trace_enable(True)
            timed(stepmix, args.steps, 0, "mixed traced")
            trm = {k: round(v[1] / args.steps, 3) for k, v in Hm.trace_read().items() if v[0]}
            Hm.trace_enable(False)
        cpm = timed(lambda: Lm.copy_(A0), 2, 0)
        phm = {"factor": round(timed(lambda: (Lm.copy_(A0), Hm.factor(Lm, info)), 2, 0) - cpm, 3),
               "refined_solve": round(timed(lambda: Hm.solve_refined(A0, Lm, y0, x=xr, check=False), 2, 0), 3),
               "adjoint": round(timed(lambda: (Lbm.copy_(Lb0), Hm.adjoint(Lm, Lbm)), 2, 0) - cpm, 3)}
        log(f"mixed phases (ms): {phm}")
        log(f"mixed trace classes (ms per step, traced steps): {trm}")
        it, etam = int(out["it"].item()), float(out["eta"].item())
        eL = (torch.linalg.norm(Lm - L) / torch.linalg.norm(L)).item()
        eA = (torch.linalg.norm(Lbm - Lb) / torch.linalg.norm(Lb)).item()
        ea = (torch.linalg.norm(xr - a) / torch.linalg.norm(a)).item()
        vm = F / (msm * 1e-3) / 1e9
        log(f"mixed: {msm:.2f} ms/step, {vm:.0f} GFLOP/s, refine iters {it} eta {etam:.2e}, "
            f"err vs fp64: L {eL:.2e} Abar {eA:.2e} alpha {ea:.2e}")
        cfg["mixed"] = {"value": round(vm, 2), "unit": "GFLOP/s", "ms_per_step": round(msm, 3),
                        "factor_block": args.block or 256,
                        "speedup_vs_fp64": round(ms / msm, 3), "refine_iters": it, "refined_eta_inf": etam,
                        "frac_of_fp64_peak": round(vm / 1e3 / PEAK_TFLOPS["f64"], 4),
                        "frac_of_fp32_peak": round(vm / 1e3 / PEAK_TFLOPS["f32"], 4),
                        "phases_ms": phm, "classes_ms_per_step": trm,
                        "err_vs_fp64_path": {"L": eL, "Abar": eA, "alpha": ea},
                        "step": "factor (FP32 trailing updates) + FP64-refined solve + log-det + adjoint"}
        del Lm, Lbm, Hm
        del A0, Lb0, L, Lb
        torch.cuda.empty_cache()

        # ---- batched: 512 uneven matrices, one persistent graph-replayed launch
        log("generating se3d batch of 512")
        bc = W.c4()
        base0 = torch.from_numpy(bc["base"]).to(dev)
        lbar0 = torch.from_numpy(bc["Lbar"]).to(dev)
        bw, lw = torch.empty_like(base0), torch.empty_like(lbar0)
        binfo = torch.zeros(len(bc["n"]), dtype=torch.int32, device=dev)
        Hb = Handle()

        def stepb():
            bw.copy_(base0)
            lw.copy_(lbar0)
            Hb.factor_adjoint_batched(bc["n"], bc["off"], bw, lw, binfo)

        msb = timed(stepb, args.steps, args.warmup, "batched")
        Fb = float(sum(W.flops_factor(int(k)) + W.flops_adjoint(int(k)) for k in bc["n"]))
        Hb.trace_enable(True)
        Hb.trace_reset()
        stepb()
        kms_b = Hb.trace_read()["batched"][1]
        Hb.trace_enable(False)
        assert int(binfo.max().item()) == 0
        log(f"batched: {msb:.2f} ms/step (launch {kms_b:.2f} ms), {Fb / (kms_b * 1e-3) / 1e9:.0f} GFLOP/s")
        cfg["batched"] = {"workload": "se3d-batch512 n~U{32..1024} factor+adjoint", "matrices": len(bc["n"]),
                          "flops": Fb, "launch_ms": round(kms_b, 3), "ms_per_step_with_copies": round(msb, 3),
                          "value": round(Fb / (kms_b * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "form": "fp64"}
        # the same batch in the mixed form (FP32 trailing / B-bar / R-bar products)
        ref_l, ref_a = bw.clone(), lw.clone()
        Hbm = Handle()
        Hbm.set_options(precision=GPC_MIXED)

        def stepbm():
            bw.copy_(base0)
            lw.copy_(lbar0)
            Hbm.factor_adjoint_batched(bc["n"], bc["off"], bw, lw, binfo)

        msbm = timed(stepbm, args.steps, args.warmup, "batched mixed")
        Hbm.trace_enable(True)
        Hbm.trace_reset()
        stepbm()
        kms_bm = Hbm.trace_read()["batched"][1]
        Hbm.trace_enable(False)
        assert int(binfo.max().item()) == 0
        el = (torch.linalg.norm(bw - ref_l) / torch.linalg.norm(ref_l)).item()
        ea = (torch.linalg.norm(lw - ref_a) / torch.linalg.norm(ref_a)).item()
        log(f"batched mixed: launch {kms_bm:.2f} ms, err vs fp64 batch: L {el:.2e} Abar {ea:.2e}")
        cfg["batched"]["mixed"] = {"launch_ms": round(kms_bm, 3), "ms_per_step_with_copies": round(msbm, 3),
                                   "value": round(Fb / (kms_bm * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                                   "err_vs_fp64_batch": {"L": el, "Abar": ea}}
        del base0, lbar0, bw, lw, bc, Hb, Hbm, ref_l, ref_a
        torch.cuda.empty_cache()

        # ---- GP marginal log-likelihood gradient at n = 30000
        log("generating se-ard 8-d n=30000")
        gc = W.c5()
        X = torch.from_numpy(gc["x"]).to(dev)
        Y = torch.from_numpy(gc["y"]).to(dev)
        thetas = torch.from_numpy(gc["thetas"]).to(dev)
        ngp = X.shape[0]
        Hg = Handle()
        gp = {}
        for name, prec in (("fp64", GPC_FP64), ("mixed", GPC_MIXED)):
            def ev(e=[0]):
                th = thetas[e[0] % thetas.shape[0]].clone().requires_grad_(True)
                e[0] += 1
                f = gp_mll(X, Y, th, precision=prec, handle=Hg, check=False)
                f.backward()
                return f, th.grad
            log(f"gp {name}: 1 warmup + {args.gp_evals} timed evaluations")
            msg = timed(ev, args.gp_evals, 1, f"gp {name}")
            Hg.check()
            Fg = W.flops_factor(ngp) + W.flops_adjoint(ngp)
            ne = thetas.shape[0]
            gp[name] = {"ms_per_eval": round(msg, 2), "gflops_factor_adjoint": round(Fg / (msg * 1e-3) / 1e9, 2),
                        f"s_for_{ne}_evals": round(msg * ne / 1e3, 2),
                        "timing": (f"{args.gp_evals} evaluations timed (jittered thetas 1..{args.gp_evals} of {ne}, "
                                   f"after 1 warmup); s_for_{ne}_evals = ms_per_eval x {ne}"
                                   + ("" if args.gp_evals >= ne else ", extrapolated"))}
            log(f"gp {name}: {msg:.1f} ms per value+gradient evaluation")
        th0 = thetas[0].clone().requires_grad_(True)
        f64v = gp_mll(X, Y, th0, precision=GPC_FP64, handle=Hg)
        f64v.backward()
        g64 = th0.grad.clone()
        th1 = thetas[0].clone().requires_grad_(True)
        fmv = gp_mll(X, Y, th1, precision=GPC_MIXED, handle=Hg)
        fmv.backward()
        gp["mixed"]["err_vs_fp64"] = {"f": abs((fmv - f64v).item()) / abs(f64v.item()),
                                      "grad": (torch.linalg.norm(th1.grad - g64) / torch.linalg.norm(g64)).item()}
        gp["speedup_mixed_vs_fp64"] = round(gp["fp64"]["ms_per_eval"] / gp["mixed"]["ms_per_eval"], 3)
        cfg["gp"] = {"workload": f"se-ard8d-n{ngp} GP marginal log-likelihood + gradient (10 hyperparameters)",
                     "evals_timed": args.gp_evals, **gp}
        del X, Y, Hg
        torch.cuda.empty_cache()

    if not args.headline_only and not args.no_ops:
        log("operations beside the factor")
        cfg["ops"] = ops_bench()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle) at n={args.cpu_sample}")
        cpu = cpu_baseline(args.cpu_sample, not args.no_oracle_configs)

    out = {"metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg, "roofline": roof,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
