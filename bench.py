#!/usr/bin/env python3
"""Benchmark of randomized block-CG on one MI355X.

Headline workload: the dense SPD system with d = 8192, lambda_i = i^-1.5,
mu = 1e-4, b ~ N(0, I) and a 8192 x 64 Gaussian block Omega, solved to a
relative FP64 residual of 1e-10.  One step = one complete solve through the
C ABI (rbcg_solve): the mixed-precision path (FP32 MFMA block products with
FP32 accumulation, everything else FP64, FP64 iterative refinement).  The
plain FP64 GPU solve of the same system is timed beside it.

In the same run (sub-objects of the one JSON line, each timed with its own
step count, skipped with --no-ridge / --no-batch / --no-outofcore):
  ridge      the 64-shift ridge path, Z = G diag(exp(-j/400)) with n = 200000,
             d = 4096, k = 128: BF16 products + FP64 refinement against FP64
             products, with the HBM and MFMA rates of the BF16 Gram product;
  batched    200 independent dense SPD systems of uneven d and k in one
             batched call (FP64 products, and FP32 products + refinement)
             against the same systems solved one call at a time in FP64;
  outofcore  the headline system with A in page-locked host memory, streamed
             in row chunks for every product (the paper's wall-clock
             setting): block-CG in FP64, with FP32 chunks + FP64 refinement,
             and Nystrom PCG from the same Omega.

Printed (one JSON line): solves/s of the mixed path, the plain FP64 rate,
the Nystrom-PCG rate with the same Omega (the paper's comparison method),
the error of each against the FP64 oracle, the roofline of the dominant
kernel (the block-product GEMM, timed with HIP events on the library's
stream over the timed region), the CPU oracle's rate on this host (about
10 s of complete solves, with the CPU model and thread count), and the
sub-objects above.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
PEAK_HBM_GBS = 8000.0

# HBM traffic of the dominant kernel comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs summarised in
# this file; it is used only while the kernel's source is the one the counters were taken on.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_block_product_f32_d8192.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2501_18717_amd", "csrc", f) for f in ("device_common.inc", "mv_f32_wide.hip")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the FP32 block product, or None when absent or stale."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ":" in ln and ln.startswith("- "):
            key, val = ln[2:].split(":", 1)
            vals[key.strip()] = val.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_probe(dev):
    """Three untimed 1 GiB device-to-device copies: a known-size reference for HBM counter runs."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    log("copy probe: 3 x 1 GiB device copies done")


def cpu_model():
    """Model name of the host CPU (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.lower().startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or None


def a_err(A, mu, x, xref):
    import numpy as np
    e = x - xref
    return float(np.sqrt(max(e @ (A @ e) + mu * (e @ e), 0.0) / (xref @ (A @ xref) + mu * (xref @ xref))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-ridge", action="store_true", help="default run: skip the ridge-path sub-object")
    ap.add_argument("--no-batch", action="store_true", help="default run: skip the batched sub-object")
    ap.add_argument("--no-nystrom", action="store_true", help="default run: skip the Nystrom-PCG legs")
    ap.add_argument("--no-outofcore", action="store_true", help="default run: skip the out-of-core sub-object")
    ap.add_argument("--sub-steps", type=int, default=2,
                    help="default run: timed steps of the ridge and batched sub-objects")
    ap.add_argument("--workload", choices=["dense", "batch", "ridge", "sqrt", "outofcore"], default="dense",
                    help="dense: the d=8192 system (default); batch: uneven independent systems; "
                         "ridge: the 64-shift ridge path, n=200000, d=4096; sqrt: RBF sampling, 16384 points; "
                         "outofcore: the d=8192 system with A streamed from host memory")
    ap.add_argument("--nsys", type=int, default=200, help="batch workload: number of systems")
    ap.add_argument("--no-fp64", action="store_true", help="ridge workload: skip the FP64-product leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run three untimed 1 GiB device-to-device copies (known-size reference for "
                         "HBM counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2501_18717_amd import rbcg

    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "ridge":
        run_ridge(args)
        return
    if args.workload == "sqrt":
        run_sqrt(args)
        return
    if args.workload == "outofcore":
        run_outofcore(args)
        return

    d, k, mu, rtol = 8192, 64, 1e-4, 1e-10
    log("generating the d=8192 system (seeded)")
    t0 = time.time()
    P = synth.dense_problem(2, d, 1.5, k, mu)
    log(f"generated in {time.time() - t0:.1f}s")
    A, b, Om = P["A"], P["b"], P["omega"]
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.from_numpy(b).to(dev)
    omd = torch.from_numpy(Om).to(dev)
    if args.copy_probe:
        copy_probe(dev)
    ctx = rbcg.Context()
    op = rbcg.DenseOperator(ctx, Ad, lo="f32")
    x_mix = torch.zeros_like(bd)
    x_64 = torch.zeros_like(bd)
    o_mix = rbcg.opts(48, rtol=rtol, matvec="f32", refine_max=8)
    o_64 = rbcg.opts(48, rtol=rtol, matvec="f64", refine_max=3)

    def solve(x, o):
        rc, info = rbcg.solve(ctx, [op], [mu], [bd], [omd], [x], [o])
        return info[0]

    for _ in range(args.warmup):
        solve(x_mix, o_mix)
        solve(x_64, o_64)
    torch.cuda.synchronize()

    # ---- timed: mixed precision (the reported value).  Every block product is timed with a
    # pair of HIP events (the markers cost the solve about 13 us per product; timing only every
    # fourth launch measured launch durations 10-15% below the rocprofv3 trace of the same
    # launches, so all of them are timed).
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info_mix = solve(x_mix, o_mix)
    torch.cuda.synchronize()
    t_mix = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    log(f"mixed: {args.steps} solves in {t_mix:.3f}s; {info_mix}")

    # ---- plain FP64 on the GPU, same protocol
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info_64 = solve(x_64, o_64)
    torch.cuda.synchronize()
    t_64 = time.perf_counter() - t0
    prof64 = ctx.profile_read()
    ctx.profile(False)
    log(f"fp64: {args.steps} solves in {t_64:.3f}s; {info_64}")

    # ---- Nystrom PCG from the same Omega (the paper's comparison method, Sec. 2.2.2), FP64 products:
    # preconditioner of rank 64 s from K_s(A, Omega) for s = 1 and 2, then single-vector PCG to
    # the same rtol; each call also timed stopped after one iteration (the construction: s block
    # loads, the basis, the r x r eigendecompositions, plus one iteration and the residual)
    ny = {}
    x_ny = torch.zeros_like(bd)
    for s_ny in (() if args.no_nystrom else (1, 2)):
        o_ny = rbcg.opts(2000, rtol=rtol)
        o_ny1 = rbcg.opts(1)
        for _ in range(args.warmup):
            rbcg.nystrom_pcg(ctx, op, bd, omd, s_ny, mu, x_ny, o_ny, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rbcg.nystrom_pcg(ctx, op, bd, omd, s_ny, mu, x_ny, o_ny1, check=False)
        torch.cuda.synchronize()
        t_ny1 = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rc_ny, info_ny, _, rank_ny, theta_ny = rbcg.nystrom_pcg(ctx, op, bd, omd, s_ny, mu, x_ny, o_ny,
                                                                    check=False)
        torch.cuda.synchronize()
        t_ny = time.perf_counter() - t0
        log(f"nystrom pcg s={s_ny}: {args.steps} solves in {t_ny:.3f}s; {info_ny}")
        ny[s_ny] = {"value": args.steps / t_ny, "unit": "solves/s", "ms_per_step": 1e3 * t_ny / args.steps,
                    "s": s_ny, "rank": rank_ny, "theta": theta_ny, "status": rc_ny, "iters": info_ny["iters"],
                    "matrix_loads": info_ny["matrix_loads"], "relres": info_ny["relres"],
                    "ms_construction_plus_one_iteration": 1e3 * t_ny1 / args.steps,
                    "x": x_ny.cpu().numpy()}

    xm = x_mix.cpu().numpy()
    x6 = x_64.cpu().numpy()

    # ---- CPU oracle: complete solves (t = the FP64 GPU iteration count) on this host, repeated
    # until about 10 s of CPU work (at most 40 solves)
    cpu = None
    err_mix = err_64 = None
    if not args.no_cpu:
        from oracle import block_cg as ob
        threads = None
        try:
            import threadpoolctl
            threads = max((p.get("num_threads", 0) for p in threadpoolctl.threadpool_info()), default=None)
        except Exception:
            pass
        t_ref = int(info_64["iters"])
        log(f"CPU oracle: block-CG with t={t_ref} block products")
        t0 = time.perf_counter()
        n_cpu = 0
        while True:
            Xo, _ = ob.bcg(A, [mu], b, Om, t_ref)
            n_cpu += 1
            if time.perf_counter() - t0 >= 10.0 or n_cpu >= 40:
                break
        t_all = time.perf_counter() - t0
        t_cpu = t_all / n_cpu
        xo = Xo[0]
        rel_o = float(np.linalg.norm(b - (A @ xo + mu * xo)) / np.linalg.norm(b))
        err_mix = a_err(A, mu, xm, xo)
        err_64 = a_err(A, mu, x6, xo)
        for v in ny.values():
            v["rel_a_err_vs_oracle"] = a_err(A, mu, v["x"], xo)
        cpu = {"value": 1.0 / t_cpu, "unit": "solves/s", "cores": int(threads or os.cpu_count() or 1),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": f"{n_cpu} full solves of the d=8192 k=64 system by the FP64 oracle (t={t_ref} block "
                         f"products each, relres {rel_o:.2e}) in {t_all:.1f}s"}
        log(f"oracle: {n_cpu} solves in {t_all:.1f}s, err mixed {err_mix:.2e}, err fp64 {err_64:.2e}")

    # ---- roofline of the dominant kernel: the FP32 block-product GEMM (2 d^2 m flops per launch)
    avg_ms = prof["ms"] / max(prof["launches"], 1)
    flops_per = prof["flops"] / max(prof["launches"], 1)
    achieved = flops_per / (avg_ms * 1e-3) / 1e12
    avg_ms64 = prof64["ms"] / max(prof64["launches"], 1)
    flops64 = prof64["flops"] / max(prof64["launches"], 1)
    out = {
        "metric": "solves/s at 1e-8 rel A-norm err: mixed+batched vs plain FP64; HBM/MFMA % peak",
        "value": args.steps / t_mix,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_mix / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mfma+f64",
        "data": "synthetic",
        "config": {"workload": "dense SPD d=8192, lambda_i=i^-1.5, mu=1e-4, k=64, rtol=1e-10 (FP32 MFMA block "
                               "products + FP64 refinement)", "d": d, "k": k, "mu": mu, "rtol": rtol},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["f32"], "traffic": measured_traffic(),
                     "kernel": "k_mv_wide<2, 1, 4> (A X block product, FP32 32x32x2 MFMA + one VALU column)",
                     "avg_launch_ms": avg_ms, "launches": prof["launches"]},
        "fp64_gpu": {"value": args.steps / t_64, "unit": "solves/s", "ms_per_step": 1e3 * t_64 / args.steps,
                     "iters": info_64["iters"], "relres": info_64["relres"], "rel_a_err_vs_oracle": err_64,
                     "matvec_avg_launch_ms": avg_ms64,
                     "matvec_tflops": flops64 / (avg_ms64 * 1e-3) / 1e12 if avg_ms64 > 0 else None},
        "mixed": {"iters_last_sweep": info_mix["iters"], "refine_sweeps": info_mix["refine_sweeps"],
                  "matrix_loads": info_mix["matrix_loads"], "relres": info_mix["relres"],
                  "rel_a_err_vs_oracle": err_mix},
        "speedup_mixed_vs_fp64": t_64 / t_mix,
        "nystrom_pcg": [dict({k: v for k, v in ny[s_].items() if k != "x"},
                             note="Nystrom PCG from the same Omega (rank 64 s from K_s(A, Omega)), FP64 products, "
                                  "single-vector loads after the s block loads") for s_ in sorted(ny)],
        "cpu_baseline": cpu,
    }
    # free the dense system before the sub-objects
    del op, ctx, Ad, bd, omd, x_mix, x_64
    torch.cuda.empty_cache()
    if not args.no_ridge:
        out["ridge"] = ridge_leg(args.sub_steps, 1)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = batch_leg(args.sub_steps, 1, args.nsys)
        torch.cuda.empty_cache()
    if not args.no_outofcore:
        out["outofcore"] = outofcore_leg(args.sub_steps, 1)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def run_outofcore(args):
    sub = outofcore_leg(args.steps, args.warmup)
    out = {
        "metric": "solves/s at 1e-8 rel A-norm err: mixed+batched vs plain FP64; HBM/MFMA % peak",
        "value": sub["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sub["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": sub.pop("workload")},
    }
    out.update({k: v for k, v in sub.items() if k not in ("value", "ms_per_step", "unit")})
    print(json.dumps(out), flush=True)


def outofcore_leg(steps, warmup):
    """The out-of-core setting of the paper's wall-clock experiment (Sec. 7.1.1, intro figure):
    the d = 8192 system's A stays in page-locked host memory and every product streams it to the
    GPU in 8 row chunks of 1024 rows.  Block-CG (k = 64, FP64 products), block-CG with FP32 chunks
    and FP64 refinement, and Nystrom PCG from the same Omega (s = 1, rank 64) solve to rtol 1e-10;
    the run time follows the matrix-loads and their bytes."""
    import torch

    import synth
    from paper_2501_18717_amd import rbcg

    d, k, mu, rtol, chunk = 8192, 64, 1e-4, 1e-10, 1024
    P = synth.dense_problem(2, d, 1.5, k, mu)
    Ah = torch.from_numpy(P["A"]).pin_memory()
    dev = torch.device("cuda:0")
    bd = torch.from_numpy(P["b"]).to(dev)
    omd = torch.from_numpy(P["omega"]).to(dev)
    # host-to-device copy rate of the whole matrix from the same page-locked buffer (reference)
    tmp = torch.empty((d, d), dtype=torch.float64, device=dev)
    tmp.copy_(Ah, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        tmp.copy_(Ah, non_blocking=True)
    torch.cuda.synchronize()
    h2d_gbs = 3 * d * d * 8.0 / (time.perf_counter() - t0) / 1e9
    del tmp
    torch.cuda.empty_cache()
    ctx = rbcg.Context()
    op = rbcg.DenseHostOperator(ctx, Ah, chunk, lo="f32")
    x = torch.zeros_like(bd)
    xm = torch.zeros_like(bd)
    o = rbcg.opts(48, rtol=rtol)
    o_mix = rbcg.opts(48, rtol=rtol, matvec="f32", refine_max=8)

    def solve(xv, ov):
        rc, info = rbcg.solve(ctx, [op], [mu], [bd], [omd], [xv], [ov], check=False)
        return rc, info[0]

    def timed(xv, ov):
        for _ in range(warmup):
            solve(xv, ov)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = solve(xv, ov)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    t_bcg, (rc, info) = timed(x, o)
    log(f"out-of-core block-CG: {1e3 * t_bcg:.1f} ms per solve, rc={rc}, {info}")
    t_mix, (rc_m, info_m) = timed(xm, o_mix)
    log(f"out-of-core block-CG, FP32 chunks + FP64 refinement: {1e3 * t_mix:.1f} ms per solve, rc={rc_m}, "
        f"{info_m}")
    o_ny = rbcg.opts(2000, rtol=rtol)
    xn = torch.zeros_like(bd)
    for _ in range(warmup):
        rbcg.nystrom_pcg(ctx, op, bd, omd, 1, mu, xn, o_ny, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc_ny, info_ny, _, rank_ny, _ = rbcg.nystrom_pcg(ctx, op, bd, omd, 1, mu, xn, o_ny, check=False)
    torch.cuda.synchronize()
    t_ny = (time.perf_counter() - t0) / steps
    log(f"out-of-core Nystrom PCG s=1: {1e3 * t_ny:.1f} ms per solve, rc={rc_ny}, {info_ny}")
    # the answers against each other (each converged to rtol 1e-10 in FP64)
    Ad = torch.from_numpy(P["A"]).to(dev)

    def adiff(u, v):
        e = u - v
        return float(torch.sqrt((e @ (Ad @ e) + mu * (e @ e)) / (v @ (Ad @ v) + mu * (v @ v))))

    diff = adiff(xn, x)
    diff_m = adiff(xm, x)
    del Ad
    gb = d * d * 8.0 / 1e9
    return {
        "workload": "dense SPD d=8192 (lambda_i=i^-1.5, mu=1e-4) with A in page-locked host memory, "
                    "streamed in 8 row chunks of 1024 rows per product; rtol 1e-10, FP64 products",
        "value": 1.0 / t_bcg, "unit": "solves/s", "ms_per_step": 1e3 * t_bcg, "status": rc,
        "matrix_loads": info["matrix_loads"], "iters": info["iters"], "relres": info["relres"],
        "stream_GBs": info["matrix_loads"] * gb / t_bcg, "h2d_copy_GBs": h2d_gbs,
        "nystrom_pcg": {"value": 1.0 / t_ny, "unit": "solves/s", "ms_per_step": 1e3 * t_ny, "s": 1,
                        "rank": rank_ny, "status": rc_ny, "matrix_loads": info_ny["matrix_loads"],
                        "iters": info_ny["iters"], "relres": info_ny["relres"],
                        "stream_GBs": info_ny["matrix_loads"] * gb / t_ny},
        "mixed": {"value": 1.0 / t_mix, "unit": "solves/s", "ms_per_step": 1e3 * t_mix, "status": rc_m,
                  "matrix_loads": info_m["matrix_loads"], "refine_sweeps": info_m["refine_sweeps"],
                  "relres": info_m["relres"], "rel_a_diff_vs_fp64": diff_m,
                  "note": "FP32 copy of A streamed (half the bytes per load), FP64 residuals stream A"},
        "speedup_mixed_vs_fp64": t_bcg / t_mix,
        "speedup_bcg_vs_nystrom": t_ny / t_bcg,
        "rel_a_diff_bcg_vs_nystrom": diff,
        "note": "stream_GBs: matrix-loads x 0.537 GB per solve over its wall time; h2d_copy_GBs: one "
                "host-to-device copy of A from the same buffer",
    }


def run_batch(args):
    sub = batch_leg(args.steps, args.warmup, args.nsys)
    out = {
        "metric": "solves/s at 1e-8 rel A-norm err: mixed+batched vs plain FP64; HBM/MFMA % peak",
        "value": sub["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sub["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": sub.pop("workload"), "nsys": sub["nsys"]},
    }
    out.update({k: v for k, v in sub.items() if k not in ("value", "ms_per_step", "unit")})
    print(json.dumps(out), flush=True)


def batch_leg(steps, warmup, nsys):
    """Independent systems of uneven size: d ~ U{1000..16000}, lambda_i = i^-p with p ~ U[1, 3],
    mu = 10^U[-6, -2], k ~ U{8, 16, 32, 64, 128}; eigenbases from four Householder reflectors,
    formed on the GPU.  One step = all systems solved to rtol 1e-10 (FP64 products) by one batched
    rbcg_solve call; the same systems solved one call at a time are timed beside it."""
    import numpy as np
    import torch

    import synth
    from paper_2501_18717_amd import rbcg

    rtol, t_max = 1e-10, 64
    dev = torch.device("cuda:0")
    params = synth.batch_params(5, nsys, 1000, 16000)
    log(f"batch: forming {len(params)} systems on the GPU")
    t0 = time.time()
    ctx = rbcg.Context()
    ops, mus, bs, oms, Ads = [], [], [], [], []
    for pr in params:
        S = synth.batch_system_fast(5, pr)
        A = synth.spd_from_reflectors_torch(S["lam"], S["V"], dev)
        Ads.append(A)
        ops.append(rbcg.DenseOperator(ctx, A, lo="f32"))
        mus.append(S["mu"])
        bs.append(torch.from_numpy(S["b"]).to(dev))
        oms.append(torch.from_numpy(S["omega"]).to(dev))
    torch.cuda.synchronize()
    gb = sum(p["d"] ** 2 for p in params) * 8 / 1e9
    log(f"batch: formed in {time.time() - t0:.1f}s, {gb:.1f} GB of FP64 matrices")
    opts = [rbcg.opts(t_max, rtol=rtol, matvec="f64", refine_max=3) for _ in params]
    opts_mx = [rbcg.opts(t_max, rtol=rtol, matvec="f32", refine_max=20) for _ in params]

    def batched(o=opts):
        xs = [torch.zeros_like(b) for b in bs]
        rc, info = rbcg.solve(ctx, ops, mus, bs, oms, xs, o, check=False)
        return rc, info

    def one_at_a_time():
        infos = []
        rc = 0
        for i in range(len(params)):
            x = torch.zeros_like(bs[i])
            r, info = rbcg.solve(ctx, [ops[i]], [mus[i]], [bs[i]], [oms[i]], [x], [opts[i]], check=False)
            rc = rc or r
            infos += info
        return rc, infos

    for _ in range(warmup):
        batched()
        one_at_a_time()
    torch.cuda.synchronize()
    t_b = 0.0
    for _ in range(steps):
        t1 = time.time()
        rc_b, info_b = batched()
        torch.cuda.synchronize()
        t_b += time.time() - t1
        log(f"batch: batched call {time.time() - t1:.2f}s rc={rc_b}")
    batched(opts_mx)
    torch.cuda.synchronize()
    t_m = 0.0
    for _ in range(steps):
        t1 = time.time()
        rc_m, info_m = batched(opts_mx)
        torch.cuda.synchronize()
        t_m += time.time() - t1
        log(f"batch: batched mixed call {time.time() - t1:.2f}s rc={rc_m}")
    t_1 = 0.0
    for _ in range(steps):
        t1 = time.time()
        rc_1, info_1 = one_at_a_time()
        torch.cuda.synchronize()
        t_1 += time.time() - t1
        log(f"batch: one at a time {time.time() - t1:.2f}s rc={rc_1}")
    loads = [i["matrix_loads"] for i in info_b]
    flops = sum(2.0 * p["d"] ** 2 * (p["k"] + 1) * i["matrix_loads"] for p, i in zip(params, info_b))
    sub = {
        "workload": f"batch of {len(params)} independent dense SPD systems, d in [1000, 16000], "
                    "lambda_i=i^-p p in [1,3], mu in [1e-6, 1e-2], k in {8..128}, rtol 1e-10",
        "nsys": len(params), "gbytes": gb, "steps": steps,
        "value": len(params) * steps / t_b, "unit": "solves/s", "ms_per_step": 1e3 * t_b / steps,
        "note": "value: FP64 products, one batched call",
        "one_at_a_time": {"value": len(params) * steps / t_1, "unit": "solves/s",
                          "ms_per_step": 1e3 * t_1 / steps, "note": "FP64 products, one call per system"},
        "batched_mixed": {"value": len(params) * steps / t_m, "unit": "solves/s",
                          "ms_per_step": 1e3 * t_m / steps, "status": rc_m,
                          "max_relres": max(i["relres"] for i in info_m),
                          "loads_total": sum(i["matrix_loads"] for i in info_m),
                          "note": "FP32-MFMA products + FP64 refinement, one batched call"},
        "speedup_batched_mixed_vs_one_at_a_time_fp64": t_1 / t_m,
        "speedup_batched_vs_one_at_a_time": t_1 / t_b,
        "status": {"batched": rc_b, "one_at_a_time": rc_1,
                   "max_relres": max(i["relres"] for i in info_b),
                   "loads_min_max": [min(loads), max(loads)]},
        "block_product_tflops_avg": flops * steps / t_b / 1e12,
    }
    del ops, Ads, bs, oms, ctx
    return sub


def _timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    t = 0.0
    out = None
    for _ in range(steps):
        t1 = time.time()
        out = fn()
        torch.cuda.synchronize()
        t += time.time() - t1
    return t, out


def run_ridge(args):
    if args.copy_probe:
        import torch
        copy_probe(torch.device("cuda:0"))
    sub = ridge_leg(args.steps, args.warmup, fp64=not args.no_fp64)
    out = {
        "metric": "solves/s at 1e-8 rel A-norm err: mixed+batched vs plain FP64; HBM/MFMA % peak",
        "value": sub["value"], "unit": sub["unit"], "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sub["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-mfma+f64", "data": "synthetic",
        "config": {"workload": sub.pop("workload"), "n": 200000, "d": 4096, "k": 128, "shifts": sub["shifts"]},
    }
    out.update({k: v for k, v in sub.items() if k not in ("value", "ms_per_step", "unit")})
    print(json.dumps(out), flush=True)


def ridge_leg(steps, warmup, fp64=True):
    """Ridge path: Z = G diag(exp(-j/400)) (n = 200000, d = 4096, FP32), 64 shifts log-spaced over
    [1e-6, 1], k = 128.  One step = the whole path: plain FP64 products at t = 32 (the Krylov space
    is the whole space, 32 * 129 >= 4096), and BF16 products with FP64 refinement to rtol 2e-12.
    The BF16 Gram product's two passes (Y = Z X, then Z^T Y) are timed with HIP events on the
    library's stream over the BF16 timed region."""
    import torch

    import synth
    from paper_2501_18717_amd import rbcg

    n, d, k = 200000, 4096, 128
    log(f"ridge: generating Z ({n} x {d}, seeded)")
    t0 = time.time()
    P = synth.ridge_problem(3, n, d, k)
    log(f"ridge: generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ctx = rbcg.Context()
    Zd = torch.from_numpy(P["Z"]).to(dev)
    op64 = rbcg.GramOperator(ctx, Zd, lo="f64")
    op16 = rbcg.GramOperator(ctx, Zd, lo="bf16")
    bd = torch.from_numpy(P["b"]).to(dev)
    omd = torch.from_numpy(P["omega"]).to(dev)
    mus = list(P["mus"])
    del P
    X = torch.zeros((len(mus), d), dtype=torch.float64, device=dev)
    o64 = rbcg.opts(32)
    o16 = rbcg.opts(32, rtol=2e-12, matvec="bf16", refine_max=20)
    for _ in range(warmup):
        if fp64:
            rbcg.path(ctx, op64, bd, omd, mus, X, o64, check=False)
        rbcg.path(ctx, op16, bd, omd, mus, X, o16, check=False)
    if fp64:
        t64, (rc64, i64) = _timed(lambda: rbcg.path(ctx, op64, bd, omd, mus, X, o64, check=False), steps)
        log(f"ridge: fp64 {t64 / steps:.3f}s per path rc={rc64}")
    ctx.profile(True)
    t16, (rc16, i16) = _timed(lambda: rbcg.path(ctx, op16, bd, omd, mus, X, o16, check=False), steps)
    prof = ctx.profile_read()
    ctx.profile(False)
    log(f"ridge: bf16 {t16 / steps:.3f}s per path rc={rc16} sweeps {i16[0]['refine_sweeps']}; product passes {prof}")
    # one pass streams Z (BF16, 2 n d bytes) once: the algorithmic bytes; its MFMA work is 3 x 2 n d N flops
    # (the right operand in three BF16 parts)
    npass = max(prof["launches"], 1)
    avg_ms = prof["ms"] / npass
    gbs = prof["bytes"] / npass / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    tfs = 3.0 * prof["flops"] / npass / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else None
    sub = {
        "workload": "ridge path n=200000 d=4096 k=128, 64 shifts in [1e-6, 1], BF16 Z with FP64 refinement to "
                    "rtol 2e-12",
        "shifts": len(mus), "steps": steps,
        "value": len(mus) * steps / t16, "unit": "shift solves/s", "ms_per_step": 1e3 * t16 / steps,
        "note": "value: BF16-MFMA products + FP64 refinement",
        "fp64_gpu": {"value": len(mus) * steps / t64, "unit": "shift solves/s",
                     "ms_per_step": 1e3 * t64 / steps, "status": rc64, "loads": i64[0]["matrix_loads"],
                     "relres_max": max(i["relres"] for i in i64)} if fp64 else None,
        "mixed": {"status": rc16, "refine_sweeps": i16[0]["refine_sweeps"], "loads": i16[0]["matrix_loads"],
                  "relres_max": max(i["relres"] for i in i16)},
        "speedup_mixed_vs_fp64": t64 / t16 if fp64 else None,
        "gram_bf16_pass": {"kernel": "k_gram_bf16<9> (one pass over Z or Z^T, 16x16x32 BF16 MFMA)",
                           "launches": prof["launches"], "avg_launch_ms": avg_ms,
                           "algorithmic_bytes": prof["bytes"] / npass, "achieved_GBs": gbs,
                           "hbm_frac": gbs / PEAK_HBM_GBS if gbs else None,
                           "mfma_TFLOPs": tfs, "mfma_frac": tfs / PEAK_TFLOPS["bf16"] if tfs else None},
    }
    del op64, op16, Zd, ctx
    return sub


def run_sqrt(args):
    """Gaussian sampling A^(1/2) B: RBF kernel on 16384 points in [0,1]^3 (length scale 0.1, nugget
    1e-6), 256 samples in groups of 32, 32 quadrature nodes, t = 64 block products.  One step = all
    256 samples, with FP64 products and with FP32 products; then the inverse square root A^(-1/2) B
    (FP64 products) on the same samples."""
    import torch

    import synth
    from paper_2501_18717_amd import rbcg

    log("sqrt: generating the RBF kernel matrix (16384 points, seeded)")
    P = synth.rbf_problem(4, 16384, 256)
    dev = torch.device("cuda:0")
    ctx = rbcg.Context()
    Ad = torch.from_numpy(P["A"]).to(dev)
    op = rbcg.DenseOperator(ctx, Ad, lo="f32")
    Bd = torch.from_numpy(P["B"]).to(dev)
    Y = torch.zeros_like(Bd)
    o64 = rbcg.opts(64, nquad=32, group=32)
    o32 = rbcg.opts(64, nquad=32, group=32, matvec="f32")
    for _ in range(args.warmup):
        rbcg.sqrt_apply(ctx, op, Bd, Y, o64, check=False)
        rbcg.sqrt_apply(ctx, op, Bd, Y, o32, check=False)
    t64, (rc64, _) = _timed(lambda: rbcg.sqrt_apply(ctx, op, Bd, Y, o64, check=False), args.steps)
    t32, (rc32, _) = _timed(lambda: rbcg.sqrt_apply(ctx, op, Bd, Y, o32, check=False), args.steps)
    log(f"sqrt: fp64 {t64 / args.steps:.3f}s, fp32 {t32 / args.steps:.3f}s per 256 samples")
    # the inverse square root (whitening) runs the same spaces and rule without the leading A
    for _ in range(args.warmup):
        rbcg.invsqrt_apply(ctx, op, Bd, Y, o64, check=False)
    ti, (rci, _) = _timed(lambda: rbcg.invsqrt_apply(ctx, op, Bd, Y, o64, check=False), args.steps)
    log(f"inverse sqrt: fp64 {ti / args.steps:.3f}s per 256 samples")
    out = {
        "metric": "solves/s at 1e-8 rel A-norm err: mixed+batched vs plain FP64; HBM/MFMA % peak",
        "value": 256 * args.steps / t64, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t64 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "RBF sampling 16384 points, 256 samples (8 groups of 32), 32 nodes, t=64, FP64 "
                               "products", "d": 16384, "samples": 256, "nodes": 32, "t": 64},
        "fp32_products": {"value": 256 * args.steps / t32, "unit": "samples/s", "ms_per_step": 1e3 * t32 / args.steps,
                          "status": rc32, "note": "about 6e-3 from the FP64 result (no refinement for sampling)"},
        "inverse_sqrt": {"value": 256 * args.steps / ti, "unit": "samples/s", "ms_per_step": 1e3 * ti / args.steps,
                         "status": rci, "note": "A^(-1/2) B, FP64 products, same spaces and rule"},
        "status": rc64,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
