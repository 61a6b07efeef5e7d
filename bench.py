#!/usr/bin/env python3
"""Benchmark of randomized block-CG on one MI355X.

Workload (default): the dense SPD system with d = 8192, lambda_i = i^-1.5,
mu = 1e-4, b ~ N(0, I) and a 8192 x 64 Gaussian block Omega, solved to a
relative FP64 residual of 1e-10.  One step = one complete solve through the
C ABI (rbcg_solve): the mixed-precision path (FP32 MFMA block products with
FP32 accumulation, everything else FP64, FP64 iterative refinement).  The
plain FP64 GPU solve of the same system is timed beside it.

Printed (one JSON line): solves/s of the mixed path, the plain FP64 rate,
the error of both against the FP64 oracle, the roofline of the dominant
kernel (the block-product GEMM, timed with HIP events on the library's
stream over the timed region), and the CPU oracle's rate on this host.
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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2501_18717_amd", "csrc", f) for f in ("device_common.inc", "gemm_nt_f32.hip")]


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
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 3 x 1 GiB device copies done")
    ctx = rbcg.Context()
    op = rbcg.DenseOperator(ctx, Ad, lo="f32")
    x_mix = torch.zeros_like(bd)
    x_64 = torch.zeros_like(bd)
    o_mix = rbcg.opts(48, rtol=rtol, matvec="f32", refine_max=6)
    o_64 = rbcg.opts(48, rtol=rtol, matvec="f64", refine_max=3)

    def solve(x, o):
        rc, info = rbcg.solve(ctx, [op], [mu], [bd], [omd], [x], [o])
        return info[0]

    for _ in range(args.warmup):
        solve(x_mix, o_mix)
        solve(x_64, o_64)
    torch.cuda.synchronize()

    # ---- timed: mixed precision (the reported value)
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

    xm = x_mix.cpu().numpy()
    x6 = x_64.cpu().numpy()

    # ---- CPU oracle: one complete solve (t = the FP64 GPU iteration count) on this host
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
        Xo, _ = ob.bcg(A, [mu], b, Om, t_ref)
        t_cpu = time.perf_counter() - t0
        xo = Xo[0]
        rel_o = float(np.linalg.norm(b - (A @ xo + mu * xo)) / np.linalg.norm(b))
        err_mix = a_err(A, mu, xm, xo)
        err_64 = a_err(A, mu, x6, xo)
        cpu = {"value": 1.0 / t_cpu, "unit": "solves/s", "cores": int(threads or os.cpu_count() or 1),
               "kind": "oracle",
               "sample": f"one full solve of the d=8192 k=64 system by the FP64 oracle (t={t_ref} block products, "
                         f"relres {rel_o:.2e}), {t_cpu:.1f}s"}
        log(f"oracle: {t_cpu:.1f}s, err mixed {err_mix:.2e}, err fp64 {err_64:.2e}")

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
                     "kernel": "k_mv_tall<DT_F32, TN=5> (A X block product)",
                     "avg_launch_ms": avg_ms, "launches": prof["launches"]},
        "fp64_gpu": {"value": args.steps / t_64, "unit": "solves/s", "ms_per_step": 1e3 * t_64 / args.steps,
                     "iters": info_64["iters"], "relres": info_64["relres"], "rel_a_err_vs_oracle": err_64,
                     "matvec_avg_launch_ms": avg_ms64,
                     "matvec_tflops": flops64 / (avg_ms64 * 1e-3) / 1e12 if avg_ms64 > 0 else None},
        "mixed": {"iters_last_sweep": info_mix["iters"], "refine_sweeps": info_mix["refine_sweeps"],
                  "matrix_loads": info_mix["matrix_loads"], "relres": info_mix["relres"],
                  "rel_a_err_vs_oracle": err_mix},
        "speedup_mixed_vs_fp64": t_64 / t_mix,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
