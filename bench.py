"""Benchmark of the objective-and-gradient evaluation (Algorithm 2).

One step = one symtd_fg call: f, g_lambda and G_A for the large single
instance d=3, n=1000, r=100, p=100000 (Gaussian-mixture observations,
sigma=1e-2, nu=1/p), fp32 storage and fp32 matrix-core products with fp64
reductions and assembly.  Inputs are resident in device memory before the
timed region starts.

Prints one JSON line with the throughput (evals/s), the roofline figures of
the dominant kernel (timed with HIP events on the launch stream during the
timed region) and the CPU oracle timed on the host as a reported baseline.

    python bench.py [--steps K] [--warmup W] [--prec fp32|fp64] [--no-cpu-baseline]
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

import synth  # noqa: E402

WORKLOAD = dict(d=3, n=1000, r=100, p=100_000, sigma=1e-2)
# MI355X published dense matrix-core peaks (TFLOP/s) and HBM bandwidth (GB/s)
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
PEAK_HBM_GBS = 8000.0
# HBM bytes per evaluation (summed over the launches of one evaluation) of the
# two products, from rocprofv3 FETCH_SIZE (x 2.000) and WRITE_SIZE (x 1.000)
# counters, the factors being what the same counters read for a plain copy of
# known size.  They hold for the kernel sources whose hash is stored with them
# and are reported as null once those sources change.
TRAFFIC_SOURCES = ("paper_1911_03813_amd/csrc/fg_kernels.hip", "paper_1911_03813_amd/csrc/kernels.hpp",
                   "paper_1911_03813_amd/csrc/kcommon.hpp")
TRAFFIC_SHA = "857cbde6129424ac"
TRAFFIC_BYTES = {("fp32", "gemm1"): 492.3e6, ("fp32", "gemm2"): 474.4e6,
                 ("fp64", "gemm1"): 1796.9e6, ("fp64", "gemm2"): 1748.6e6}


def traffic_for(prec, kernel):
    return TRAFFIC_BYTES.get((prec, kernel)) if kernel_source_hash() == TRAFFIC_SHA else None


def kernel_source_hash():
    """Hash of the kernel sources' code (line comments and blank lines left out)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for s in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, s)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serial", action="store_true", help="model terms on the caller's stream")
    ap.add_argument("--g1-blocks", type=int, default=0)
    ap.add_argument("--g2-splits", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB elementwise copy a few times (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A copy kernel of known size: reads and writes 256 MiB per launch."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 3}))


def cpu_baseline(V64, nu, A64, lam, d, seconds):
    """The fp64 oracle on the host cores, repeated for about `seconds`."""
    from oracle.fg import fg_implicit
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 0)) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    fg_implicit(V64, nu, A64, lam, d, 0.0, with_intermediates=False)   # first touch
    t0 = time.perf_counter()
    k = 0
    while True:
        fg_implicit(V64, nu, A64, lam, d, 0.0, with_intermediates=False)
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} full fp64 evaluations of the same workload on the host ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the evaluation would shard over observations with one all-reduce of Y and w).",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch

    import paper_1911_03813_amd as S

    W = WORKLOAD
    d, n, r, p = W["d"], W["n"], W["r"], W["p"]
    dt = torch.float32 if args.prec == "fp32" else torch.float64
    V, nu, _ = synth.gmm(n, r, p, W["sigma"], 3)
    A = synth.gauss_factors(n, r, 3, 5)
    lam = np.ones(r)
    Vs = V.astype(np.float32).astype(np.float64) if args.prec == "fp32" else V
    As = A.astype(np.float32).astype(np.float64) if args.prec == "fp32" else A

    dev = torch.device("cuda:0")
    Vd = S.colmajor(torch.from_numpy(np.ascontiguousarray(Vs)).to(dt)).to(dev)
    Ad = S.colmajor(torch.from_numpy(np.ascontiguousarray(As)).to(dt)).to(dev)
    nud = torch.from_numpy(nu).to(dev)
    lamd = torch.from_numpy(lam).to(dev)
    ctx = S.Context(0)
    S.symtd_set_tuning(ctx, S.TUNE_SERIAL, int(args.serial))
    S.symtd_set_tuning(ctx, S.TUNE_G1_BLOCKS, args.g1_blocks)
    S.symtd_set_tuning(ctx, S.TUNE_G2_SPLITS, args.g2_splits)
    out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(r, dtype=torch.float64, device=dev),
           S.colmajor(torch.empty(n, r, dtype=dt, device=dev)))
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        S.symtd_fg(ctx, Vd, nud, Ad, lamd, d, 0.0, out=out)
    torch.cuda.synchronize()

    S.symtd_profile_reset(ctx)
    S.symtd_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.symtd_fg(ctx, Vd, nud, Ad, lamd, d, 0.0, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.symtd_profile_enable(ctx, False)
    per_kernel = {}
    for k, name in enumerate(S.profile_names()):
        ms, cnt = S.symtd_profile_read(ctx, k)
        if cnt:
            per_kernel[name] = {"avg_us": 1e3 * ms / cnt, "launches": cnt, "step_us": 1e3 * ms / args.steps}
    S.symtd_profile_reset(ctx)

    sec = (t1 - t0) / args.steps
    evals = 1.0 / sec
    flop_gemm = 2.0 * n * p * r                       # each of the two products
    flop_step = 2 * flop_gemm + 4.0 * n * r * r       # plus B = A'A and A D_lambda C
    peak = PEAK_TFLOPS[args.prec]
    # the dominant product; with r > 16 * (subtiles per launch) it runs as
    # several column-group launches, so its algorithmic flops per step are
    # divided by its summed launch time per step
    dom = max(("gemm1", "gemm2"), key=lambda k: per_kernel.get(k, {"step_us": 0})["step_us"])
    dom_us = per_kernel[dom]["step_us"]
    achieved = flop_gemm / (dom_us * 1e-6) / 1e12
    traffic = traffic_for(args.prec, dom)

    res = {
        "metric": "f+grad f evals/s (n=1000, p=1e5, r=100, d=3)",
        "value": evals,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "large single instance: Gaussian mixture d=3 n=1000 r=100 p=100000 sigma=1e-2",
                   "d": d, "n": n, "r": r, "p": p, "precision": args.prec, "storage": args.prec},
        "step_mfma_frac": flop_step * evals / (peak * 1e12),
        "roofline": {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "launches_per_step": per_kernel[dom]["launches"] / args.steps},
        "kernels_us_per_step": {k: round(v["step_us"], 2) for k, v in per_kernel.items()},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(Vs, nu, As, lam, d, args.cpu_seconds)
    ctx.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
