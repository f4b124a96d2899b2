"""Benchmark of the objective-and-gradient evaluation (Algorithm 2), with the
small and mid-size workloads, the batched and served solve forms beside it.

Headline: one step = one symtd_fg call, f, g_lambda and G_A for the large
single instance d=3, n=1000, r=100, p=100000 (Gaussian-mixture observations,
sigma=1e-2, nu=1/p), in the paper's arithmetic: fp64 storage, fp64
matrix-core products, fp64 reductions and assembly (--prec selects fp32 or
the 16-bit products instead).  Inputs are resident in device memory before
the timed region starts.  The JSON line carries the throughput (evals/s),
per-call duration quantiles, the rate of the same evaluation replayed from a
captured graph, the roofline figures of the dominant kernel (timed with HIP
events on its launch stream during the timed region) and the CPU oracle
timed on the host.

Legs of the default run:
"precisions": the same evaluation in fp64, fp32, fp16 and bf16x3 products.
"normx": ||X||^2 of the large data set.
"small": d=3, n=10, r=3, p=750, fp64: one evaluation and 200 L-BFGS
iterations from a Gaussian start.
"mid": d=4, n=100, r=20, p=5000, fp64 and fp32: evaluation throughput, and a
full solve (10 randomized-range-finder restarts) for each sigma in {1e-4,
1e-3, 1e-2, 1e-1} with its relative error and similarity score.
"table1": Section 4.1's explicit (stored n^d tensor, Algorithm 1) against
implicit (Algorithm 2) evaluation at Table 1's scenarios, fp64.
"stochastic": Section 5's comparison at d=3, n=500, r=10, p=500,000,
sigma=0.1: L-BFGS on the full data against Adam on s in {10, 100, 1000}
sampled columns per step, from the same ten starts.
"corrected": moments corrected for spherical Gaussian noise (n=50, r=5,
p=100,000, sigma=0.3, d in {3, 4}, fp64): plain against corrected solves,
with the similarity score and the distance from the noiseless moment.
"batched": 512 problems, n ~ U{16..256}, r ~ U{2..32}, p = 250 r, d in
{3, 4}, sigma in {1e-3, 1e-2}, 4 randomized-range-finder restarts each, fp32,
solved together by symtd_solve_batched, against the plain loop of
symtd_solve calls on the same problems, with per-problem error differences.
"served": Poisson arrivals (200 requests/s) of problems drawn the same way to
a symtd_server; p50/p99 latency (arrival to result) and solves/s, against
the plain first-in-first-out loop of symtd_solve calls replaying the same
arrival trace.

    python bench.py [--steps K] [--warmup W] [--prec fp64|fp32|fp16|bf16x3]
                    [--no-cpu-baseline] [--only-fg] [--legs a,b,...] [--batched N]
                    [--batched-max-evals K] [--no-batched-loop] [--served N] [--study]
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
SMALL = dict(d=3, n=10, r=3, p=750, sigma=1e-2)
MID = dict(d=4, n=100, r=20, p=5000)
# MI355X published dense matrix-core peaks (TFLOP/s) and HBM bandwidth (GB/s)
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "fp16": 2500.0}
PEAK_HBM_GBS = 8000.0
# HBM bytes per evaluation (summed over the launches of one evaluation) of the
# two products, from rocprofv3 FETCH_SIZE (x 2.000) and WRITE_SIZE (x 1.000)
# counters, the factors being what the same counters read for a plain copy of
# known size.  They hold for the kernel sources whose hash is stored with them
# and are reported as null once those sources change.
TRAFFIC_SOURCES = ("paper_1911_03813_amd/csrc/fg_kernels.hip", "paper_1911_03813_amd/csrc/kernels.hpp",
                   "paper_1911_03813_amd/csrc/kcommon.hpp", "paper_1911_03813_amd/csrc/lp_kernels.hip",
                   "paper_1911_03813_amd/csrc/lp.hpp")
TRAFFIC_SHA = "72b7bcb35ce945af"
TRAFFIC_BYTES = {("fp32", "gemm1"): 506.8e6, ("fp32", "gemm2"): 468.0e6,
                 ("fp64", "gemm1"): 1092.8e6, ("fp64", "gemm2"): 932.6e6,
                 ("fp16", "gemm1"): 273.5e6, ("fp16", "gemm2"): 242.3e6,
                 ("bf16x3", "gemm1"): 509.0e6, ("bf16x3", "gemm2"): 469.7e6}


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
    ap.add_argument("--prec", choices=["fp32", "fp64", "fp16", "bf16x3"], default="fp64")
    ap.add_argument("--pgtol", type=float, default=1e-6,
                    help="gradient tolerance (of f / alpha) of the batched, served and mid-size solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stoch", action="store_true", help="skip the stochastic (Adam) comparison leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--g1-blocks", type=int, default=0)
    ap.add_argument("--g2-splits", type=int, default=0)
    ap.add_argument("--only-fg", action="store_true", help="headline only (no batched/served legs)")
    ap.add_argument("--batched", type=int, default=512, help="problems of the batched leg")
    ap.add_argument("--batched-max-evals", type=int, default=0,
                    help="cap every batched problem's evaluations (0 = the solver's default); with a small cap "
                         "every problem stays in the batch, so a profile sees full steps only")
    ap.add_argument("--no-batched-loop", action="store_true", help="skip the plain loop beside the batched leg")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs after the headline (precisions, normx, small, mid, table1, "
                         "stochastic, corrected, batched, served) or all")
    ap.add_argument("--served", type=int, default=600, help="requests of the served leg")
    ap.add_argument("--rate", type=float, default=200.0, help="arrival rate of the served leg (requests/s)")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_1911_03813_amd", "tuning", "mi355x.json"),
                    help="tuning table (JSON cache written by paper_1911_03813_amd.autotune) to load first")
    ap.add_argument("--no-tuning", action="store_true", help="run with the built-in launch shapes")
    ap.add_argument("--study", action="store_true",
                    help="only run the Section 4.2 studies (mean recovery over ranks, RRF against random starts)")
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
    """The fp64 oracle on the host cores, repeated for about `seconds`, and
    on one thread for about a third of that."""
    from oracle.fg import fg_implicit
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([int(i.get("num_threads", 0)) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()

    def rate(budget):
        fg_implicit(V64, nu, A64, lam, d, 0.0, with_intermediates=False)   # first touch
        t0 = time.perf_counter()
        k = 0
        while True:
            fg_implicit(V64, nu, A64, lam, d, 0.0, with_intermediates=False)
            k += 1
            if time.perf_counter() - t0 >= budget:
                break
        return k, time.perf_counter() - t0

    k, dt = rate(seconds)
    out = {"value": k / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "sample": f"{k} full fp64 evaluations of the same workload on the host ({dt:.1f} s)"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            k1, dt1 = rate(seconds / 3)
        out["one_thread"] = {"value": k1 / dt1, "unit": "evals/s", "cores": 1,
                             "sample": f"{k1} evaluations on one thread ({dt1:.1f} s)"}
    try:
        import subprocess
        model = [ln.split(":", 1)[1].strip() for ln in subprocess.run(["lscpu"], capture_output=True, text=True)
                 .stdout.splitlines() if ln.startswith("Model name")]
        if model:
            out["cpu_model"] = model[0]
    except Exception:
        pass
    return out


def grouped_problems(count, key, pgtol, restarts=4, max_evals=0):
    """Problems of the grouped workload (device tensors) and their sigmas
    (max_evals > 0 caps every problem's evaluations)."""
    import torch

    import paper_1911_03813_amd as S
    shapes = synth.batch_shapes(count, key)
    probs = []
    for i, s in enumerate(shapes):
        V, nu, _ = synth.gmm(s["n"], s["r"], s["p"], s["sigma"], key, i)
        probs.append(dict(V=S.colmajor(torch.from_numpy(V).float()).cuda(), nu=torch.from_numpy(nu).cuda(),
                          d=s["d"], r=s["r"], restarts=restarts, seed=1000 + i, pgtol=pgtol))
        if max_evals > 0:
            probs[-1]["max_evals"] = max_evals
    return probs, np.array([s["sigma"] for s in shapes])


def rel_err_summary(rel, sigma=None):
    """Final relative errors of a set of solves.  Their distribution is
    bimodal on this workload (a solve either reaches the noise floor of its
    sigma or stops in a local minimum near 0.2), so the median alone moves
    with a few problems: quantiles, the fraction below 1e-2 and the fraction
    reaching 1e-4 (per sigma: the floor of sigma = 1e-2 lies above 1e-4)
    go with it."""
    rel = np.asarray(rel, dtype=np.float64)
    out = {"median": float(np.median(rel)),
           "q10_q50_q90": [float(x) for x in np.quantile(rel, [0.1, 0.5, 0.9])],
           "frac_below_1e-2": float(np.mean(rel < 1e-2)),
           "frac_at_most_1e-4": float(np.mean(rel <= 1e-4))}
    if sigma is not None:
        out["frac_at_most_1e-4_by_sigma"] = {f"{sg:g}": float(np.mean(rel[sigma == sg] <= 1e-4))
                                             for sg in sorted(set(sigma.tolist()))}
    return out


def delta_summary(a, b):
    """Per-problem |rel_err_a - rel_err_b| of the same problems solved two ways."""
    dlt = np.abs(np.asarray(a) - np.asarray(b))
    return {"q50_q90_q99_max": [float(x) for x in np.quantile(dlt, [0.5, 0.9, 0.99, 1.0])],
            "frac_within_1e-4": float(np.mean(dlt <= 1e-4))}


def exit_histogram(S, results):
    names = [S.EXIT_NAMES.get(int(r["exit_reason"]), str(r["exit_reason"])) for r in results]
    return {k: names.count(k) for k in sorted(set(names))}


def loop_solve(S, ctx, pr):
    kw = {k: v for k, v in pr.items() if k not in ("V", "nu", "d", "r")}
    return S.symtd_solve(ctx, pr["V"], pr["nu"], pr["d"], pr["r"], **kw)


def normx_leg(S, ctx, Vs, nu, d, reps=3):
    """||X||^2 of the large data set (fp32 storage, fp64 products): time per
    call and the rate of its algorithmic flop, n p (p + 1) (the p x p Gram
    matrix's upper triangle with the diagonal, 2 flop per multiply-add)."""
    import torch
    n, p = Vs.shape
    Vd = S.colmajor(torch.from_numpy(np.ascontiguousarray(Vs)).to(torch.float32)).cuda()
    nud = torch.from_numpy(nu).cuda()
    a = S.symtd_normX(ctx, Vd, nud, d)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        S.symtd_normX(ctx, Vd, nud, d, out=a)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    flop = float(n) * p * (p + 1)
    peak = PEAK_TFLOPS["fp64"]
    out = {"workload": f"d={d} n={n} p={p}, fp32 storage, fp64 matrix products", "calls": reps,
           "ms_per_call": t * 1e3, "tflops": flop / t / 1e12, "peak_tflops": peak,
           "frac": flop / t / 1e12 / peak, "value": float(a.cpu()[0])}
    # the oracle's value of the same data set, stored by tests/golden/make_normx_full.py
    gold = os.path.join(ROOT, "tests", "golden", "normx_gmm_n1000_p1e5_d3.json")
    if os.path.exists(gold):
        with open(gold) as fh:
            g = json.load(fh)
        if (g["workload"]["n"], g["workload"]["p"], g["workload"]["d"]) == (n, p, d):
            out["oracle_value"] = g["value"]
            out["error_vs_oracle_rel_scale"] = abs(out["value"] - g["value"]) / g["scale_abs"]
    return out


def precision_leg(S, ctx, Vs, nu, As, lam, d, steps, warmup):
    """evals/s, product times and error against the fp64 products of every
    product precision on the large workload (fp32 storage for fp32 / fp16 /
    bf16x3; the fp64 products evaluate the same stored values widened)."""
    import torch
    n, p = Vs.shape
    r = As.shape[1]
    flop_gemm = 2.0 * n * p * r
    out = {}
    ref = None
    for name, prec, dt in (("fp64", S.PREC_FP64, torch.float64), ("fp32", S.PREC_FP32, torch.float32),
                           ("fp16", S.PREC_FP16, torch.float32), ("bf16x3", S.PREC_BF16X3, torch.float32)):
        Vd = S.colmajor(torch.from_numpy(np.ascontiguousarray(Vs)).to(dt)).cuda()
        Ad = S.colmajor(torch.from_numpy(np.ascontiguousarray(As)).to(dt)).cuda()
        nud = torch.from_numpy(nu).cuda()
        lamd = torch.from_numpy(lam).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        data = S.Data(ctx, Vd, nud, prec)
        torch.cuda.synchronize()
        conv = time.perf_counter() - t0
        res = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty(r, dtype=torch.float64, device="cuda"),
               S.colmajor(torch.empty(n, r, dtype=dt, device="cuda")))
        S.symtd_profile_enable(ctx, True, kernels=("gemm1", "gemm2"))
        for _ in range(warmup):
            data.fg(Ad, lamd, d, 0.0, out=res)
        torch.cuda.synchronize()
        S.symtd_profile_reset(ctx)
        k = steps if name != "fp64" else max(10, steps // 4)
        t0 = time.perf_counter()
        for _ in range(k):
            data.fg(Ad, lamd, d, 0.0, out=res)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / k
        S.symtd_profile_enable(ctx, False)
        kus = {}
        for i, kn in enumerate(S.profile_names()):
            ms, cnt = S.symtd_profile_read(ctx, i)
            if cnt:
                kus[kn] = 1e3 * ms / k
        S.symtd_profile_reset(ctx)
        fv = float(res[0].cpu()[0])
        gv = res[1].cpu().numpy()
        Gv = res[2].cpu().numpy().astype(np.float64)
        if ref is None:
            ref = (fv, gv, Gv)
        g1 = kus.get("gemm1", float("nan"))
        entry = {"evals_per_s": 1.0 / sec, "ms_per_eval": 1e3 * sec,
                 "kernels_us_per_eval": {kk: round(v, 2) for kk, v in kus.items()}}
        if name != "fp64":
            # norm-wise relative errors against the fp64 products on the same stored inputs
            entry["error_vs_fp64"] = {"f": abs(fv - ref[0]) / abs(ref[0]),
                                      "g_lambda": float(np.max(np.abs(gv - ref[1])) / np.max(np.abs(ref[1]))),
                                      "G_A": float(np.linalg.norm(Gv - ref[2]) / np.linalg.norm(ref[2])),
                                      "stated_bound": S.prec_bound(prec, d)}
        if name in ("fp64", "fp32"):
            entry["gemm1_mfma_frac"] = flop_gemm / (g1 * 1e-6) / (PEAK_TFLOPS[name] * 1e12)
        else:
            mult = 3.0 if name == "bf16x3" else 1.0
            vbytes = n * p * (4 if name == "bf16x3" else 2)
            entry["conversion_s"] = conv
            entry["gemm1_mfma_frac"] = mult * flop_gemm / (g1 * 1e-6) / (PEAK_TFLOPS["fp16"] * 1e12)
            entry["gemm1_hbm_GBs"] = vbytes / (g1 * 1e-6) / 1e9
            entry["gemm1_hbm_frac"] = vbytes / (g1 * 1e-6) / (PEAK_HBM_GBS * 1e9)
            entry["mfma_flop_per_product"] = "3 x 2npr (hi hi, hi lo, lo hi)" if name == "bf16x3" else "2npr"
        data.close()
        del Vd, Ad, res
        out[name] = entry
    return out


def small_leg(S, ctx):
    """d=3, n=10, r=3, p=750 (sigma 1e-2), fp64: one evaluation at a
    Gaussian start (normalised columns, lambda = 1), then 200 L-BFGS
    iterations from it, timed (no other stopping test)."""
    import torch
    W = SMALL
    V, nu, means = synth.gmm(W["n"], W["r"], W["p"], W["sigma"], 11)
    A0 = synth.gauss_factors(W["n"], W["r"], 11, 5)
    Vd = S.colmajor(torch.from_numpy(V)).cuda()
    nud = torch.from_numpy(nu).cuda()
    A0d = S.colmajor(torch.from_numpy(A0)).cuda()
    lam = torch.ones(W["r"], dtype=torch.float64, device="cuda")
    out = S.symtd_fg(ctx, Vd, nud, A0d, lam, W["d"], 0.0)
    kw = dict(prec=S.PREC_FP64, pgtol=0.0, ftol=0.0, max_iters=200, restarts=1, init=S.INIT_GAUSS, A0=A0d)
    S.symtd_solve(ctx, Vd, nud, W["d"], W["r"], **kw)          # warm
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        S.symtd_fg(ctx, Vd, nud, A0d, lam, W["d"], 0.0, out=out)
    torch.cuda.synchronize()
    fg_s = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    res = S.symtd_solve(ctx, Vd, nud, W["d"], W["r"], **kw)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    return {"workload": "d=3 n=10 r=3 p=750 sigma=1e-2, fp64, Gaussian start, 200 L-BFGS iterations",
            "fg_us": 1e6 * fg_s, "solve_ms": 1e3 * solve_s, "iters": int(res["iters"]), "evals": int(res["evals"]),
            "exit": S.EXIT_NAMES.get(int(res["exit_reason"])), "rel_err": float(res["rel_err"]),
            "score": S.metrics.similarity_score(means, res["A"].cpu().double().numpy())}


def mid_leg(S, ctx, pgtol, steps=100):
    """d=4, n=100, r=20, p=5000: evaluation throughput in fp64 and fp32, and
    a solve with 10 randomized-range-finder restarts for each sigma, with its
    relative error (fp64 evaluation at the final point) and the similarity
    score of the recovered factors against the true means."""
    import torch
    W = MID
    out = {"workload": "d=4 n=100 r=20 p=5000, Gaussian mixture, 10 RRF restarts", "fg": {}, "solves": []}
    for name, prec, dt in (("fp64", S.PREC_FP64, torch.float64), ("fp32", S.PREC_FP32, torch.float32)):
        V, nu, _ = synth.gmm(W["n"], W["r"], W["p"], 1e-2, 12)
        A = synth.gauss_factors(W["n"], W["r"], 12, 5)
        Vd = S.colmajor(torch.from_numpy(V).to(dt)).cuda()
        Ad = S.colmajor(torch.from_numpy(A).to(dt)).cuda()
        nud = torch.from_numpy(nu).cuda()
        lam = torch.ones(W["r"], dtype=torch.float64, device="cuda")
        res = S.symtd_fg(ctx, Vd, nud, Ad, lam, W["d"], 0.0)
        for _ in range(10):
            S.symtd_fg(ctx, Vd, nud, Ad, lam, W["d"], 0.0, out=res)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            S.symtd_fg(ctx, Vd, nud, Ad, lam, W["d"], 0.0, out=res)
        torch.cuda.synchronize()
        out["fg"][name] = {"evals_per_s": steps / (time.perf_counter() - t0)}
    for k, sigma in enumerate((1e-4, 1e-3, 1e-2, 1e-1)):
        V, nu, means = synth.gmm(W["n"], W["r"], W["p"], sigma, 13, k)
        for name, prec, dt in (("fp64", S.PREC_FP64, torch.float64), ("fp32", S.PREC_FP32, torch.float32)):
            Vd = S.colmajor(torch.from_numpy(V).to(dt)).cuda()
            nud = torch.from_numpy(nu).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = S.symtd_solve(ctx, Vd, nud, W["d"], W["r"], prec=prec, restarts=10, seed=50 + k, pgtol=pgtol)
            torch.cuda.synchronize()
            out["solves"].append({"sigma": sigma, "precision": name, "seconds": time.perf_counter() - t0,
                                  "rel_err": float(res["rel_err"]), "iters": int(res["iters"]),
                                  "evals": int(res["evals"]), "exit": S.EXIT_NAMES.get(int(res["exit_reason"])),
                                  "score": S.metrics.similarity_score(means, res["A"].cpu().double().numpy())})
    return out


def stoch_leg(S, ctx, pgtol):
    """The comparison of Section 5 (Table stoch): d=3, n=500, r=10,
    p=500,000, sigma=0.1, fp32.  The standard method (L-BFGS on the full
    data) and Adam on s sampled columns per step (s in {10, 100, 1000},
    the paper's schedule), each from the same 10 randomized-range-finder
    starts, all restarts of a method run together; the shifted objective
    (alpha = 0) of the best restart, its similarity score and the wall time
    of all ten runs."""
    import torch
    n, r, p, d = 500, 10, 500_000, 3
    V, nu, means = synth.gmm(n, r, p, 0.1, 14, congruent=True)   # the paper's means: pairwise cosine 0.5
    Vd = S.colmajor(torch.from_numpy(V).float()).cuda()
    nud = torch.from_numpy(nu).cuda()
    del V
    out = {"workload": "d=3 n=500 r=10 p=500000 sigma=0.1, congruent means, fp32, 10 RRF starts shared by all "
                       "methods, shifted f",
           "methods": []}

    def row(name, sec, res, extra):
        out["methods"].append({"method": name, "seconds": sec, "best_f_shifted": float(res["f"]),
                               "score": S.metrics.similarity_score(means, res["A"].cpu().double().numpy()), **extra})

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = S.symtd_solve(ctx, Vd, nud, d, r, restarts=10, seed=41, pgtol=pgtol, alpha=0.0)
    torch.cuda.synchronize()
    row("standard (L-BFGS, full data)", time.perf_counter() - t0, res, {"iters": int(res["iters"]),
                                                                      "evals": int(res["evals"])})
    for s in (10, 100, 1000):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = S.symtd_solve_adam(ctx, Vd, nud, d, r, samples=s, restarts=10, seed=41)
        torch.cuda.synchronize()
        row(f"Adam, s={s}", time.perf_counter() - t0, res, {"epochs": int(res["epochs"]),
                                                            "steps": int(res["iters"])})
    del Vd
    return out


def corrected_leg(S, ctx, pgtol):
    """Moments corrected for spherical Gaussian noise of known level: a
    Gaussian mixture (n=50, r=5, p=100,000, sigma=0.3, congruent means) at
    d = 3 and 4, solved with 5 RRF restarts in fp64 on the plain objective
    and on the corrected one.  For each: wall time, the similarity score
    against the true means, and the relative distance of the model from the
    noiseless moment C = sum_j w_j mu_j^{(x)d}, from the Kruskal identity
    <sum_j l_j a_j^d, sum_k w_k u_k^d> = l' [A'U]^d w (no tensor formed)."""
    import torch
    n, r, p, sigma = 50, 5, 100_000, 0.3
    out = {"workload": f"Gaussian mixture n={n} r={r} p={p} sigma={sigma}, congruent means, fp64, 5 RRF restarts",
           "rows": []}
    for d in (3, 4):
        V, nu, means = synth.gmm(n, r, p, sigma, 18, d, congruent=True)
        w = np.bincount((np.arange(p) * r) // p, minlength=r) / p
        Vd = S.colmajor(torch.from_numpy(V)).cuda()
        nud = torch.from_numpy(nu).cuda()

        def dist(lam, A):
            kr = lambda l1, A1, l2, A2: float(l1 @ (A1.T @ A2) ** d @ l2)
            mm, mc, cc = kr(lam, A, lam, A), kr(lam, A, w, means), kr(w, means, w, means)
            return float(np.sqrt(max(mm - 2 * mc + cc, 0.0) / cc))

        row = {"d": d}
        for name, sg in (("plain", 0.0), ("corrected", sigma)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = S.symtd_solve(ctx, Vd, nud, d, r, restarts=5, seed=51, pgtol=pgtol, sigma=sg)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            A = res["A"].cpu().numpy()
            lam = res["lam"].cpu().numpy()
            row[name] = {"seconds": sec, "evals": int(res["evals"]), "exit": S.EXIT_NAMES[int(res["exit_reason"])],
                         "score": S.metrics.similarity_score(means, A), "dist_to_clean_moment": dist(lam, A)}
        out["rows"].append(row)
        del Vd
    return out


# Table 1's scenarios (d, n, p, r) and the paper's seconds per iteration
# (explicit, implicit), MATLAB on the CPU it names: context only
TABLE1 = [(3, 75, 750, 5, 5.30e-04, 4.36e-04), (3, 75, 750, 25, 1.91e-03, 5.91e-04),
          (3, 75, 3750, 5, 5.17e-04, 7.96e-04), (3, 75, 3750, 25, 1.90e-03, 1.03e-03),
          (3, 375, 3750, 5, 2.29e-02, 4.82e-03), (4, 75, 3750, 5, 1.47e-02, 9.22e-04)]


def table1_leg(S, ctx, reps=50):
    """Section 4.1: the explicit route (Algorithm 1 on the stored n^d
    tensor) against the implicit one (Algorithm 2) per evaluation, fp64,
    V ~ U(0,1), at Table 1's scenarios.  The tensor's formation is timed
    apart (the paper leaves it out of the comparison)."""
    import torch
    rows = []
    for k, (d, n, p, r, pe, pi) in enumerate(TABLE1):
        V, nu = synth.uniform_obs(n, p, 15, k)
        A = synth.gauss_factors(n, r, 15, k, 5)
        Vd = S.colmajor(torch.from_numpy(V)).cuda()
        Ad = S.colmajor(torch.from_numpy(A)).cuda()
        nud = torch.from_numpy(nu).cuda()
        lam = torch.ones(r, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = S.symtd_form_moment(ctx, Vd, nud, d)
        torch.cuda.synchronize()
        t_form = time.perf_counter() - t0

        def rate(fn):
            out = fn(None)
            for _ in range(5):
                fn(out)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                fn(out)
            torch.cuda.synchronize()
            return (time.perf_counter() - t1) / reps

        t_exp = rate(lambda o: S.symtd_fg_explicit(ctx, X, n, d, Ad, lam, 0.0, out=o))
        t_imp = rate(lambda o: S.symtd_fg(ctx, Vd, nud, Ad, lam, d, 0.0, out=o))
        rows.append({"d": d, "n": n, "p": p, "r": r, "explicit_us": 1e6 * t_exp, "implicit_us": 1e6 * t_imp,
                     "speedup_implicit": t_exp / t_imp, "form_ms": 1e3 * t_form,
                     "explicit_tensor_MB": 8 * n ** d / 1e6,
                     "paper_s_per_iter": {"explicit": pe, "implicit": pi}})
        del X
    return {"workload": "Table 1 scenarios, V ~ U(0,1), fp64, per evaluation (f, g_lambda, G_A)", "rows": rows}


def gmm_study(S, ctx):
    """Section 4.2's mean-recovery sweep: n=500, d in {3, 4}, r in {3, 5, 10}
    components with congruent means (pairwise cosine 0.5), sigma in {1e-4,
    1e-3, 1e-2, 1e-1}, p = 250 r, fitted with every rank r^ in r-2 .. r+2,
    best of 10 RRF restarts (pgtol 1e-4, of f / alpha), fp64.  Relative
    error of the best restart and its similarity score (eq. (Score)); every
    (d, r) group is one batched solve, timed."""
    import torch
    out = {"workload": "n=500, d in {3,4}, r in {3,5,10}, r^ in r-2..r+2, sigma in {1e-4..1e-1}, p=250r, "
                       "congruent means, 10 RRF restarts, pgtol 1e-4, fp64", "groups": []}
    for d in (3, 4):
        for r in (3, 5, 10):
            probs, meta = [], []
            for k, sigma in enumerate((1e-4, 1e-3, 1e-2, 1e-1)):
                V, nu, means = synth.gmm(500, r, 250 * r, sigma, 16, d, r, k, congruent=True)
                Vd = S.colmajor(torch.from_numpy(V)).cuda()
                nud = torch.from_numpy(nu).cuda()
                for rh in range(max(1, r - 2), r + 3):
                    probs.append(dict(V=Vd, nu=nud, d=d, r=rh, restarts=10, seed=100 * k + rh, pgtol=1e-4))
                    meta.append((sigma, rh, means))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = S.symtd_solve_batched(ctx, probs)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            rows = [{"sigma": sg, "r_hat": rh, "rel_err": float(q["rel_err"]),
                     "score": S.metrics.similarity_score(mu, q["A"].cpu().numpy())}
                    for (sg, rh, mu), q in zip(meta, res)]
            out["groups"].append({"d": d, "r": r, "seconds": sec, "solves": len(probs), "rows": rows})
    return out


def init_study(S, ctx, runs=100):
    """Section 4.2's comparison of starts: d=3, n=500, r = r^ = 3, p=750,
    congruent means, fp64, for each sigma 100 runs from RRF starts (pgtol
    1e-4) and from N(0,1) starts (pgtol 1e-4 and 1e-6).  A run succeeds if
    its final f / alpha is within 0.01 of the best over all 300 runs of that
    sigma; time of each method's 4 x 100 runs (one batched solve)."""
    import torch
    d, n, r, p = 3, 500, 3, 750
    sigmas = (1e-4, 1e-3, 1e-2, 1e-1)
    data = []
    for k, sigma in enumerate(sigmas):
        V, nu, _ = synth.gmm(n, r, p, sigma, 17, k, congruent=True)
        data.append((S.colmajor(torch.from_numpy(V)).cuda(), torch.from_numpy(nu).cuda()))
    methods = [("RRF, pgtol 1e-4", S.INIT_RRF, 1e-4), ("random, pgtol 1e-4", S.INIT_GAUSS, 1e-4),
               ("random, pgtol 1e-6", S.INIT_GAUSS, 1e-6)]
    finals = {}
    times = {}
    for mi, (name, init, pg) in enumerate(methods):
        probs = [dict(V=Vd, nu=nud, d=d, r=r, restarts=runs, seed=1000 * mi + k, pgtol=pg, init=init)
                 for k, (Vd, nud) in enumerate(data)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = S.symtd_solve_batched(ctx, probs)
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0
        finals[name] = [np.asarray(q["f_restarts"]) / q["alpha"] for q in res]
    rows = []
    for k, sigma in enumerate(sigmas):
        best = min(float(np.min(finals[name][k])) for name, _, _ in methods)
        rows.append({"sigma": sigma, "best_f_over_alpha": best,
                     "successes": {name: int(np.sum(finals[name][k] <= best + 0.01)) for name, _, _ in methods}})
    return {"workload": f"d=3 n=500 r=r^=3 p=750, congruent means, fp64, {runs} runs per start kind and sigma",
            "seconds": times, "rows": rows}


def batched_leg(S, ctx, count, pgtol, max_evals=0, loop=True):
    import torch
    probs, sigma = grouped_problems(count, 4, pgtol, max_evals=max_evals)
    S.symtd_solve_batched(ctx, probs[:4])              # warm the path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = S.symtd_solve_batched(ctx, probs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    rb = np.array([r["rel_err"] for r in res])
    out = {"workload": f"{count} problems n~U{{16..256}} r~U{{2..32}} p=250r d in {{3,4}} sigma in {{1e-3,1e-2}}, "
                       f"4 restarts, fp32, pgtol {pgtol:g}" + (f", at most {max_evals} evaluations" if max_evals else ""),
           "solves_per_s": count / tb, "restart_solves_per_s": 4 * count / tb,
           "seconds": tb, "steps": int(res[0]["steps"]),
           "rel_err": rel_err_summary(rb, sigma), "exit": exit_histogram(S, res),
           "evals_median": float(np.median([r["evals"] for r in res])),
           # a problem leaves the batch at the step its last restart stops:
           # every live restart takes one evaluation per step
           "finish_step_q50_q90_q99_max": [float(x) for x in np.quantile(
               [max(r["evals_restarts"]) for r in res], [0.5, 0.9, 0.99, 1.0])]}
    if loop:
        # the plain loop of symtd_solve calls on every problem of the batch
        t0 = time.perf_counter()
        lo = [loop_solve(S, ctx, pr) for pr in probs]
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        rl = np.array([r["rel_err"] for r in lo])
        out.update({"loop": {"problems": count, "solves_per_s": count / tl, "seconds": tl},
                    "speedup_vs_loop": tl / tb, "rel_err_loop": rel_err_summary(rl, sigma),
                    "rel_err_abs_diff_vs_loop": delta_summary(rb, rl), "exit_loop": exit_histogram(S, lo)})
    return out


def served_leg(S, ctx, count, rate, pgtol):
    import torch
    probs, sigma = grouped_problems(count, 5, pgtol)
    arrivals = synth.poisson_arrivals(rate, count, 5)
    warm = count // 10
    srv = S.Server(0, torch.float32, memory_bytes=16 << 30)
    try:
        sub = {}
        got = {}
        t_start = time.perf_counter()
        for i, pr in enumerate(probs):
            while True:
                now = time.perf_counter() - t_start
                if now >= arrivals[i]:
                    break
                for res in srv.poll(64, timeout_ms=0):
                    got[res["id"]] = res
                time.sleep(min(0.0005, arrivals[i] - now))
            sub[srv.submit(**pr)] = i
        while len(got) < count:
            for res in srv.poll(256, timeout_ms=100):
                got[res["id"]] = res
        stats = srv.stats()
    finally:
        srv.close()
    order = sorted(sub, key=sub.get)
    # latency from the arrival of a request (its submit) to its result, on the server clock
    lat = np.array([got[k]["t_done"] - got[k]["t_submit"] for k in order])
    done_t = np.array([got[k]["t_done"] for k in order])
    sub_t = np.array([got[k]["t_submit"] for k in order])
    admit_t = np.array([got[k]["t_admit"] for k in order])
    meas = slice(warm, count)
    span = done_t[meas].max() - sub_t[meas].min()
    rel = np.array([got[k]["rel_err"] for k in order])
    # requests on the device at once, from the admission and completion times
    ev = sorted([(t, 1) for t in admit_t] + [(t, -1) for t in done_t], key=lambda e: (e[0], e[1]))
    cur = peak = 0
    for _, k in ev:
        cur += k
        peak = max(peak, cur)
    # the plain loop: each request solved alone in arrival order (FIFO), service times measured
    service = []
    for pr in probs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = loop_solve(S, ctx, pr)
        torch.cuda.synchronize()
        service.append((time.perf_counter() - t0, r["rel_err"]))
    free_at = 0.0
    lat_loop = []
    for a, (sv, _) in zip(arrivals, service):
        start = max(a, free_at)
        free_at = start + sv
        lat_loop.append(free_at - a)
    lat_loop = np.array(lat_loop)
    rel_loop = np.array([s[1] for s in service])
    span_loop = free_at - arrivals[warm]
    return {"workload": f"{count} requests, Poisson {rate:g}/s, problems as the batched leg, 4 restarts, fp32, "
                        f"pgtol {pgtol:g} (first {warm} excluded)",
            "p50_ms": 1e3 * float(np.percentile(lat[meas], 50)), "p99_ms": 1e3 * float(np.percentile(lat[meas], 99)),
            "solves_per_s": (count - warm) / span, "peak_requests_on_device": peak,
            "loop": {"p50_ms": 1e3 * float(np.percentile(lat_loop[meas], 50)),
                     "p99_ms": 1e3 * float(np.percentile(lat_loop[meas], 99)),
                     "solves_per_s": (count - warm) / span_loop,
                     "mean_service_ms": 1e3 * float(np.mean([s[0] for s in service]))},
            "rel_err": rel_err_summary(rel[meas], sigma[meas]), "rel_err_loop": rel_err_summary(rel_loop[meas],
                                                                                              sigma[meas]),
            "rel_err_abs_diff_vs_loop": delta_summary(rel[meas], rel_loop[meas]),
            "steps": int(stats["steps"])}


def call_stats(evaluate, calls):
    """Durations of single evaluations, each bracketed by events on the
    stream the library launches on (the current stream)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for a, b in ev:
        a.record()
        evaluate()
        b.record()
    torch.cuda.synchronize()
    us = np.array([1e3 * a.elapsed_time(b) for a, b in ev])
    return {"calls": calls, "p10_us": float(np.percentile(us, 10)), "median_us": float(np.median(us)),
            "p90_us": float(np.percentile(us, 90))}


def graph_rate(evaluate, out, steps):
    """The evaluation captured once as a graph and replayed: evals/s, and
    whether every replay gives the eager bits."""
    import torch
    evaluate()
    torch.cuda.synchronize()
    ref = [x.clone() for x in out]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        evaluate()                               # warm on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        evaluate()
    g.replay()
    torch.cuda.synchronize()
    same = all(torch.equal(x, y) for x, y in zip(out, ref))
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    same = same and all(torch.equal(x, y) for x, y in zip(out, ref))
    del g
    return {"evals_per_s": 1.0 / sec, "ms_per_eval": 1e3 * sec, "replays": steps, "replays_equal_eager": same}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the evaluation would shard over observations with one all-reduce of Y and w).",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.study:
        import torch  # noqa: F401  (the GPU runtime comes up before the library's)

        import paper_1911_03813_amd as S
        ctx = S.Context(0)
        print(json.dumps({"gmm": gmm_study(S, ctx), "init": init_study(S, ctx)}))
        ctx.close()
        return

    import torch

    import paper_1911_03813_amd as S

    from paper_1911_03813_amd import autotune
    autotune.clear()
    tuning = {"cache": None, "entries": 0}
    if not args.no_tuning and os.path.exists(args.tuning):
        tuning = {"cache": os.path.relpath(args.tuning, ROOT), "entries": autotune.load(args.tuning)}

    W = WORKLOAD
    d, n, r, p = W["d"], W["n"], W["r"], W["p"]
    lowp = args.prec in ("fp16", "bf16x3")
    dt = torch.float64 if args.prec == "fp64" else torch.float32
    V, nu, _ = synth.gmm(n, r, p, W["sigma"], 3)
    A = synth.gauss_factors(n, r, 3, 5)
    lam = np.ones(r)
    Vs = V if args.prec == "fp64" else V.astype(np.float32).astype(np.float64)
    As = A if args.prec == "fp64" else A.astype(np.float32).astype(np.float64)

    dev = torch.device("cuda:0")
    Vd = S.colmajor(torch.from_numpy(np.ascontiguousarray(Vs)).to(dt)).to(dev)
    Ad = S.colmajor(torch.from_numpy(np.ascontiguousarray(As)).to(dt)).to(dev)
    nud = torch.from_numpy(nu).to(dev)
    lamd = torch.from_numpy(lam).to(dev)
    ctx = S.Context(0)
    S.symtd_set_tuning(ctx, S.TUNE_G1_BLOCKS, args.g1_blocks)
    S.symtd_set_tuning(ctx, S.TUNE_G2_SPLITS, args.g2_splits)
    out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(r, dtype=torch.float64, device=dev),
           S.colmajor(torch.empty(n, r, dtype=dt, device=dev)))
    # the 16-bit precisions evaluate on a prepared data handle (conversion outside the timed region)
    data = S.Data(ctx, Vd, nud, S.PREC_FP16 if args.prec == "fp16" else S.PREC_BF16X3) if lowp else None

    def evaluate():
        if lowp:
            data.fg(Ad, lamd, d, 0.0, out=out)
        else:
            S.symtd_fg(ctx, Vd, nud, Ad, lamd, d, 0.0, out=out)

    # The timed region brackets the two products with HIP events (the
    # roofline's kernel durations); the events come from the library's pool,
    # filled during the warmup, so the region creates none.
    timed_kernels = ("gemm1", "gemm2")
    S.symtd_profile_enable(ctx, True, kernels=timed_kernels)
    for _ in range(args.warmup):
        evaluate()
    torch.cuda.synchronize()
    S.symtd_profile_reset(ctx)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        evaluate()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.symtd_profile_enable(ctx, False)

    def read_profile(steps):
        out = {}
        for k, name in enumerate(S.profile_names()):
            ms, cnt = S.symtd_profile_read(ctx, k)
            if cnt:
                out[name] = {"avg_us": 1e3 * ms / cnt, "launches": cnt, "step_us": 1e3 * ms / steps}
        S.symtd_profile_reset(ctx)
        return out

    per_kernel = read_profile(args.steps)
    # every kernel's duration, from a shorter pass after the timed region
    bsteps = max(10, args.steps // 4)
    S.symtd_profile_enable(ctx, True)
    for _ in range(bsteps):
        evaluate()
    torch.cuda.synchronize()
    S.symtd_profile_enable(ctx, False)
    breakdown = read_profile(bsteps)
    # per-call duration quantiles, and the evaluation replayed from a graph
    calls = call_stats(evaluate, max(20, args.steps))
    graph = graph_rate(evaluate, out, max(20, args.steps))

    sec = (t1 - t0) / args.steps
    evals = 1.0 / sec
    flop_gemm = 2.0 * n * p * r                       # each of the two products
    flop_step = 2 * flop_gemm + 4.0 * n * r * r       # plus B = A'A and A D_lambda C
    peak = PEAK_TFLOPS["fp16" if lowp else args.prec]
    mult = 3.0 if args.prec == "bf16x3" else 1.0     # executed matrix-core flops per algorithmic flop
    # the dominant product; with r > 16 * (subtiles per launch) it runs as
    # several column-group launches, so its algorithmic flops per step are
    # divided by its summed launch time per step
    dom = max(("gemm1", "gemm2"), key=lambda k: per_kernel.get(k, {"step_us": 0})["step_us"])
    dom_us = per_kernel[dom]["step_us"]
    traffic = traffic_for(args.prec, dom)
    if lowp:
        # the 16-bit products stream V at ~112 flop per byte (2 r flop per
        # 2-byte value), under the ridge 2500 / 8 = 312: HBM-bound.  Their
        # algorithmic bytes: V's 16-bit copy (both planes for bf16x3), A's
        # copy and W (written by gemm1, read by gemm2), all once.
        planes = 2 if args.prec == "bf16x3" else 1
        alg_bytes = 2.0 * planes * (n * p + n * r + p * r)
        roof = {"kernel": dom, "bound": "hbm", "achieved": alg_bytes / (dom_us * 1e-6) / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "algorithmic_bytes": alg_bytes}
    else:
        roof = {"kernel": dom, "bound": "mfma", "achieved": mult * flop_gemm / (dom_us * 1e-6) / 1e12, "peak": peak,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic
    roof["launches_per_step"] = per_kernel[dom]["launches"] / args.steps

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
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16", "bf16x3": "bf16x3"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "large single instance: Gaussian mixture d=3 n=1000 r=100 p=100000 sigma=1e-2",
                   "d": d, "n": n, "r": r, "p": p, "precision": args.prec,
                   "storage": "fp64" if args.prec == "fp64" else "fp32"},
        "step_mfma_frac": mult * flop_step * evals / (peak * 1e12),
        "roofline": roof,
        "kernels_us_per_step": {k: round(v["step_us"], 2) for k, v in breakdown.items()},
        "kernels_us_per_step_note": f"every kernel, timed over {bsteps} steps after the timed region",
        "per_call": calls,
        "graph_replay": graph,
        "tuning": tuning,
    }
    if data is not None:
        data.close()
    del Vd, Ad, out
    if not args.only_fg:
        legs = set(args.legs.split(",")) if args.legs != "all" else None
        want = lambda name: legs is None or name in legs
        V32 = V.astype(np.float32).astype(np.float64)
        A32 = A.astype(np.float32).astype(np.float64)
        if want("precisions"):
            res["precisions"] = precision_leg(S, ctx, V32, nu, A32, lam, d, args.steps, args.warmup)
        if want("normx"):
            res["normx"] = normx_leg(S, ctx, V32, nu, d)
        if want("small"):
            res["small"] = small_leg(S, ctx)
        if want("mid"):
            res["mid"] = mid_leg(S, ctx, args.pgtol)
        if want("table1"):
            res["table1"] = table1_leg(S, ctx)
        if want("stochastic") and not args.no_stoch:
            res["stochastic"] = stoch_leg(S, ctx, args.pgtol)
        if want("corrected"):
            res["corrected"] = corrected_leg(S, ctx, args.pgtol)
        if want("batched") and args.batched > 0:
            res["batched"] = batched_leg(S, ctx, args.batched, args.pgtol, args.batched_max_evals,
                                         not args.no_batched_loop)
        if want("served") and args.served > 0:
            res["served"] = served_leg(S, ctx, args.served, args.rate, args.pgtol)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(Vs, nu, As, lam, d, args.cpu_seconds)
    ctx.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
