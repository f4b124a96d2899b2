"""The autotuner's Python side: run the library's tuners, and keep the
process-wide tuning table (include/symtd.h, symtd_tune_*) in a JSON cache.

    python -m paper_1911_03813_amd.autotune --out CACHE.json [--quick]

tunes, on cuda:0, the single evaluation of the large (d=3, n=1000, p=1e5,
r=100), mid-size (d=4, n=100, p=5000, r=20) and small (d=3, n=10, p=750,
r=3) workloads in fp64 and fp32, and the grouped second product for every
(n, p, columns) bucket of the batched workload (n ~ U{16..256}, r ~
U{2..32}, p = 250 r, 4 restarts), and writes the table.  load(CACHE.json)
puts a saved table back; an evaluation planned afterwards uses it.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys

from . import (F32, F64, PREC_FP32, PREC_FP64, Context, SymtdError, TuneEntry, _check, _dt, _mat, _stream, _vec,
               colmajor, lib)

KIND_FG, KIND_GROUPED = 0, 1
FIELDS = ("kind", "prec", "n_bucket", "p_bucket", "r_bucket", "v0", "v1", "us")


def entries():
    """The table as a list of dicts."""
    out = []
    e = TuneEntry()
    for i in range(int(lib().symtd_tune_count())):
        _check(None, lib().symtd_tune_get(i, ctypes.byref(e)))
        out.append({k: getattr(e, k) for k in FIELDS})
    return out


def put(entry: dict):
    e = TuneEntry(**{k: entry[k] for k in FIELDS})
    st = lib().symtd_tune_put(ctypes.byref(e))
    if st != 0:
        raise SymtdError(st, f"bad tuning entry {entry}")


def clear():
    lib().symtd_tune_clear()


def save(path: str, meta: dict | None = None):
    with open(path, "w") as fh:
        json.dump({"meta": meta or {}, "entries": entries()}, fh, indent=1)


def load(path: str) -> int:
    """Put every entry of a saved table; returns their number."""
    with open(path) as fh:
        doc = json.load(fh)
    for e in doc["entries"]:
        put(e)
    return len(doc["entries"])


def bucket(x: int) -> int:
    return max(0, math.ceil(math.log2(max(int(x), 1))))


def tune_fg(ctx: Context, V, nu, A, lam, d: int, reps: int = 10, stream=None) -> dict:
    """symtd_autotune_fg on the given device data (fp64 or fp32 products)."""
    Vp, ldv = _mat(V, "V")
    Ap, lda = _mat(A, "A", V.dtype)
    n, p = V.shape
    r = A.shape[1]
    prec = PREC_FP64 if _dt(V) == F64 else PREC_FP32
    e = TuneEntry()
    _check(ctx, lib().symtd_autotune_fg(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p, Ap,
                                        lda, _vec(lam, "lambda", r), r, int(d), prec, int(reps), ctypes.byref(e)))
    return {k: getattr(e, k) for k in FIELDS}


def tune_grouped(ctx: Context, V, nu, d: int, cols: int, copies: int = 64, reps: int = 3, stream=None) -> dict:
    """symtd_autotune_grouped for instances shaped like (V, nu, d, cols)."""
    Vp, ldv = _mat(V, "V")
    n, p = V.shape
    e = TuneEntry()
    _check(ctx, lib().symtd_autotune_grouped(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p,
                                             int(d), int(cols), int(copies), int(reps), ctypes.byref(e)))
    return {k: getattr(e, k) for k in FIELDS}


def _main(argv=None):
    import os

    import numpy as np
    import torch

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--quick", action="store_true", help="fewer grouped buckets (a smoke run of the tuner)")
    a = ap.parse_args(argv)
    ctx = Context(0)
    clear()
    for (d, n, p, r, key) in ((3, 1000, 100_000, 100, 3), (4, 100, 5000, 20, 12), (3, 10, 750, 3, 11)):
        V, nu, _ = synth.gmm(n, r, p, 1e-2, key)
        A = synth.gauss_factors(n, r, key, 5)
        for dt in (torch.float64, torch.float32):
            Vd = colmajor(torch.from_numpy(V).to(dt)).cuda()
            Ad = colmajor(torch.from_numpy(A).to(dt)).cuda()
            e = tune_fg(ctx, Vd, torch.from_numpy(nu).cuda(), Ad, torch.ones(r, dtype=torch.float64, device="cuda"),
                        d, reps=5 if n * p > 1e7 else 20)
            print(f"fg d={d} n={n} p={p} r={r} {dt}: {e}", flush=True)
            del Vd, Ad
    # grouped buckets of the batched workload: one representative per bucket
    shapes = synth.batch_shapes(512, 4)
    reps = {}
    for s in shapes:
        key = (bucket(s["n"]), bucket(s["p"]), bucket(4 * s["r"]))
        reps.setdefault(key, s)
    keys = sorted(reps)
    if a.quick:
        keys = keys[:4]
    for i, key in enumerate(keys):
        s = reps[key]
        V, nu, _ = synth.gmm(s["n"], s["r"], s["p"], s["sigma"], 4, 10_000 + i)
        Vd = colmajor(torch.from_numpy(V).float()).cuda()
        e = tune_grouped(ctx, Vd, torch.from_numpy(nu).cuda(), s["d"], 4 * s["r"])
        print(f"grouped n={s['n']} p={s['p']} cols={4 * s['r']}: {e}", flush=True)
    save(a.out, {"device": torch.cuda.get_device_name(0), "grouped_copies": 64,
                 "note": "symtd tuning table (include/symtd.h, symtd_tune_entry)"})
    print(f"wrote {len(entries())} entries to {a.out}", flush=True)
    ctx.close()


if __name__ == "__main__":
    _main()
