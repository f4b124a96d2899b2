"""The C ABI library: loads, exports every declared symbol, rejects bad
arguments without touching a GPU (CPU-only tests)."""

import ctypes
import os
import re

import pytest

import paper_1911_03813_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(symtd_\w+)\s*\(", txt))
    return names


def test_library_built():
    assert os.path.exists(S.LIB_PATH), "run __graft_entry__.build() first"


def test_exports_every_declared_symbol():
    lib = S.lib()
    declared = _declared()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(lib, name), f"libsymtd.so does not export {name}"
    # the Python binding marshals every declared entry point
    assert declared <= set(S.SIGNATURES), declared - set(S.SIGNATURES)


def test_status_strings():
    lib = S.lib()
    for code, name in S.STATUS.items():
        assert lib.symtd_status_string(code).decode() == name


def test_null_context_rejected():
    lib = S.lib()
    assert lib.symtd_fg(None, None, 0, None, 1, None, 1, 1, None, 1, None, 1, 3, 0.0, 0,
                        None, None, None, 1) == -1
    assert lib.symtd_normX(None, None, 0, None, 1, None, 1, 1, 3, None) == -1
    assert lib.symtd_create(0, None) == -1
    assert lib.symtd_last_error(None).decode() == "null context"


def test_profile_names():
    names = S.profile_names()
    assert names[:2] == ["gemm1", "gemm2"]


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of the solve structs have the C header's sizes and offsets
    import ctypes
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    pass
    checks = {
        "symtd_problem": (S.Problem, ["dt", "V", "ldv", "nu", "n", "p", "d", "r"]),
        "symtd_solve_opts": (S.SolveOpts, ["prec", "m", "pgtol", "ftol", "max_iters", "max_evals", "restarts",
                                           "seed", "init", "alpha_mode", "alpha", "A0", "check_every", "sigma",
                                           "pause_after", "state_out", "state_in"]),
        "symtd_fg_item": (S.FgItem, ["V", "ldv", "nu", "n", "p", "d", "A", "lda", "lambda", "r", "models",
                                     "alpha", "f", "g_lambda", "G_A", "ldg"]),
        "symtd_adam_opts": (S.AdamOpts, ["prec", "samples", "est_samples", "epoch_len", "max_epochs", "lr0",
                                         "lr1", "beta1", "beta2", "eps", "restarts", "seed", "init", "A0"]),
        "symtd_server_opts": (S.ServerOpts, ["device", "dt", "prec", "memory_bytes", "check_every", "use_graph"]),
        "symtd_server_result": (S.ServerResult, ["id", "status", "f", "alpha", "rel_err", "iters", "evals",
                                                 "exit_reason", "best_restart", "n", "r", "A", "lambda",
                                                 "t_submit", "t_admit", "t_done"]),
        "symtd_server_stats": (S.ServerStats, ["submitted", "admitted", "completed", "cancelled", "queued",
                                               "running", "steps", "memory_used", "memory_bytes"]),
        "symtd_solve_result": (S.SolveResult, ["A", "lda", "lambda", "f_restarts", "iters_restarts",
                                               "evals_restarts", "exit_restarts", "f_trace", "trace_len", "f",
                                               "alpha", "rel_err", "iters", "evals", "exit_reason",
                                               "best_restart", "steps"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "symtd.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        for fld in fields:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {fld}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for cname, (cls, fields) in checks.items():
        want.append(ctypes.sizeof(cls))
        names = [f[0] for f in cls._fields_]
        for fld in fields:
            fld_py = "lam" if fld == "lambda" else fld
            assert fld_py in names, (cname, fld)
            want.append(getattr(cls, fld_py).offset)
    assert got == want


def test_solve_state_bytes():
    # the size of a paused solve's state: host-only, so it runs without a GPU
    import ctypes

    def size(dt=0, n=30, r=4, restarts=3, m=5, trace_len=0):
        pb = S.Problem(dt, None, n, None, n, 1000, 3, r)
        o = S.SolveOpts()
        assert S.lib().symtd_solve_opts_default(ctypes.byref(o)) == 0
        o.restarts, o.m = restarts, m
        out = ctypes.c_size_t()
        st = S.lib().symtd_solve_state_bytes(ctypes.byref(pb), ctypes.byref(o), trace_len, ctypes.byref(out))
        return st, out.value

    st, base = size()
    assert st == 0
    N = 4 + 30 * 4
    # x, g, d and m pairs of S, Y per restart; fp64 trial factors; per-restart state
    assert base >= 3 * (3 + 2 * 5) * N * 8 + 3 * 4 * 8 + 30 * 4 * 3 * 8
    assert size(m=6)[1] == base + 2 * 3 * N * 8
    assert size(trace_len=10)[1] == base + 3 * 10 * 8
    assert size(dt=1)[1] == base - 30 * 4 * 3 * 4
    assert size(restarts=4)[1] > base
    for bad in (dict(r=0), dict(restarts=0), dict(restarts=4097), dict(m=0), dict(m=9), dict(trace_len=-1),
                dict(dt=7)):
        assert size(**bad)[0] == -1, bad
