"""The host side of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

`python -m paper_1911_03813_amd._build --host-sanitizers` builds the library
with both sanitizers on its host code (its device code unchanged) into
_build_asan/.  A child process preloads clang's shared ASan runtime, loads
that build through the binding (SYMTD_LIBRARY) and drives every entry point
that needs no device: the status strings, the option defaults, the size of a
paused solve's state, the process-wide tuning table (including its growth
and replacement of entries), context creation (which fails without a GPU)
and the null-argument refusals of the compute entry points.  Any sanitizer
report ends the child with a non-zero status.
"""

import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_LIB = os.path.join(ROOT, "_build_asan", "libsymtd_asan.so")
RUNTIMES = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

CHILD = textwrap.dedent("""
    import ctypes
    import paper_1911_03813_amd as S
    L = S.lib()
    assert L._name.endswith("libsymtd_asan.so"), L._name
    for st in range(-8, 1):
        assert L.symtd_status_string(st)
    assert L.symtd_last_error(None) is not None
    o = S.SolveOpts()
    assert L.symtd_solve_opts_default(ctypes.byref(o)) == 0 and o.m == 5 and o.restarts == 1
    assert L.symtd_solve_opts_default(None) == -1
    ao = S.AdamOpts()
    assert L.symtd_adam_opts_default(ctypes.byref(ao)) == 0
    pb = S.Problem(0, None, 30, None, 30, 1000, 3, 4)
    nb = ctypes.c_size_t()
    for R, m, tl in ((1, 1, 0), (3, 5, 10), (4096, 8, 1000)):
        o.restarts, o.m = R, m
        assert L.symtd_solve_state_bytes(ctypes.byref(pb), ctypes.byref(o), tl, ctypes.byref(nb)) == 0
        assert nb.value > 0
    assert L.symtd_solve_state_bytes(None, ctypes.byref(o), 0, ctypes.byref(nb)) == -1
    assert L.symtd_solve_state_bytes(ctypes.byref(pb), ctypes.byref(o), -1, ctypes.byref(nb)) == -1
    # the tuning table: many entries (growth), replacement of an existing key, reads past the end
    L.symtd_tune_clear()
    for i in range(300):
        e = S.TuneEntry(i % 2, i % 3, i % 11, i % 17, i % 7, 64 + i, 3 + i, 10.0 + i)
        assert L.symtd_tune_put(ctypes.byref(e)) == 0
    count = L.symtd_tune_count()
    assert 0 < count <= 300
    g = S.TuneEntry()
    for i in range(count):
        assert L.symtd_tune_get(i, ctypes.byref(g)) == 0
    assert L.symtd_tune_get(count, ctypes.byref(g)) != 0
    assert L.symtd_tune_get(-1, ctypes.byref(g)) != 0
    assert L.symtd_tune_put(None) == -1
    # the same key again replaces its entry
    e = S.TuneEntry(0, 0, 0, 0, 0, 999, 7, 1.0)
    assert L.symtd_tune_put(ctypes.byref(e)) == 0
    assert L.symtd_tune_count() == count
    L.symtd_tune_clear()
    assert L.symtd_tune_count() == 0
    # no GPU here: creating a context fails cleanly
    h = ctypes.c_void_p()
    assert L.symtd_create(0, ctypes.byref(h)) != 0 and not h.value
    assert L.symtd_create(0, None) != 0
    L.symtd_destroy(None)
    L.symtd_data_destroy(None)
    L.symtd_server_destroy(None)
    # compute entry points refuse a null context before touching anything
    assert L.symtd_normX(None, None, 0, None, 1, None, 1, 1, 3, None) == -1
    assert L.symtd_check(None, None) == -1
    assert L.symtd_solve(None, None, ctypes.byref(pb), ctypes.byref(o), None) == -1
    h2 = ctypes.c_void_p()
    assert L.symtd_server_create(None, ctypes.byref(h2)) == -1
    print("host paths done")
""")


@pytest.mark.skipif(not RUNTIMES, reason="clang's shared ASan runtime is not installed")
def test_host_entry_points_under_asan_and_ubsan():
    srcs = glob.glob(os.path.join(ROOT, "paper_1911_03813_amd", "csrc", "*"))
    stale = (not os.path.exists(ASAN_LIB)
             or os.path.getmtime(ASAN_LIB) < max(os.path.getmtime(s) for s in srcs + [os.path.join(ROOT, "include", "symtd.h")]))
    if stale:
        subprocess.run([sys.executable, "-m", "paper_1911_03813_amd._build", "--host-sanitizers"], cwd=ROOT,
                       check=True, capture_output=True, timeout=900)
    env = dict(os.environ)
    # the ASan runtime first, in front of whatever the environment already preloads
    env["LD_PRELOAD"] = ":".join([RUNTIMES[-1]] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:exitcode=86:alloc_dealloc_mismatch=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    env["SYMTD_LIBRARY"] = ASAN_LIB
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    res = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=300)
    report = res.stdout + res.stderr
    assert res.returncode == 0, report[-4000:]
    assert "host paths done" in res.stdout
    assert "AddressSanitizer" not in report and "runtime error:" not in report, report[-4000:]


@pytest.mark.skipif(not RUNTIMES, reason="clang's shared ASan runtime is not installed")
def test_the_preloaded_runtime_halts_on_an_overflow():
    # the same preload and options stop a process at a heap overflow (a write
    # one byte past a malloc'd block through the intercepted memset)
    env = dict(os.environ)
    env["LD_PRELOAD"] = ":".join([RUNTIMES[-1]] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:exitcode=86:alloc_dealloc_mismatch=0"
    code = ("import ctypes; c = ctypes.CDLL(None); c.malloc.restype = ctypes.c_void_p; "
            "p = c.malloc(16); c.memset(ctypes.c_void_p(p), 0, 17)")
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert res.returncode == 86 and "heap-buffer-overflow" in res.stderr, res.stderr[-2000:]
