"""Build libsymtd.so (the HIP kernels and the C ABI) in-tree for gfx950.

Usage: python -m paper_1911_03813_amd._build [--verbose] [--resource-usage] [--host-sanitizers]

Every .hip file under csrc/ is compiled with hipcc to an object file under
_build/, and the objects are linked into paper_1911_03813_amd/libsymtd.so.

--host-sanitizers builds the same library with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (the device code is the
same), under _build_asan/ into _build_asan/libsymtd_asan.so.  Its sanitizer
symbols are left for the process to supply: it is loaded into a process
that preloads clang's shared ASan runtime (tests/test_host_sanitizers.py).
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsymtd.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = "/opt/rocm/lib"
BUILD_ASAN = os.path.join(ROOT, "_build_asan")
LIB_ASAN = os.path.join(BUILD_ASAN, "libsymtd_asan.so")
# host-side only: each sanitizer flag applies to the host compilation alone
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # keep hand-written and compiler-generated fp32 math off the packed-fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def _compile(src: str, verbose: bool, resource: bool, asan: bool = False) -> str:
    obj = os.path.join(BUILD_ASAN if asan else BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *(ASAN_FLAGS if asan else []), "-c", src, "-o", obj]
    if resource:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = res.stdout + res.stderr
    # hipcc's host pass does not know the device-only feature above; that note is harmless
    lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
    if verbose or resource or res.returncode != 0:
        if lines:
            print("\n".join(lines), file=sys.stderr)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, resource: bool = False, asan: bool = False) -> str:
    os.makedirs(BUILD_ASAN if asan else BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, resource, asan), srcs))
    out = LIB_ASAN if asan else LIB
    tmp = out + ".tmp"
    # roctx: the solve, step and admission ranges that rocprofv3 --marker-trace records
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L", ROCM_LIB,
           "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        print(res.stdout + res.stderr, file=sys.stderr)
        raise RuntimeError("link of libsymtd.so failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--resource-usage", action="store_true")
    ap.add_argument("--host-sanitizers", action="store_true")
    a = ap.parse_args()
    print(build(a.verbose, a.resource_usage, a.host_sanitizers))
