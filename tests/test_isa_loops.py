"""The matrix-core loops of the hot kernels keep their accumulators in place.

LLVM's AMDGPU backend may give loop-carried MFMA accumulators VGPRs and then
copy every one of them to AGPRs and back (v_accvgpr_read / write / mov) at
each step of the k loop, or spill them; the kernels pin them with an empty
inline-asm AGPR operand instead.  This test compiles the kernel sources for
gfx950 (device code only, to assembly, with the library's own flags) and
checks, for the benchmark's instantiations, that the innermost loops holding
the most MFMA instructions of each kernel contain no accumulator copies and
no scratch accesses.  A compiler or source change that brings the copies back
fails here, on the CPU.  (The 16-bit first product's chunk loop holds the
hand-off's wait loop, so it has no innermost MFMA loop and is not covered.)
"""

import collections
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_1911_03813_amd import _build

CSRC = _build.CSRC
HIPCC = _build.HIPCC

# source file -> mangled-name prefixes of the kernels checked in it
KERNELS = {
    "fg_kernels.hip": [
        "_ZN5symtd7k_gemm1IdLi7ELb1ELb1E",     # fp64 first product, DMA path, narrow last subtile
        "_ZN5symtd7k_gemm1IfLi7ELb1ELb1E",     # fp32
        "_ZN5symtd7k_gemm2IdLi7ELi2ELb1ELb1E",  # fp64 second product
        "_ZN5symtd7k_gemm2IfLi7ELi3ELb1ELb1E",  # fp32
    ],
    "normx_kernels.hip": [
        "_ZN5symtd7k_normxIfLb1E",
        "_ZN5symtd7k_normxIdLb1E",
    ],
    "lp_kernels.hip": [
        "_ZN5symtd10k_lp_gemm2ILi0ELi7E",      # fp16 second product
        "_ZN5symtd10k_lp_gemm2ILi1ELi7E",      # bf16x3
    ],
    "grouped_kernels.hip": [
        "_ZN5symtd8k_ggemm1IdLb1E",
        "_ZN5symtd8k_ggemm1IfLb1E",
        "_ZN5symtd8k_ggemm2IdLb1E",
        "_ZN5symtd8k_ggemm2IfLb1E",
    ],
}


def assemble(src, out_dir):
    out = os.path.join(out_dir, src[:-4] + ".s")
    cmd = [HIPCC, *_build.CFLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    with open(out) as fh:
        return fh.read()


def functions(asm):
    """name -> body lines of every function in an assembly listing."""
    out = {}
    for m in re.finditer(r"^(_ZN5symtd\S+):[^\n]*\n", asm, re.M):
        end = asm.index(".Lfunc_end", m.end())
        out[m.group(1)] = asm[m.end():end].split("\n")
    return out


def loops(body):
    """(first, last) line pairs of the loops: a branch back to an earlier label."""
    labels = {ln.split(":")[0]: i for i, ln in enumerate(body) if re.match(r"^\.LBB\S+:", ln)}
    found = []
    for i, ln in enumerate(body):
        m = re.match(r"\s+s_(?:c?branch\w*)\s+(\.LBB\S+)", ln)
        if m and m.group(1) in labels and labels[m.group(1)] < i:
            found.append((labels[m.group(1)], i))
    return found


def mix(body, lo, hi):
    ops = collections.Counter()
    for ln in body[lo:hi + 1]:
        t = ln.split()
        if t and not t[0].startswith((";", ".")):
            ops[t[0]] += 1
    return ops


def main_loops(body):
    """The innermost loops with the most MFMA instructions, with their mixes."""
    ls = loops(body)
    inner = [a for a in ls if not any(b != a and a[0] <= b[0] and b[1] <= a[1] for b in ls)]
    mixes = {a: mix(body, *a) for a in inner}
    nmfma = {a: sum(v for k, v in mixes[a].items() if "_mfma_" in k) for a in inner}
    top = max(nmfma.values(), default=0)
    return [(a, mixes[a], nmfma[a]) for a in inner if top and nmfma[a] == top]


@pytest.fixture(scope="module")
def listings(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc is not installed")
    d = str(tmp_path_factory.mktemp("isa"))
    with cf.ThreadPoolExecutor(max_workers=len(KERNELS)) as ex:
        futs = {src: ex.submit(assemble, src, d) for src in KERNELS}
        return {src: functions(f.result()) for src, f in futs.items()}


@pytest.mark.parametrize("src,prefix", [(s, p) for s, ps in KERNELS.items() for p in ps])
def test_k_loop_keeps_accumulators_in_place(listings, src, prefix):
    names = [n for n in listings[src] if n.startswith(prefix)]
    assert len(names) == 1, (prefix, names)
    found = main_loops(listings[src][names[0]])
    assert found, f"no MFMA loop found in {names[0]}"
    for (lo, hi), ops, nmfma in found:
        copies = {k: v for k, v in ops.items() if k.startswith("v_accvgpr_")}
        scratch = {k: v for k, v in ops.items() if k.startswith("scratch_")}
        assert not copies and not scratch, (names[0], (lo, hi), nmfma, copies, scratch)
