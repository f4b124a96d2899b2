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
