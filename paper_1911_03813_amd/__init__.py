"""symtd: implicit symmetric CP decomposition of moment tensors on MI355X.

Thin Python binding of the C ABI in include/symtd.h (libsymtd.so, built
in-tree by ``paper_1911_03813_amd._build``).  The functions here carry the
same names as the C entry points and only marshal arguments: every step of
the computation runs in the library's HIP kernels.  There is no CPU
fallback; if the library is missing, every call raises.

Matrices are torch tensors on the GPU in column-major layout: an n x p
matrix has shape (n, p) and strides (1, ld) with ld >= n.  ``colmajor``
makes such a tensor from any tensor.
"""

from __future__ import annotations

import ctypes
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libsymtd.so")

SYMTD_OK = 0
STATUS = {0: "SYMTD_OK", -1: "SYMTD_EINVAL", -2: "SYMTD_EALIGN", -3: "SYMTD_ENOMEM",
          -4: "SYMTD_EDEVICE", -5: "SYMTD_EUNSUPPORTED", -6: "SYMTD_ENONFINITE", -7: "SYMTD_EREJECTED"}
F64, F32 = 0, 1
PREC_FP64, PREC_FP32 = 0, 1


class SymtdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_c = ctypes
_vp = _c.c_void_p
_i64 = _c.c_int64
_int = _c.c_int
_dbl = _c.c_double

# (name, restype, argtypes) of every C entry point
SIGNATURES = {
    "symtd_create": (_int, [_int, _c.POINTER(_vp)]),
    "symtd_destroy": (None, [_vp]),
    "symtd_last_error": (_c.c_char_p, [_vp]),
    "symtd_status_string": (_c.c_char_p, [_int]),
    "symtd_fg": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _int,
                        _dbl, _int, _vp, _vp, _vp, _i64]),
    "symtd_normX": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _int, _vp]),
    "symtd_set_tuning": (_int, [_vp, _int, _i64]),
    "symtd_profile_enable": (_int, [_vp, _int]),
    "symtd_profile_reset": (_int, [_vp]),
    "symtd_profile_read": (_int, [_vp, _int, _c.POINTER(_dbl), _c.POINTER(_i64)]),
    "symtd_profile_name": (_c.c_char_p, [_int]),
}


def lib():
    """The loaded libsymtd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1911_03813_amd._build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, status: int):
    if status != SYMTD_OK:
        msg = lib().symtd_last_error(ctx._h if ctx is not None else None)
        raise SymtdError(status, msg.decode() if msg else "")


class Context:
    """A symtd context on one HIP device (owns the device workspace)."""

    def __init__(self, device: int = 0):
        h = _vp()
        st = lib().symtd_create(device, ctypes.byref(h))
        if st != SYMTD_OK:
            raise SymtdError(st, f"symtd_create(device={device}) failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().symtd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


# --- tensor marshalling -------------------------------------------------------

def colmajor(t):
    """A column-major copy (strides (1, rows)) of a 2-D tensor."""
    return t.t().contiguous().t()


def _mat(t, name, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if t.dtype not in (torch.float32, torch.float64):
        raise TypeError(f"{name} must be float32 or float64")
    rows, cols = t.shape
    if t.stride(0) != 1 and rows > 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    ld = t.stride(1) if cols > 1 else max(rows, 1)
    return t.data_ptr(), int(ld)


def _vec(t, name, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.dim() != 1 or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a 1-D float64 GPU tensor")
    if t.stride(0) != 1 and t.numel() > 1:
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    return t.data_ptr()


def _dt(t):
    import torch
    return F64 if t.dtype == torch.float64 else F32


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# --- entry points -------------------------------------------------------------

def symtd_fg(ctx: Context, V, nu, A, lam, d: int, alpha: float = 0.0, prec: int | None = None,
             out=None, stream=None):
    """f, g_lambda, G_A of Algorithm 2 for (nu, V) and the model (lam, A).

    Returns device tensors (f: shape (1,) float64, g_lambda: (r,) float64,
    G_A: (n, r) column-major with A's dtype).  Asynchronous on `stream`.
    """
    import torch
    Vp, ldv = _mat(V, "V")
    Ap, lda = _mat(A, "A", V.dtype)
    n, p = V.shape
    n2, r = A.shape
    if n2 != n:
        raise ValueError("A must have as many rows as V")
    nup = _vec(nu, "nu", p)
    lp = _vec(lam, "lambda", r)
    if prec is None:
        prec = PREC_FP64 if V.dtype == torch.float64 else PREC_FP32
    if out is None:
        f = torch.empty(1, dtype=torch.float64, device=V.device)
        g = torch.empty(r, dtype=torch.float64, device=V.device)
        G = colmajor(torch.empty(n, r, dtype=V.dtype, device=V.device))
    else:
        f, g, G = out
    Gp, ldg = _mat(G, "G_A", V.dtype)
    st = lib().symtd_fg(ctx.handle, _stream(stream), _dt(V), Vp, ldv, nup, n, p, Ap, lda, lp, r, int(d),
                        float(alpha), int(prec), _vec(f, "f", 1), _vec(g, "g_lambda", r), Gp, ldg)
    _check(ctx, st)
    return f, g, G


def symtd_normX(ctx: Context, V, nu, d: int, out=None, stream=None):
    """alpha = ||X||^2 = nu'[V'V]^d nu as a (1,) float64 device tensor."""
    import torch
    Vp, ldv = _mat(V, "V")
    n, p = V.shape
    nup = _vec(nu, "nu", p)
    a = out if out is not None else torch.empty(1, dtype=torch.float64, device=V.device)
    st = lib().symtd_normX(ctx.handle, _stream(stream), _dt(V), Vp, ldv, nup, n, p, int(d), _vec(a, "alpha", 1))
    _check(ctx, st)
    return a


TUNE_G1_BLOCKS, TUNE_G2_SPLITS, TUNE_SERIAL = 0, 1, 2


def symtd_set_tuning(ctx: Context, key: int, value: int):
    """Override a work-split choice of the evaluation kernels (0 = automatic)."""
    _check(ctx, lib().symtd_set_tuning(ctx.handle, int(key), int(value)))


def symtd_profile_enable(ctx: Context, enable: bool = True):
    _check(ctx, lib().symtd_profile_enable(ctx.handle, int(bool(enable))))


def symtd_profile_reset(ctx: Context):
    _check(ctx, lib().symtd_profile_reset(ctx.handle))


def symtd_profile_read(ctx: Context, which: int):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(ctx, lib().symtd_profile_read(ctx.handle, int(which), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def symtd_profile_name(which: int):
    s = lib().symtd_profile_name(int(which))
    return s.decode() if s else None


def profile_names():
    out = []
    i = 0
    while True:
        s = symtd_profile_name(i)
        if s is None:
            return out
        out.append(s)
        i += 1
