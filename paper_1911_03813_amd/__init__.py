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
# SYMTD_LIBRARY names another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree libsymtd.so
LIB_PATH = os.environ.get("SYMTD_LIBRARY") or os.path.join(PKG_DIR, "libsymtd.so")

SYMTD_OK = 0
NOALLOC_SCRATCH_BYTES = 64 << 20   # SYMTD_NOALLOC_SCRATCH_BYTES of include/symtd.h
STATUS = {0: "SYMTD_OK", -1: "SYMTD_EINVAL", -2: "SYMTD_EALIGN", -3: "SYMTD_ENOMEM",
          -4: "SYMTD_EDEVICE", -5: "SYMTD_EUNSUPPORTED", -6: "SYMTD_ENONFINITE", -7: "SYMTD_EREJECTED"}
F64, F32 = 0, 1
PREC_FP64, PREC_FP32, PREC_FP16, PREC_BF16X3 = 0, 1, 2, 3


def prec_bound(prec: int, d: int) -> float:
    """The stated error bound of a product precision (relative to the
    cancelling terms): fp64 1e-12, fp32 1e-5, bf16x3 2(d+1) 3 2^-16, fp16
    2(d+1) 2 2^-11."""
    return {PREC_FP64: 1e-12, PREC_FP32: 1e-5, PREC_BF16X3: 2 * (d + 1) * 3 * 2.0**-16,
            PREC_FP16: 2 * (d + 1) * 2 * 2.0**-11}[prec]


class SymtdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_c = ctypes


class Problem(ctypes.Structure):
    """symtd_problem"""
    _fields_ = [("dt", ctypes.c_int), ("V", ctypes.c_void_p), ("ldv", ctypes.c_int64), ("nu", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("p", ctypes.c_int64), ("d", ctypes.c_int), ("r", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    """symtd_solve_opts"""
    _fields_ = [("prec", ctypes.c_int), ("m", ctypes.c_int), ("pgtol", ctypes.c_double), ("ftol", ctypes.c_double),
                ("max_iters", ctypes.c_int64), ("max_evals", ctypes.c_int64), ("restarts", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("init", ctypes.c_int), ("alpha_mode", ctypes.c_int),
                ("alpha", ctypes.c_double), ("A0", ctypes.c_void_p), ("check_every", ctypes.c_int),
                ("sigma", ctypes.c_double), ("pause_after", ctypes.c_int64), ("state_out", ctypes.c_void_p),
                ("state_in", ctypes.c_void_p)]


class FgItem(ctypes.Structure):
    """symtd_fg_item"""
    _fields_ = [("V", ctypes.c_void_p), ("ldv", ctypes.c_int64), ("nu", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("p", ctypes.c_int64), ("d", ctypes.c_int), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("lam", ctypes.c_void_p), ("r", ctypes.c_int64), ("models", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("f", ctypes.c_void_p), ("g_lambda", ctypes.c_void_p),
                ("G_A", ctypes.c_void_p), ("ldg", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    """symtd_server_opts"""
    _fields_ = [("device", ctypes.c_int), ("dt", ctypes.c_int), ("prec", ctypes.c_int),
                ("memory_bytes", ctypes.c_size_t), ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int)]


class ServerResult(ctypes.Structure):
    """symtd_server_result"""
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int), ("f", ctypes.c_double),
                ("alpha", ctypes.c_double), ("rel_err", ctypes.c_double), ("iters", ctypes.c_int64),
                ("evals", ctypes.c_int64), ("exit_reason", ctypes.c_int), ("best_restart", ctypes.c_int),
                ("n", ctypes.c_int64), ("r", ctypes.c_int64), ("A", ctypes.POINTER(ctypes.c_double)),
                ("lam", ctypes.POINTER(ctypes.c_double)), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    """symtd_server_stats"""
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("memory_used", ctypes.c_size_t), ("memory_bytes", ctypes.c_size_t)]


class AdamOpts(ctypes.Structure):
    """symtd_adam_opts"""
    _fields_ = [("prec", ctypes.c_int), ("samples", ctypes.c_int64), ("est_samples", ctypes.c_int64),
                ("epoch_len", ctypes.c_int), ("max_epochs", ctypes.c_int64), ("lr0", ctypes.c_double),
                ("lr1", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("restarts", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("init", ctypes.c_int), ("A0", ctypes.c_void_p)]


class TuneEntry(ctypes.Structure):
    """symtd_tune_entry"""
    _fields_ = [("kind", ctypes.c_int), ("prec", ctypes.c_int), ("n_bucket", ctypes.c_int),
                ("p_bucket", ctypes.c_int), ("r_bucket", ctypes.c_int), ("v0", ctypes.c_int64),
                ("v1", ctypes.c_int64), ("us", ctypes.c_double)]


class SolveResult(ctypes.Structure):
    """symtd_solve_result"""
    _fields_ = [("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("lam", ctypes.c_void_p),
                ("f_restarts", ctypes.POINTER(ctypes.c_double)), ("iters_restarts", ctypes.POINTER(ctypes.c_int64)),
                ("evals_restarts", ctypes.POINTER(ctypes.c_int64)), ("exit_restarts", ctypes.POINTER(ctypes.c_int)),
                ("f_trace", ctypes.POINTER(ctypes.c_double)), ("trace_len", ctypes.c_int64),
                ("f", ctypes.c_double), ("alpha", ctypes.c_double), ("rel_err", ctypes.c_double),
                ("iters", ctypes.c_int64), ("evals", ctypes.c_int64), ("exit_reason", ctypes.c_int),
                ("best_restart", ctypes.c_int), ("steps", ctypes.c_int64)]

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
    "symtd_check": (_int, [_vp, _vp]),
    "symtd_fg": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _int,
                        _dbl, _int, _vp, _vp, _vp, _i64]),
    "symtd_fg_noalloc": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _int,
                                _dbl, _int, _vp, _vp, _vp, _i64]),
    "symtd_fg_multi": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _i64, _int,
                              _dbl, _int, _vp, _vp, _vp, _i64]),
    "symtd_normX": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _int, _vp]),
    "symtd_set_tuning": (_int, [_vp, _int, _i64]),
    "symtd_data_create": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _int, _c.POINTER(_vp)]),
    "symtd_data_destroy": (None, [_vp]),
    "symtd_fg_data": (_int, [_vp, _vp, _vp, _vp, _i64, _vp, _i64, _int, _dbl, _vp, _vp, _vp, _i64]),
    "symtd_solve_opts_default": (_int, [_c.POINTER(SolveOpts)]),
    "symtd_solve": (_int, [_vp, _vp, _c.POINTER(Problem), _c.POINTER(SolveOpts), _c.POINTER(SolveResult)]),
    "symtd_solve_state_bytes": (_int, [_c.POINTER(Problem), _c.POINTER(SolveOpts), _i64, _c.POINTER(_c.c_size_t)]),
    "symtd_form_moment": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _int, _vp]),
    "symtd_moment_stats": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _vp]),
    "symtd_fg_corrected": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _int, _dbl,
                                  _int, _dbl, _vp, _vp, _vp, _vp, _vp, _i64]),
    "symtd_alpha_corrected": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _int, _dbl, _vp, _vp, _dbl,
                                     _c.POINTER(_dbl)]),
    "symtd_fg_explicit": (_int, [_vp, _vp, _int, _vp, _i64, _int, _vp, _i64, _vp, _i64, _dbl, _int, _vp, _vp, _vp,
                                 _i64]),
    "symtd_fg_sampled": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _i64, _c.c_uint64, _i64, _vp, _i64,
                                _vp, _i64, _int, _int, _vp, _vp, _vp, _i64, _vp]),
    "symtd_adam_opts_default": (_int, [_c.POINTER(AdamOpts)]),
    "symtd_solve_adam": (_int, [_vp, _vp, _c.POINTER(Problem), _c.POINTER(AdamOpts), _c.POINTER(SolveResult)]),
    "symtd_fg_batched": (_int, [_vp, _vp, _int, _int, _i64, _c.POINTER(FgItem)]),
    "symtd_server_create": (_int, [_c.POINTER(ServerOpts), _c.POINTER(_vp)]),
    "symtd_server_submit": (_int, [_vp, _c.POINTER(Problem), _c.POINTER(SolveOpts), _c.POINTER(_c.c_uint64)]),
    "symtd_server_poll": (_int, [_vp, _c.POINTER(ServerResult), _c.c_int32, _c.POINTER(_c.c_int32), _c.c_int32]),
    "symtd_server_cancel": (_int, [_vp, _c.c_uint64]),
    "symtd_server_stats_get": (_int, [_vp, _c.POINTER(ServerStats)]),
    "symtd_server_last_error": (_c.c_char_p, [_vp]),
    "symtd_server_result_release": (None, [_c.POINTER(ServerResult)]),
    "symtd_server_destroy": (None, [_vp]),
    "symtd_solve_batched": (_int, [_vp, _vp, _i64, _c.POINTER(Problem), _c.POINTER(SolveOpts),
                                   _c.POINTER(SolveResult)]),
    "symtd_tune_put": (_int, [_c.POINTER(TuneEntry)]),
    "symtd_tune_count": (_i64, []),
    "symtd_tune_get": (_int, [_i64, _c.POINTER(TuneEntry)]),
    "symtd_tune_clear": (None, []),
    "symtd_autotune_fg": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _int, _int, _int,
                                 _c.POINTER(TuneEntry)]),
    "symtd_autotune_grouped": (_int, [_vp, _vp, _int, _vp, _i64, _vp, _i64, _i64, _int, _i64, _int, _int,
                                      _c.POINTER(TuneEntry)]),
    "symtd_profile_enable": (_int, [_vp, ctypes.c_uint32]),
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
        msg = lib().symtd_last_error(ctx._h if ctx is not None else None) if ctx is not None else b""
        raise SymtdError(status, msg.decode() if msg else "")


class Context:
    """A symtd context on one HIP device (owns the device workspace)."""

    def __init__(self, device: int = 0):
        # torch's GPU runtime must come up before the library's in the same
        # process (torch finds no device otherwise); tensors are torch's
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
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
             out=None, stream=None, noalloc: bool = False):
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
    entry = lib().symtd_fg_noalloc if noalloc else lib().symtd_fg
    st = entry(ctx.handle, _stream(stream), _dt(V), Vp, ldv, nup, n, p, Ap, lda, lp, r, int(d),
               float(alpha), int(prec), _vec(f, "f", 1), _vec(g, "g_lambda", r), Gp, ldg)
    _check(ctx, st)
    return f, g, G


def symtd_fg_noalloc(ctx: Context, V, nu, A, lam, d: int, alpha: float = 0.0, prec: int | None = None,
                     out=None, stream=None):
    """symtd_fg through the entry point that allocates no device memory (its
    workspace is the library's fixed per-device scratch array).  With `out`
    given, nothing is allocated on the Python side either."""
    return symtd_fg(ctx, V, nu, A, lam, d, alpha, prec, out, stream, noalloc=True)


def symtd_fg_multi(ctx: Context, V, nu, A, lam, r: int, d: int, alpha: float = 0.0, prec: int | None = None,
                   out=None, stream=None):
    """Algorithm 2 for the models side by side in A (n x models*r) and lam.

    Returns (f: (models,) float64, g_lambda: (models*r,) float64, G_A: like A).
    """
    import torch
    Vp, ldv = _mat(V, "V")
    Ap, lda = _mat(A, "A", V.dtype)
    n, p = V.shape
    n2, cols = A.shape
    if n2 != n:
        raise ValueError("A must have as many rows as V")
    if r < 1 or cols % r:
        raise ValueError("A must hold a whole number of r-column models")
    models = cols // r
    nup = _vec(nu, "nu", p)
    lp = _vec(lam, "lambda", cols)
    if prec is None:
        prec = PREC_FP64 if V.dtype == torch.float64 else PREC_FP32
    if out is None:
        f = torch.empty(models, dtype=torch.float64, device=V.device)
        g = torch.empty(cols, dtype=torch.float64, device=V.device)
        G = colmajor(torch.empty(n, cols, dtype=V.dtype, device=V.device))
    else:
        f, g, G = out
    Gp, ldg = _mat(G, "G_A", V.dtype)
    st = lib().symtd_fg_multi(ctx.handle, _stream(stream), _dt(V), Vp, ldv, nup, n, p, Ap, lda, lp, int(r),
                              int(models), int(d), float(alpha), int(prec), _vec(f, "f", models),
                              _vec(g, "g_lambda", cols), Gp, ldg)
    _check(ctx, st)
    return f, g, G


INIT_GAUSS, INIT_RRF = 0, 1
ALPHA_COMPUTE, ALPHA_GIVEN, ALPHA_NONE = 0, 1, 2
EXIT_RUNNING = 0
EXIT_NAMES = {0: "RUNNING", 1: "PGTOL", 2: "FTOL", 3: "MAX_ITERS", 4: "MAX_EVALS", 5: "LINESEARCH", 6: "NONFINITE"}


class _SolveCall:
    """Marshalled arguments and host result buffers of one solve request."""

    def __init__(self, V, nu, d, r, prec=None, m=5, pgtol=1e-4, ftol=2.220446049250313e-09, max_iters=10000,
                 max_evals=50000, restarts=1, seed=0, init=None, alpha=None, A0=None, check_every=0,
                 trace_len=0, sigma=0.0, pause_after=0, state=None):
        import numpy as np
        import torch
        Vp, ldv = _mat(V, "V")
        n, p = V.shape
        nup = _vec(nu, "nu", p)
        if prec is None:
            prec = PREC_FP64 if V.dtype == torch.float64 else PREC_FP32
        self.pb = Problem(_dt(V), Vp, ldv, nup, n, p, int(d), int(r))
        o = SolveOpts()
        _check(None, lib().symtd_solve_opts_default(ctypes.byref(o)))
        o.prec, o.m, o.pgtol, o.ftol = int(prec), int(m), float(pgtol), float(ftol)
        o.max_iters, o.max_evals, o.restarts, o.seed = int(max_iters), int(max_evals), int(restarts), int(seed)
        o.init = INIT_RRF if init is None else int(init)
        if alpha is None:
            o.alpha_mode = ALPHA_COMPUTE
        elif float(alpha) > 0:
            o.alpha_mode, o.alpha = ALPHA_GIVEN, float(alpha)
        else:
            o.alpha_mode = ALPHA_NONE
        self.keep = [V, nu]
        if A0 is not None:
            A0p, lda0 = _mat(A0, "A0", V.dtype)
            if tuple(A0.shape) != (n, restarts * r) or lda0 != n:
                raise ValueError("A0 must be an n x (restarts*r) column-major tensor with leading dimension n")
            o.A0 = A0p
            self.keep.append(A0)
        o.check_every = int(check_every)
        o.sigma = float(sigma)
        o.pause_after = int(pause_after)
        self.state_out = None
        if pause_after > 0 or state is not None:
            nbytes = ctypes.c_size_t()
            _check(None, lib().symtd_solve_state_bytes(ctypes.byref(self.pb), ctypes.byref(o), int(trace_len),
                                                       ctypes.byref(nbytes)))
        if pause_after > 0:
            self.state_out = ctypes.create_string_buffer(nbytes.value)
            o.state_out = ctypes.cast(self.state_out, ctypes.c_void_p)
        if state is not None:
            # the library reads a whole state of this problem's size: refuse a shorter block here
            if len(state) != nbytes.value:
                raise SymtdError(-1, f"the saved state has {len(state)} bytes; a state of this problem and "
                                     f"these options has {nbytes.value}")
            self.state_in = ctypes.create_string_buffer(bytes(state), len(state))
            o.state_in = ctypes.cast(self.state_in, ctypes.c_void_p)
        self.opts = o
        self.A = colmajor(torch.empty(n, r, dtype=V.dtype, device=V.device))
        self.lam = torch.empty(r, dtype=torch.float64, device=V.device)
        Ap, lda = _mat(self.A, "A")
        self.fr = np.zeros(restarts)
        self.ir = np.zeros(restarts, dtype=np.int64)
        self.er = np.zeros(restarts, dtype=np.int64)
        self.xr = np.zeros(restarts, dtype=np.int32)
        self.trace_len = int(trace_len)
        self.tr = np.zeros((restarts, max(trace_len, 1)))
        res = SolveResult()
        res.A, res.lda, res.lam = Ap, lda, self.lam.data_ptr()
        res.f_restarts = self.fr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        res.iters_restarts = self.ir.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        res.evals_restarts = self.er.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        res.exit_restarts = self.xr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        res.f_trace = self.tr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if trace_len > 0 else None
        res.trace_len = self.trace_len
        self.res = res

    def result(self, res=None):
        res = self.res if res is None else res
        return {"A": self.A, "lam": self.lam, "f": res.f, "alpha": res.alpha, "rel_err": res.rel_err,
                "iters": res.iters, "evals": res.evals, "exit_reason": res.exit_reason,
                "best_restart": res.best_restart, "steps": res.steps, "f_restarts": self.fr,
                "iters_restarts": self.ir, "evals_restarts": self.er, "exit_restarts": self.xr,
                "f_trace": self.tr[:, :self.trace_len] if self.trace_len > 0 else None,
                "paused": self.state_out is not None and res.exit_reason == EXIT_RUNNING,
                "state": (self.state_out.raw if self.state_out is not None and res.exit_reason == EXIT_RUNNING
                          else None)}


def symtd_solve(ctx: Context, V, nu, d: int, r: int, *, prec: int | None = None, m: int = 5, pgtol: float = 1e-4,
                ftol: float = 2.220446049250313e-09, max_iters: int = 10000, max_evals: int = 50000,
                restarts: int = 1, seed: int = 0, init: int = INIT_RRF, alpha=None, A0=None,
                check_every: int = 0, trace_len: int = 0, sigma: float = 0.0, pause_after: int = 0,
                state: bytes | None = None, stream=None):
    """Restarted L-BFGS solve on the device (symtd_solve).

    alpha: None = compute ||X||^2 on the device, a positive number = use it,
    0 = shifted objective.  A0 (optional): n x (restarts*r) column-major
    device tensor of starts.  sigma > 0 (d = 3 or 4): fit the moment
    corrected for spherical Gaussian noise of that level; alpha then stands
    for ||X - Delta||^2.  pause_after > 0: stop after that many evaluation
    steps if a restart is still running; the dict then has paused = True and
    the solver's state as bytes under "state", which `state` takes to
    continue the same solve (same problem and options).  Returns a dict with
    the best model (A, lam as device tensors) and the host figures of the
    solve.
    """
    call = _SolveCall(V, nu, d, r, prec, m, pgtol, ftol, max_iters, max_evals, restarts, seed, init, alpha, A0,
                      check_every, trace_len, sigma, pause_after, state)
    _check(ctx, lib().symtd_solve(ctx.handle, _stream(stream), ctypes.byref(call.pb), ctypes.byref(call.opts),
                                  ctypes.byref(call.res)))
    return call.result()


def symtd_moment_stats(ctx: Context, V, nu, second: bool = True, stream=None):
    """m = sum_l nu_l v_l (n,) and, when `second`, M2 = sum_l nu_l v_l v_l'
    (n x n, column-major), fp64 device tensors."""
    import torch
    Vp, ldv = _mat(V, "V")
    n, p = V.shape
    m = torch.empty(n, dtype=torch.float64, device=V.device)
    M2 = colmajor(torch.empty(n, n, dtype=torch.float64, device=V.device)) if second else None
    _check(ctx, lib().symtd_moment_stats(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p,
                                         m.data_ptr(), M2.data_ptr() if second else None))
    return m, M2


def _m2(M2, n):
    """Device pointer of an n x n fp64 M2 stored densely (either order: M2 is symmetric)."""
    import torch
    if M2 is None:
        return None
    if not isinstance(M2, torch.Tensor) or tuple(M2.shape) != (n, n) or M2.dtype != torch.float64 or not M2.is_cuda:
        raise TypeError("M2 must be an n x n float64 GPU tensor")
    if not (M2.is_contiguous() or M2.t().is_contiguous()):
        raise ValueError("M2 must be stored densely")
    return M2.data_ptr()


def symtd_fg_corrected(ctx: Context, V, nu, A, lam, d: int, sigma: float, m, M2=None, alpha: float = 0.0,
                       prec: int | None = None, out=None, stream=None):
    """symtd_fg plus the correction for spherical Gaussian noise of level
    sigma (m, M2 from symtd_moment_stats; M2 needed for d = 4)."""
    import torch
    Vp, ldv = _mat(V, "V")
    Ap, lda = _mat(A, "A", V.dtype)
    n, p = V.shape
    if A.shape[0] != n:
        raise ValueError("A must have as many rows as V")
    r = A.shape[1]
    if prec is None:
        prec = PREC_FP64 if V.dtype == torch.float64 else PREC_FP32
    if out is None:
        f = torch.empty(1, dtype=torch.float64, device=V.device)
        g = torch.empty(r, dtype=torch.float64, device=V.device)
        G = colmajor(torch.empty(n, r, dtype=V.dtype, device=V.device))
    else:
        f, g, G = out
    Gp, ldg = _mat(G, "G_A", V.dtype)
    M2p = _m2(M2, n)
    _check(ctx, lib().symtd_fg_corrected(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p,
                                         Ap, lda, _vec(lam, "lambda", r), r, int(d), float(alpha), int(prec),
                                         float(sigma), _vec(m, "m", n), M2p, _vec(f, "f", 1),
                                         _vec(g, "g_lambda", r), Gp, ldg))
    return f, g, G


def symtd_alpha_corrected(ctx: Context, V, nu, d: int, sigma: float, m, M2, alpha: float, stream=None) -> float:
    """||X - Delta||^2 from alpha = ||X||^2 (a host float; synchronous)."""
    Vp, ldv = _mat(V, "V")
    n, p = V.shape
    out = ctypes.c_double(0.0)
    M2p = _m2(M2, n)
    _check(ctx, lib().symtd_alpha_corrected(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p,
                                            int(d), float(sigma), _vec(m, "m", n), M2p, float(alpha),
                                            ctypes.byref(out)))
    return out.value


def symtd_form_moment(ctx: Context, V, nu, d: int, out=None, stream=None):
    """The dense moment tensor X = sum_l nu_l v_l^{(x)d} as a flat device
    tensor of n^d entries (entry (i_1, .., i_d) at i_1 + n i_2 + ...)."""
    import torch
    Vp, ldv = _mat(V, "V")
    n, p = V.shape
    X = out if out is not None else torch.empty(n ** d, dtype=V.dtype, device=V.device)
    if X.dtype != V.dtype or X.numel() != n ** d or not X.is_contiguous():
        raise ValueError("out must be a contiguous tensor of n^d entries of V's dtype")
    _check(ctx, lib().symtd_form_moment(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p,
                                        int(d), X.data_ptr()))
    return X


def symtd_fg_explicit(ctx: Context, X, n: int, d: int, A, lam, alpha: float = 0.0, prec: int | None = None,
                      out=None, stream=None):
    """Algorithm 1 on a dense symmetric tensor X (flat, n^d entries)."""
    import torch
    Ap, lda = _mat(A, "A", X.dtype)
    r = A.shape[1]
    if A.shape[0] != n or X.numel() != n ** d or not X.is_contiguous() or not X.is_cuda:
        raise ValueError("X must be a contiguous GPU tensor of n^d entries and A n x r")
    if prec is None:
        prec = PREC_FP64 if X.dtype == torch.float64 else PREC_FP32
    if out is None:
        f = torch.empty(1, dtype=torch.float64, device=X.device)
        g = torch.empty(r, dtype=torch.float64, device=X.device)
        G = colmajor(torch.empty(n, r, dtype=X.dtype, device=X.device))
    else:
        f, g, G = out
    Gp, ldg = _mat(G, "G_A", X.dtype)
    _check(ctx, lib().symtd_fg_explicit(ctx.handle, _stream(stream), F64 if X.dtype == torch.float64 else F32,
                                        X.data_ptr(), n, int(d), Ap, lda, _vec(lam, "lambda", r), r, float(alpha),
                                        int(prec), _vec(f, "f", 1), _vec(g, "g_lambda", r), Gp, ldg))
    return f, g, G


def symtd_fg_sampled(ctx: Context, V, nu, A, lam, d: int, s: int, seed: int, draw: int, prec: int | None = None,
                     with_indices: bool = False, out=None, stream=None):
    """Shifted objective and gradient on draw `draw` of s sampled columns
    (Section 5, Lemma 5.1).  Returns (f, g_lambda, G_A[, indices])."""
    import torch
    Vp, ldv = _mat(V, "V")
    Ap, lda = _mat(A, "A", V.dtype)
    n, p = V.shape
    r = A.shape[1]
    if A.shape[0] != n:
        raise ValueError("A must have as many rows as V")
    if prec is None:
        prec = PREC_FP64 if V.dtype == torch.float64 else PREC_FP32
    if out is None:
        f = torch.empty(1, dtype=torch.float64, device=V.device)
        g = torch.empty(r, dtype=torch.float64, device=V.device)
        G = colmajor(torch.empty(n, r, dtype=V.dtype, device=V.device))
    else:
        f, g, G = out
    Gp, ldg = _mat(G, "G_A", V.dtype)
    idx = torch.empty(s, dtype=torch.int64, device=V.device) if with_indices else None
    st = lib().symtd_fg_sampled(ctx.handle, _stream(stream), _dt(V), Vp, ldv, _vec(nu, "nu", p), n, p, int(s),
                                int(seed), int(draw), Ap, lda, _vec(lam, "lambda", r), r, int(d), int(prec),
                                _vec(f, "f", 1), _vec(g, "g_lambda", r), Gp, ldg,
                                idx.data_ptr() if idx is not None else None)
    _check(ctx, st)
    return (f, g, G, idx) if with_indices else (f, g, G)


def symtd_solve_adam(ctx: Context, V, nu, d: int, r: int, *, samples: int = 100, est_samples: int = 1000,
                     epoch_len: int = 100, max_epochs: int = 1000, lr0: float = 0.01, lr1: float = 0.001,
                     beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, restarts: int = 1, seed: int = 0,
                     init: int = None, A0=None, prec: int | None = None, trace_len: int = 0, stream=None):
    """Adam on the sampled shifted objective with the paper's schedule
    (symtd_solve_adam).  Returns a dict like symtd_solve's; f is the shifted
    objective on the whole data set, f_trace the per-epoch estimates."""
    import numpy as np
    import torch
    Vp, ldv = _mat(V, "V")
    n, p = V.shape
    if prec is None:
        prec = PREC_FP64 if V.dtype == torch.float64 else PREC_FP32
    pb = Problem(_dt(V), Vp, ldv, _vec(nu, "nu", p), n, p, int(d), int(r))
    o = AdamOpts()
    _check(None, lib().symtd_adam_opts_default(ctypes.byref(o)))
    o.prec, o.samples, o.est_samples, o.epoch_len, o.max_epochs = int(prec), int(samples), int(est_samples), \
        int(epoch_len), int(max_epochs)
    o.lr0, o.lr1, o.beta1, o.beta2, o.eps = float(lr0), float(lr1), float(beta1), float(beta2), float(eps)
    o.restarts, o.seed = int(restarts), int(seed)
    o.init = INIT_RRF if init is None else int(init)
    keep = [V, nu]
    if A0 is not None:
        A0p, lda0 = _mat(A0, "A0", V.dtype)
        if tuple(A0.shape) != (n, restarts * r) or lda0 != n:
            raise ValueError("A0 must be an n x (restarts*r) column-major tensor with leading dimension n")
        o.A0 = A0p
        keep.append(A0)
    A = colmajor(torch.empty(n, r, dtype=V.dtype, device=V.device))
    lam = torch.empty(r, dtype=torch.float64, device=V.device)
    fr = np.zeros(restarts)
    ir = np.zeros(restarts, dtype=np.int64)
    er = np.zeros(restarts, dtype=np.int64)
    xr = np.zeros(restarts, dtype=np.int32)
    tr = np.zeros((restarts, max(trace_len, 1)))
    res = SolveResult()
    res.A, res.lda, res.lam = _mat(A, "A")[0], _mat(A, "A")[1], lam.data_ptr()
    res.f_restarts = fr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    res.iters_restarts = ir.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    res.evals_restarts = er.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    res.exit_restarts = xr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    res.f_trace = tr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if trace_len > 0 else None
    res.trace_len = int(trace_len)
    _check(ctx, lib().symtd_solve_adam(ctx.handle, _stream(stream), ctypes.byref(pb), ctypes.byref(o),
                                       ctypes.byref(res)))
    return {"A": A, "lam": lam, "f": res.f, "iters": res.iters, "epochs": res.evals, "exit_reason": res.exit_reason,
            "best_restart": res.best_restart, "f_restarts": fr, "steps_restarts": ir, "epochs_restarts": er,
            "exit_restarts": xr, "f_trace": tr[:, :trace_len] if trace_len > 0 else None}


def symtd_solve_batched(ctx: Context, problems, stream=None):
    """symtd_solve for every problem (dicts with V, nu, d, r and symtd_solve's
    keyword options), all on the grouped engine.  Returns one result dict per
    problem."""
    calls = [_SolveCall(**pr) for pr in problems]
    k = len(calls)
    pbs = (Problem * k)(*[c.pb for c in calls])
    opts = (SolveOpts * k)(*[c.opts for c in calls])
    outs = (SolveResult * k)(*[c.res for c in calls])
    _check(ctx, lib().symtd_solve_batched(ctx.handle, _stream(stream), k, pbs, opts, outs))
    return [c.result(outs[i]) for i, c in enumerate(calls)]


def symtd_fg_batched(ctx: Context, items, stream=None):
    """symtd_fg_multi for every item (dicts with V, nu, A, lam, r, d and
    optional alpha).  Returns [(f, g_lambda, G_A)] per item."""
    import torch
    arr = (FgItem * len(items))()
    outs = []
    dt = None
    for i, it in enumerate(items):
        V, nu, A, lam, r, d = it["V"], it["nu"], it["A"], it["lam"], int(it["r"]), int(it["d"])
        Vp, ldv = _mat(V, "V")
        Ap, lda = _mat(A, "A", V.dtype)
        n, p = V.shape
        cols = A.shape[1]
        if A.shape[0] != n or cols % r:
            raise ValueError("A must be n x (models r)")
        models = cols // r
        f = torch.empty(models, dtype=torch.float64, device=V.device)
        g = torch.empty(cols, dtype=torch.float64, device=V.device)
        G = colmajor(torch.empty(n, cols, dtype=V.dtype, device=V.device))
        Gp, ldg = _mat(G, "G_A")
        arr[i] = FgItem(Vp, ldv, _vec(nu, "nu", p), n, p, d, Ap, lda, _vec(lam, "lambda", cols), r, models,
                        float(it.get("alpha", 0.0)), f.data_ptr(), g.data_ptr(), Gp, ldg)
        outs.append((f, g, G))
        dt = _dt(V) if dt is None else dt
    prec = PREC_FP64 if dt == F64 else PREC_FP32
    _check(ctx, lib().symtd_fg_batched(ctx.handle, _stream(stream), dt, prec, len(items), arr))
    return outs


class Server:
    """A symtd server (symtd_server_*): continuous batching of solve requests.

    submit(V, nu, d, r, **symtd_solve options) -> request id; poll() returns
    finished results as dicts with host (numpy) A and lam.
    """

    def __init__(self, device: int = 0, dtype=None, memory_bytes: int = 8 << 30, check_every: int = 0,
                 use_graph: bool = True):
        import torch
        dtype = torch.float32 if dtype is None else dtype
        dt = F64 if dtype == torch.float64 else F32
        self.dtype = dtype
        o = ServerOpts(int(device), dt, PREC_FP64 if dt == F64 else PREC_FP32, int(memory_bytes),
                       int(check_every), int(bool(use_graph)))
        h = _vp()
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        st = lib().symtd_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != SYMTD_OK:
            raise SymtdError(st, "symtd_server_create failed")
        self._h = h

    def _err(self, st):
        if st != SYMTD_OK:
            msg = lib().symtd_server_last_error(self._h)
            raise SymtdError(st, msg.decode() if msg else "")

    def submit(self, V, nu, d: int, r: int, **opts) -> int:
        call = _SolveCall(V, nu, d, r, **opts)
        rid = ctypes.c_uint64()
        self._err(lib().symtd_server_submit(self._h, ctypes.byref(call.pb), ctypes.byref(call.opts),
                                            ctypes.byref(rid)))
        return int(rid.value)

    def poll(self, max_results: int = 64, timeout_ms: int = 0):
        import numpy as np
        buf = (ServerResult * max_results)()
        n = ctypes.c_int32()
        self._err(lib().symtd_server_poll(self._h, buf, int(max_results), ctypes.byref(n), int(timeout_ms)))
        out = []
        for i in range(n.value):
            rres = buf[i]
            d = {k: getattr(rres, k) for k in ("id", "status", "f", "alpha", "rel_err", "iters", "evals",
                                                 "exit_reason", "best_restart", "n", "r", "t_submit", "t_admit",
                                                 "t_done")}
            if rres.status == SYMTD_OK:
                nn, rr = rres.n, rres.r
                d["A"] = np.ctypeslib.as_array(rres.A, shape=(nn * rr,)).reshape(rr, nn).T.copy()
                d["lam"] = np.ctypeslib.as_array(rres.lam, shape=(rr,)).copy()
            lib().symtd_server_result_release(ctypes.byref(buf[i]))
            out.append(d)
        return out

    def cancel(self, rid: int):
        self._err(lib().symtd_server_cancel(self._h, ctypes.c_uint64(rid)))

    def stats(self):
        s = ServerStats()
        self._err(lib().symtd_server_stats_get(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().symtd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Data:
    """A prepared data set (symtd_data_create): V, nu and the product precision.

    fg(A, lam, d, alpha) evaluates f, g_lambda, G_A on it (symtd_fg_data).
    The tensors V and nu are kept referenced while the handle lives.
    """

    def __init__(self, ctx: Context, V, nu, prec: int, stream=None):
        Vp, ldv = _mat(V, "V")
        n, p = V.shape
        nup = _vec(nu, "nu", p)
        h = _vp()
        _check(ctx, lib().symtd_data_create(ctx.handle, _stream(stream), _dt(V), Vp, ldv, nup, n, p, int(prec),
                                            ctypes.byref(h)))
        self._h = h
        self.ctx, self.V, self.nu, self.prec, self.n, self.p = ctx, V, nu, prec, n, p

    def fg(self, A, lam, d: int, alpha: float = 0.0, out=None, stream=None):
        import torch
        Ap, lda = _mat(A, "A", self.V.dtype)
        n2, r = A.shape
        if n2 != self.n:
            raise ValueError("A must have as many rows as V")
        lp = _vec(lam, "lambda", r)
        if out is None:
            f = torch.empty(1, dtype=torch.float64, device=A.device)
            g = torch.empty(r, dtype=torch.float64, device=A.device)
            G = colmajor(torch.empty(self.n, r, dtype=A.dtype, device=A.device))
        else:
            f, g, G = out
        Gp, ldg = _mat(G, "G_A", self.V.dtype)
        _check(self.ctx, lib().symtd_fg_data(self.ctx.handle, _stream(stream), self._h, Ap, lda, lp, r, int(d),
                                             float(alpha), _vec(f, "f", 1), _vec(g, "g_lambda", r), Gp, ldg))
        return f, g, G

    def close(self):
        if getattr(self, "_h", None):
            lib().symtd_data_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


TUNE_G1_BLOCKS, TUNE_G2_SPLITS, TUNE_GRAPH, TUNE_SPIN_LIMIT, TUNE_FAULT_HANDOFF = 0, 1, 3, 4, 5


def symtd_check(ctx: Context, stream=None):
    """Wait for the stream; raise SymtdError (EDEVICE) if a call on this
    context recorded a device-side error (the record is then cleared)."""
    _check(ctx, lib().symtd_check(ctx.handle, _stream(stream)))


def symtd_set_tuning(ctx: Context, key: int, value: int):
    """Override a work-split choice of the evaluation kernels (0 = automatic)."""
    _check(ctx, lib().symtd_set_tuning(ctx.handle, int(key), int(value)))


def symtd_profile_enable(ctx: Context, enable: bool = True, kernels=None):
    """Time every launch of the named kernels (profile_names(); all when
    kernels is None) while enabled; off when enable is false."""
    if not enable:
        mask = 0
    elif kernels is None:
        mask = 0xFFFFFFFF
    else:
        names = profile_names()
        mask = 0
        for k in kernels:
            mask |= 1 << names.index(k)
    _check(ctx, lib().symtd_profile_enable(ctx.handle, mask))


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


from . import metrics  # noqa: E402,F401  (host-side quality measures of solve results)
