"""CPU model of the roundings of the 16-bit product paths (test helper).

The fp16 and bf16x3 paths store V, A and W = D_nu Z^{d-1} in 16 bits and
accumulate the products in fp32.  Their error bound in the parity tests is
set per shape from this model: the paths' operand roundings are applied
exactly (numpy, bit-level round-to-nearest-even), and everything else is
computed in fp64 along Algorithm 2, so that the model's error against the
fp64 oracle is the error the 16-bit storage alone causes.  The model is
evaluated for the path as built and for two broken variants that a parity
test must be able to tell from it:

* ``bf16``         one bf16 plane per operand (no hi/lo split);
* ``fp16_noscale`` fp16 with W stored unscaled (W = nu z^{d-1} falls below
  fp16's normal range when nu = 1/p is small).

This module is test infrastructure: it shares no code with the HIP library
and uses nothing from ``oracle`` but its comparison scales.
"""

from __future__ import annotations

import numpy as np

MODES = ("bf16x3", "bf16", "fp16", "fp16_noscale")


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as fp64.  The
    argument is first rounded to fp32, as the device holds it."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def fp16(x) -> np.ndarray:
    """Round to IEEE binary16 (nearest even, subnormals kept), as fp64."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _split(x):
    """hi = bf16(x), lo = bf16(x - hi) with the difference taken in fp32
    (exact: it has at most 16 significant bits)."""
    x32 = np.asarray(x, dtype=np.float32)
    hi = bf16(x32)
    lo = bf16(x32 - hi.astype(np.float32))
    return hi, lo


def wscale_of(nu) -> float:
    """The fp16 path's power of two 2^s with 2^s max|nu| in [1, 2)."""
    return float(2.0 ** (-np.floor(np.log2(np.max(np.abs(nu))))))


def emulate(V, nu, A, lam, d: int, alpha: float, mode: str):
    """(f, g_lambda, G_A) of Algorithm 2 with the operand roundings of `mode`.

    V and A are the stored fp32 values (as fp64).  B = A'A and C come from
    the fp32 A in fp64, as on the device; w = sum_l W_lj z_lj with W the fp32
    value before its 16-bit rounding; the second product uses the rounded W.
    """
    if mode not in MODES:
        raise ValueError(mode)
    V = np.asarray(V, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    if mode == "bf16x3":
        Vh, Vl = _split(V)
        Ah, Al = _split(A)
        Z = Vh.T @ Ah + (Vh.T @ Al + Vl.T @ Ah)
    elif mode == "bf16":
        Vh, Ah = bf16(V), bf16(A)
        Z = Vh.T @ Ah
    else:
        Vh, Ah = fp16(V), fp16(A)
        Z = Vh.T @ Ah
    Z = f32(Z)
    W32 = f32(nu[:, None] * Z ** (d - 1))
    w = np.sum(W32 * Z, axis=0)
    if mode == "bf16x3":
        Wh, Wl = _split(W32)
        Y = Vh @ Wh + (Vh @ Wl + Vl @ Wh)
    elif mode == "bf16":
        Y = Vh @ bf16(W32)
    else:
        s = wscale_of(nu) if mode == "fp16" else 1.0
        Y = (Vh @ fp16(s * W32)) / s
    B = A.T @ A
    C = B ** (d - 1)
    u = (B * C) @ lam
    f = alpha + lam @ u - 2.0 * (w @ lam)
    g = -2.0 * (w - u)
    G = -2.0 * d * (Y - A @ (lam[:, None] * C)) * lam[None, :]
    return float(f), g, G


def model_errors(V, nu, A, lam, d, alpha, mode, ref, mag):
    """Normalised errors (e_f, e_g, e_G) of the model against the oracle
    result `ref` with comparison scales `mag` (oracle.fg.magnitudes)."""
    f, g, G = emulate(V, nu, A, lam, d, alpha, mode)
    ef = abs(f - ref.f) / mag.f_scale
    eg = float(np.max(np.abs(g - ref.g_lambda) / mag.g_scale))
    eG = float(np.max(np.abs(G - ref.G_A) / mag.G_scale[None, :]))
    return np.array([ef, eg, eG])


# The stated bounds of the two paths, per quantity (f, g_lambda, G_A):
#   bf16x3: SPLIT_FRACTION of the single-plane bf16 model's error.  The split
#           operand carries 16 significant bits instead of 8, so a correct
#           path removes more than 99% of the single-plane error; the bound
#           asks for 90%, which leaves room for the fp32 accumulation.
#   fp16:   FP16_FACTOR times the model of the path itself; fp32
#           accumulation adds well under that on top of fp16's 2^-11
#           rounding.
# Each is also at least FLOOR, the fp32-product accumulation level of these
# shapes, so that a quantity the 16-bit rounding happens to leave almost
# untouched is not held to a bar below fp32 arithmetic.
SPLIT_FRACTION = 0.1
FP16_FACTOR = 4.0
FLOOR = 1e-7


def bounds(V, nu, A, lam, d, alpha, kind, ref, mag):
    """Per-quantity bounds (f, g_lambda, G_A) for kind "bf16x3" or "fp16",
    and the model errors they were derived from."""
    if kind == "bf16x3":
        e_plain = model_errors(V, nu, A, lam, d, alpha, "bf16", ref, mag)
        return np.maximum(SPLIT_FRACTION * e_plain, FLOOR), e_plain
    e_path = model_errors(V, nu, A, lam, d, alpha, "fp16", ref, mag)
    return np.maximum(FP16_FACTOR * e_path, FLOOR), e_path
