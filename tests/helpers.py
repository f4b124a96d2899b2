"""Shared helpers of the GPU parity tests (not collected as tests)."""

import numpy as np

import synth
from oracle.fg import fg_implicit, magnitudes

# Tolerances relative to the magnitudes of the cancelling terms (see
# oracle.fg.Magnitudes): fp64 products 1e-12, fp32 products 1e-5.
TOL = {"f64": 1e-12, "f32": 1e-5}


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def to_dev(x, dtype):
    """Column-major device copy of a numpy matrix, or a device vector."""
    import torch
    from paper_1911_03813_amd import colmajor
    t = torch.from_numpy(np.ascontiguousarray(x)).to(dtype)
    if t.dim() == 2:
        t = colmajor(t)
    return t.cuda()


def stored(x, kind):
    """The values a kind ("f32"/"f64") of storage holds, as fp64 numpy."""
    x = np.asarray(x, dtype=np.float64)
    return x.astype(np.float32).astype(np.float64) if kind == "f32" else x


def make_case(n, p, r, d, key, sigma=1e-2, kind="f64"):
    V, nu, _ = synth.gmm(n, max(1, min(r, p)), p, sigma, *key)
    A = synth.gauss_factors(n, r, *key, 5)
    lam = synth.rng(*key, 6).standard_normal(r)
    return stored(V, kind), nu, stored(A, kind), lam


def compare_fg(got, V, nu, A, lam, d, alpha, kind):
    """Element-by-element comparison with the oracle; returns the normalised
    errors (each must be <= TOL[kind])."""
    f, g, G = got
    ref = fg_implicit(V, nu, A, lam, d, alpha)
    mag = magnitudes(V, nu, A, lam, d, alpha)
    ef = abs(float(f) - ref.f) / mag.f_scale
    eg = np.max(np.abs(g - ref.g_lambda) / mag.g_scale)
    eG = np.max(np.abs(G - ref.G_A) / mag.G_scale[None, :])
    return ef, eg, eG
