"""Explicit dense d-way tensors (Section 2 of the paper), for brute force.

Only for tiny sizes: an n^d array is formed in memory.  Nothing here uses
the implicit identities of Section 3; these are the plain definitions.
"""

from __future__ import annotations

import numpy as np


def outer_power(a: np.ndarray, d: int) -> np.ndarray:
    """a^{(x)d}: the d-way outer product of a with itself, eq. (outer_product)."""
    t = np.asarray(a)
    out = t
    for _ in range(d - 1):
        out = np.multiply.outer(out, t)
    return out


def inner(x: np.ndarray, y: np.ndarray):
    """<X, Y> = sum over all multi-indices of x_i y_i, eq. (tensorIP)."""
    return np.sum(x * y)


def kruskal(weights: np.ndarray, factors: np.ndarray, d: int) -> np.ndarray:
    """sum_j weights_j * a_j^{(x)d} for the columns a_j of factors,
    eq. (cp_element) for the model M and eq. (tensorX) for the data X."""
    n, r = factors.shape
    dtype = np.result_type(weights, factors)
    out = np.zeros((n,) * d, dtype=dtype)
    for j in range(r):
        out = out + weights[j] * outer_power(factors[:, j], d)
    return out


def ttsv_all_but_one(x: np.ndarray, a: np.ndarray) -> np.ndarray:
    """X a^{d-1}: contract every mode but the first with a, eq. (ExpXbdd)."""
    t = x
    while t.ndim > 1:
        t = np.tensordot(t, a, axes=([t.ndim - 1], [0]))
    return t


def ttsv_all(x: np.ndarray, a: np.ndarray):
    """X a^d: contract every mode with a, eq. (ExpXbd)."""
    return ttsv_all_but_one(x, a) @ a
