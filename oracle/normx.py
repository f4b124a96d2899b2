"""The constant term ||X||^2 of the objective.

Applying Lemma 3.4 to X = sum_l nu_l v_l^{(x)d} itself gives
||X||^2 = nu' [V'V]^d nu (elementwise power), an O(n p^2) computation
(Section 3.3).  ``normx_implicit`` is that expression, evaluated over row
blocks of the p x p Gram matrix so that the whole matrix is never held.
``normx_explicit`` is the plain definition sum_i x_i^2 on an explicit X.
"""

from __future__ import annotations

import numpy as np

from . import tensor as T


def normx_implicit(V, nu, d: int, block: int = 2048) -> float:
    V = np.asarray(V, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    p = V.shape[1]
    total = 0.0
    for s in range(0, p, block):
        e = min(p, s + block)
        G = V[:, s:e].T @ V                      # rows s..e of V'V
        total += nu[s:e] @ (G ** d) @ nu
    return float(total)


def normx_explicit(V, nu, d: int) -> float:
    X = T.kruskal(np.asarray(nu, dtype=np.float64), np.asarray(V, dtype=np.float64), d)
    return float(T.inner(X, X))
