"""Starting points and the restarted solve (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Starts (Section 4.2): lambda_0 = 1 and either
  * GAUSS: A_0 ~ N(0, 1)^{n x r} with columns normalised to unit length, or
  * RRF: A_0 = V Omega with Omega ~ N(0, 1)^{p x r} (the randomized range
    finder, eq. (rrf)), columns normalised to unit length.
The normals are those of ``oracle.philox`` for (seed, restart).

The solve minimises phi(x) = f(x) / s over x = [lambda; vec(A)] (A
column-major) with s = alpha = ||X||^2 when alpha is known (so that the
tolerances are relative to the size of the data tensor) and s = 1 otherwise,
using ``oracle.lbfgs``.  Every restart runs independently from its own start;
the best is the one with the lowest final f, the lowest restart index on ties
(Section 4.2 keeps the best of ten runs by final f).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .fg import fg_implicit
from .lbfgs import lbfgs
from .philox import STREAM_GAUSS_A0, STREAM_RRF_OMEGA, gaussian_matrix

INIT_GAUSS, INIT_RRF = 0, 1


def start(V, r, kind, seed, restart):
    """(lambda_0, A_0) of one restart."""
    n, p = V.shape
    if kind == INIT_GAUSS:
        A = gaussian_matrix(n, r, seed, restart, STREAM_GAUSS_A0)
    elif kind == INIT_RRF:
        A = V @ gaussian_matrix(p, r, seed, restart, STREAM_RRF_OMEGA)
    else:
        raise ValueError("unknown start kind")
    A = A / np.linalg.norm(A, axis=0)
    return np.ones(r), A


def pack(lam, A):
    return np.concatenate([np.asarray(lam, dtype=np.float64), np.asarray(A, dtype=np.float64).reshape(-1, order="F")])


def unpack(x, n, r):
    return x[:r].copy(), x[r:].reshape((n, r), order="F").copy()


def objective(V, nu, d, r, alpha):
    """x -> (f/s, grad/s) with s = alpha if alpha > 0 else 1; f includes alpha."""
    n = V.shape[0]
    s = alpha if alpha > 0 else 1.0

    def fun(x):
        lam, A = unpack(x, n, r)
        o = fg_implicit(V, nu, A, lam, d, alpha, with_intermediates=False)
        g = np.concatenate([o.g_lambda, o.G_A.reshape(-1, order="F")])
        return o.f / s, g / s
    return fun


@dataclass
class SolveResult:
    lam: np.ndarray
    A: np.ndarray
    f: float                 # final f of the best restart (unscaled, alpha included)
    best: int
    f_restarts: list         # final f of every restart
    runs: list               # oracle.lbfgs.LbResult of every restart (scaled values)
    alpha: float
    scale: float


def solve(V, nu, d, r, alpha=0.0, restarts=1, init=INIT_RRF, seed=0, m=5, pgtol=1e-4,
          ftol=2.220446049250313e-09, max_iters=10000, max_evals=50000, starts=None):
    """Restarted L-BFGS solve; `starts` may give the (lambda_0, A_0) of each restart."""
    n = V.shape[0]
    s = alpha if alpha > 0 else 1.0
    fun = objective(V, nu, d, r, alpha)
    runs = []
    for k in range(restarts):
        lam0, A0 = starts[k] if starts is not None else start(V, r, init, seed, k)
        runs.append(lbfgs(fun, pack(lam0, A0), m=m, pgtol=pgtol, ftol=ftol, max_iters=max_iters,
                          max_evals=max_evals))
    fs = [run.f * s for run in runs]
    best = int(np.argmin(fs))
    lam, A = unpack(runs[best].x, n, r)
    return SolveResult(lam, A, fs[best], best, fs, runs, alpha, s)
