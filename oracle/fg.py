"""Objective f(lambda, A) = ||X - M||^2 and its gradient (paper Sections 2-3).

Two independent fp64 routes:

* ``fg_bruteforce`` forms X = sum_l nu_l v_l^{(x)d} (eq. (tensorX)) and
  M = sum_j lambda_j a_j^{(x)d} (eq. (cp_element)) as explicit n^d arrays
  and differentiates ||X - M||^2 directly.  Tiny sizes only.
* ``fg_implicit`` is Algorithm 2 (fg_implicit): the TTSVs of X come from
  eq. (Y), Y = V D_nu [V'A]^{d-1}, and the model terms from Lemma 3.4,
  so X is never formed.

``grad_paper_explicit`` evaluates the gradient exactly as printed in
eqs. (gradl) and (gradb), on an explicit X, as a third witness.

All three accept complex A (transposes, never conjugates), so that the
complex-step derivative Im f(A + i h E) / h can pin the gradient.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import tensor as T


@dataclass
class FG:
    f: complex | float
    g_lambda: np.ndarray
    G_A: np.ndarray
    # intermediates of Algorithm 2, kept for diagnostics and tolerances
    Y: np.ndarray | None = None
    w: np.ndarray | None = None
    u: np.ndarray | None = None
    C: np.ndarray | None = None


def fg_implicit(V, nu, A, lam, d: int, alpha: float = 0.0, with_intermediates: bool = True) -> FG:
    """Algorithm 2 of the paper, step by step, in fp64 (or complex128).

    V: n x p observations (columns), nu: p weights, A: n x r factors,
    lam: r weights, d: tensor order, alpha: the constant ||X||^2 term
    (0 gives the "shifted" objective used in Section 5).
    """
    V = np.asarray(V, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    A = np.asarray(A)
    lam = np.asarray(lam)
    if not np.iscomplexobj(A):
        A = A.astype(np.float64)
    # line 2, eq. (Y): all r TTSVs X a_j^{d-1} at once (Lemma 3.3)
    Z = V.T @ A                                   # p x r inner products <v_l, a_j>
    Y = V @ (nu[:, None] * Z ** (d - 1))          # n x r
    # line 3: w_j = a_j' y_j  (= X a_j^d, so <X, M> = w' lambda by Lemma 3.5)
    w = np.sum(A * Y, axis=0)
    # lines 4-6: B = A'A, C = B^{d-1} (elementwise), u = (B * C) lambda
    B = A.T @ A
    C = B ** (d - 1)
    u = (B * C) @ lam
    # line 7: f = alpha + lambda' u - 2 w' lambda  (||M||^2 = lambda' u by Lemma 3.4)
    f = alpha + lam @ u - 2.0 * (w @ lam)
    # line 8
    g_lambda = -2.0 * (w - u)
    # line 9: G_A = -2 d (Y - A D_lambda C) D_lambda
    G_A = -2.0 * d * (Y - A @ (lam[:, None] * C)) * lam[None, :]
    if not with_intermediates:
        return FG(f, g_lambda, G_A)
    return FG(f, g_lambda, G_A, Y=Y, w=w, u=u, C=C)


def fg_bruteforce(V, nu, A, lam, d: int, alpha: float | None = None) -> FG:
    """f = ||X - M||^2 and its exact derivatives from explicit tensors.

    With R = X - M (explicit), f = <R, R> (eq. (optFunc)); differentiating
    <R, R> gives df/dlambda_j = -2 <R, a_j^{(x)d}> and, by the symmetry of R,
    df/da_j = -2 d lambda_j R a_j^{d-1}.  If alpha is given, f is shifted so
    that its constant term equals alpha instead of ||X||^2.
    """
    A = np.asarray(A)
    lam = np.asarray(lam)
    X = T.kruskal(np.asarray(nu, dtype=np.float64), np.asarray(V, dtype=np.float64), d)
    M = T.kruskal(lam, A, d)
    R = X - M
    f = T.inner(R, R)
    if alpha is not None:
        f = f - T.inner(X, X) + alpha
    r = A.shape[1]
    g = np.array([-2.0 * T.inner(R, T.outer_power(A[:, j], d)) for j in range(r)])
    G = np.stack([-2.0 * d * lam[j] * T.ttsv_all_but_one(R, A[:, j]) for j in range(r)], axis=1)
    return FG(f, g, G)


def grad_paper_explicit(V, nu, A, lam, d: int):
    """Gradient exactly as printed in eqs. (gradl) and (gradb), with the
    TTSVs X a_j^d and X a_j^{d-1} taken on an explicit X (eqs. (ExpXbd),
    (ExpXbdd))."""
    A = np.asarray(A)
    X = T.kruskal(np.asarray(nu, dtype=np.float64), np.asarray(V, dtype=np.float64), d)
    r = A.shape[1]
    g = np.empty(r, dtype=np.result_type(A, lam))
    G = np.empty(A.shape, dtype=np.result_type(A, lam))
    for j in range(r):
        aj = A[:, j]
        dots = A.T @ aj                                   # <a_j, a_k>
        g[j] = -2.0 * (T.ttsv_all(X, aj) - np.sum(lam * dots ** d))
        G[:, j] = -2.0 * d * lam[j] * (T.ttsv_all_but_one(X, aj) - A @ (lam * dots ** (d - 1)))
    return g, G


def fg_explicit(X, A, lam, d: int, alpha: float = 0.0) -> FG:
    """Algorithm 1 (fg_explicit) on a given dense symmetric X (n^d entries):
    the TTSVs y_j = X a_j^{d-1} by eq. (ExpXbdd), w_j = a_j' y_j, then the
    same closing lines as Algorithm 2."""
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    r = A.shape[1]
    Y = np.stack([T.ttsv_all_but_one(X, A[:, j]) for j in range(r)], axis=1)
    w = np.sum(A * Y, axis=0)
    B = A.T @ A
    C = B ** (d - 1)
    u = (B * C) @ lam
    f = alpha + lam @ u - 2.0 * (w @ lam)
    g_lambda = -2.0 * (w - u)
    G_A = -2.0 * d * (Y - A @ (lam[:, None] * C)) * lam[None, :]
    return FG(f, g_lambda, G_A, Y=Y, w=w, u=u, C=C)


@dataclass
class Magnitudes:
    """Sizes of the terms that cancel in f, g_lambda and G_A.

    A rounding error of relative size eps in every product and sum gives an
    error of order eps times these magnitudes, so tolerances are stated
    relative to them:

    f_scale       = |alpha| + |lambda' u| + 2 |w' lambda|
    g_scale[j]    = 2 (sum_l |nu_l| |z_lj|^d + sum_k |B_jk|^d |lambda_k|)
    G_scale[j]    = 2 d |lambda_j| (max_i Yabs_ij + max_i (|A| D_|lambda| |C|)_ij)

    with Yabs = |V| D_|nu| |Z|^{d-1}.  G_scale is per column, so the
    element-wise comparison |dG_ij| <= tol * G_scale[j] is invariant to the
    scaling gauge of column j.
    """
    f_scale: float
    g_scale: np.ndarray
    G_scale: np.ndarray


def magnitudes(V, nu, A, lam, d: int, alpha: float = 0.0) -> Magnitudes:
    V = np.asarray(V, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    out = fg_implicit(V, nu, A, lam, d, alpha)
    Z = np.abs(V.T @ A)
    Yabs = np.abs(V) @ (np.abs(nu)[:, None] * Z ** (d - 1))
    wabs = np.abs(nu) @ Z ** d
    Babs = np.abs(A.T @ A)
    uabs = Babs ** d @ np.abs(lam)
    f_scale = abs(alpha) + abs(lam @ out.u) + 2.0 * abs(out.w @ lam)
    g_scale = 2.0 * (wabs + uabs)
    ADC = np.abs(A) @ (np.abs(lam)[:, None] * np.abs(out.C))
    G_scale = 2.0 * d * np.abs(lam) * (Yabs.max(axis=0) + ADC.max(axis=0))
    return Magnitudes(float(f_scale), g_scale, G_scale)


def magnitudes_explicit(X, A, lam, d: int, alpha: float = 0.0) -> Magnitudes:
    """The scales of Magnitudes for Algorithm 1, whose TTSVs sum the terms
    X_{i i_2 .. i_d} a_{i_2} .. a_{i_d} of eq. (ExpXbdd): Yabs = |X| |a|^{d-1}
    and the w terms |X| |a|^d replace their implicit counterparts."""
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    out = fg_explicit(X, A, lam, d, alpha)
    Xa = np.abs(X)
    Aa = np.abs(A)
    r = A.shape[1]
    Yabs = np.stack([T.ttsv_all_but_one(Xa, Aa[:, j]) for j in range(r)], axis=1)
    wabs = np.sum(Aa * Yabs, axis=0)
    Babs = np.abs(A.T @ A)
    uabs = Babs ** d @ np.abs(lam)
    f_scale = abs(alpha) + abs(lam @ out.u) + 2.0 * abs(out.w @ lam)
    g_scale = 2.0 * (wabs + uabs)
    ADC = Aa @ (np.abs(lam)[:, None] * np.abs(out.C))
    G_scale = 2.0 * d * np.abs(lam) * (Yabs.max(axis=0) + ADC.max(axis=0))
    return Magnitudes(float(f_scale), g_scale, G_scale)
