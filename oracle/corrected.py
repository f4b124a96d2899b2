"""Moments corrected for spherical Gaussian noise (the lower-order terms the
paper points to in Section 4.2 and leaves to future work, Section 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For v = mu + sigma g with g ~ N(0, I), the odd moments of g vanish and
E[g g'] = I, E[g^{(x)4}] = sym3(I (x) I) (Isserlis), so

  d = 3:  E[v^{(x)3}] = E[mu^{(x)3}] + sigma^2 sym3(E[mu] (x) I)
  d = 4:  E[v^{(x)4}] = E[mu^{(x)4}] + sigma^2 sym6(E[mu mu'] (x) I)
                        + sigma^4 sym3(I (x) I)

where symK sums the K distinct placements of the factors over the d index
positions (sym3(m (x) I)_{ijk} = m_i d_jk + m_j d_ik + m_k d_ij, and so on).
With the data's own statistics m = sum_l nu_l v_l and M2 = sum_l nu_l v_l
v_l' (so that E[mu mu'] is estimated by S = M2 - sigma^2 I), the correction
tensor is

  Delta = sigma^2 sym3(m (x) I)                                  (d = 3)
  Delta = sigma^2 sym6(S (x) I) + sigma^4 sym3(I (x) I)          (d = 4)

and the corrected data tensor X_c = X - Delta estimates the noiseless
moment sum_j w_j mu_j^{(x)d}.  The corrected objective is

  f_c = ||X_c - M||^2 = f + 2 <M, Delta> + (||Delta||^2 - 2 <X, Delta>),

with <M, Delta> = sum_j lambda_j Delta a_j^d.  Contractions used (t = a'a):

  d = 3:  Delta a^3 = 3 sigma^2 (m'a) t
          Delta a^2 = sigma^2 (t m + 2 (m'a) a)
  d = 4:  Delta a^4 = 6 sigma^2 (a'Sa) t + 3 sigma^4 t^2
          Delta a^3 = 3 sigma^2 (t S a + (a'Sa) a) + 3 sigma^4 t a

and the constants ||Delta||^2 = sigma^4 ||m||^2 (3n + 6) for d = 3 and, for
d = 4, sigma^4 (6 (n + 4) ||S||_F^2 + 6 (tr S)^2) + 12 sigma^6 (n + 2) tr S
+ sigma^8 (3 n^2 + 6 n); <X, Delta> = sum_l nu_l Delta v_l^d.
"""

from __future__ import annotations

import itertools

import numpy as np

from .fg import FG, fg_implicit
from . import tensor as T


def stats(V, nu):
    """m = sum nu_l v_l and M2 = sum nu_l v_l v_l' (fp64)."""
    V = np.asarray(V, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return V @ nu, (V * nu) @ V.T


def delta_tensor(m, M2, sigma: float, d: int) -> np.ndarray:
    """Delta as an explicit n^d array, from the placements one by one."""
    n = len(m)
    eye = np.eye(n)
    out = np.zeros((n,) * d)
    if d == 3:
        for pos in range(3):
            # m on index `pos`, the identity on the other two
            t = np.einsum("i,jk->ijk", m, eye)
            out += np.moveaxis(t, 0, pos)
        return sigma ** 2 * out
    if d == 4:
        S = M2 - sigma ** 2 * eye
        base = np.einsum("ij,kl->ijkl", S, eye)
        for pair in itertools.combinations(range(4), 2):
            rest = [q for q in range(4) if q not in pair]
            out += np.transpose(base, np.argsort(list(pair) + rest))
        q4 = np.zeros((n,) * 4)
        ii = np.einsum("ij,kl->ijkl", eye, eye)
        for perm in ((0, 1, 2, 3), (0, 2, 1, 3), (0, 3, 1, 2)):
            q4 += np.transpose(ii, np.argsort(perm))
        return sigma ** 2 * out + sigma ** 4 * q4
    raise ValueError("corrections are derived for d = 3 and d = 4")


def delta_contractions(A, m, M2, sigma: float, d: int):
    """(Delta a_j^d for every column, Delta a_j^{d-1} as the columns of an n x r array)."""
    A = np.asarray(A, dtype=np.float64)
    t = np.sum(A * A, axis=0)
    s2 = sigma ** 2
    if d == 3:
        u = m @ A
        return 3.0 * s2 * u * t, s2 * (np.outer(m, t) + 2.0 * A * u)
    if d == 4:
        S = M2 - s2 * np.eye(len(m))
        SA = S @ A
        q = np.sum(A * SA, axis=0)
        full = 6.0 * s2 * q * t + 3.0 * s2 * s2 * t * t
        part = 3.0 * s2 * (SA * t + A * q) + 3.0 * s2 * s2 * A * t
        return full, part
    raise ValueError("corrections are derived for d = 3 and d = 4")


def delta_norm2(m, M2, sigma: float, d: int) -> float:
    """||Delta||^2 in closed form."""
    n = len(m)
    s2 = sigma ** 2
    if d == 3:
        return s2 * s2 * float(m @ m) * (3 * n + 6)
    S = M2 - s2 * np.eye(n)
    fro = float(np.sum(S * S))
    tr = float(np.trace(S))
    return (s2 ** 2 * (6 * (n + 4) * fro + 6 * tr * tr) + 12 * s2 ** 3 * (n + 2) * tr + s2 ** 4 * (3 * n * n + 6 * n))


def x_dot_delta(V, nu, m, M2, sigma: float, d: int) -> float:
    """<X, Delta> = sum_l nu_l Delta v_l^d."""
    full, _ = delta_contractions(V, m, M2, sigma, d)
    return float(np.asarray(nu, dtype=np.float64) @ full)


def fg_corrected(V, nu, A, lam, d: int, sigma: float, alpha: float = 0.0, m=None, M2=None) -> FG:
    """Corrected objective f + 2 sum_j lambda_j Delta a_j^d (+ alpha) and its
    gradient; with alpha = ||X||^2 - 2 <X, Delta> + ||Delta||^2 it is
    ||X - Delta - M||^2 itself."""
    if m is None:
        m, M2 = stats(V, nu)
    base = fg_implicit(V, nu, A, lam, d, alpha)
    lam = np.asarray(lam, dtype=np.float64)
    full, part = delta_contractions(A, m, M2, sigma, d)
    f = base.f + 2.0 * float(lam @ full)
    g = base.g_lambda + 2.0 * full
    G = base.G_A + 2.0 * d * part * lam[None, :]
    return FG(f, g, G)


def alpha_corrected(V, nu, d: int, sigma: float, alpha: float, m=None, M2=None) -> float:
    """||X - Delta||^2 from ||X||^2 = alpha."""
    if m is None:
        m, M2 = stats(V, nu)
    return alpha - 2.0 * x_dot_delta(V, nu, m, M2, sigma, d) + delta_norm2(m, M2, sigma, d)


def gaussian_moment(mu, sigma: float, d: int, points: int = 3) -> np.ndarray:
    """E[(mu + sigma g)^{(x)d}] for g ~ N(0, I) by tensor-product Gauss-Hermite
    quadrature (probabilists' weights), exact for d <= 2 points - 1."""
    x, w = np.polynomial.hermite_e.hermegauss(points)
    w = w / w.sum()
    n = len(mu)
    out = np.zeros((n,) * d)
    for idx in itertools.product(range(points), repeat=n):
        g = x[list(idx)]
        out += np.prod(w[list(idx)]) * T.outer_power(mu + sigma * g, d)
    return out
