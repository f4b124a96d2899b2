"""Quality metrics of a decomposition (paper Section 4.2).

* relative error ||X - M|| / ||X||, computed implicitly from the full
  objective f = ||X - M||^2 and alpha = ||X||^2;
* the similarity score of eq. (Score): the best one-to-one matching of
  |cosine| between true and recovered means, averaged over the smaller set;
* a gauge-invariant distance between two symmetric Kruskal models, from
  Lemma 3.1 as used in Lemma 3.4:
  ||M1 - M2||^2 = l1'[A1'A1]^d l1 - 2 l1'[A1'A2]^d l2 + l2'[A2'A2]^d l2.
"""

from __future__ import annotations

import itertools

import numpy as np


def rel_err(f: float, alpha: float) -> float:
    """sqrt(max(f, 0) / alpha); rounding can push f slightly below 0."""
    return float(np.sqrt(max(float(f), 0.0) / float(alpha)))


def _unit_cols(a):
    a = np.asarray(a, dtype=np.float64)
    return a / np.linalg.norm(a, axis=0, keepdims=True)


def score_bruteforce(true_means, A) -> float:
    """eq. (Score) by enumerating every injective map (small ranks only)."""
    M = _unit_cols(true_means)
    Ah = _unit_cols(A)
    r, rh = M.shape[1], Ah.shape[1]
    cos = np.abs(M.T @ Ah)                    # r x rh
    best = -np.inf
    if rh < r:
        for pi in itertools.permutations(range(r), rh):
            best = max(best, sum(cos[pi[j], j] for j in range(rh)) / rh)
    else:
        for pi in itertools.permutations(range(rh), r):
            best = max(best, sum(cos[j, pi[j]] for j in range(r)) / r)
    return float(best)


def score(true_means, A) -> float:
    """eq. (Score) as a rectangular assignment problem (any rank)."""
    from scipy.optimize import linear_sum_assignment

    M = _unit_cols(true_means)
    Ah = _unit_cols(A)
    cos = np.abs(M.T @ Ah)
    rows, cols = linear_sum_assignment(cos, maximize=True)
    return float(cos[rows, cols].sum() / min(M.shape[1], Ah.shape[1]))


def model_dist2(lam1, A1, lam2, A2, d: int) -> float:
    """||M1 - M2||^2 for symmetric Kruskal models (lam, A) of order d."""
    A1 = np.asarray(A1, dtype=np.float64)
    A2 = np.asarray(A2, dtype=np.float64)
    lam1 = np.asarray(lam1, dtype=np.float64)
    lam2 = np.asarray(lam2, dtype=np.float64)
    t11 = lam1 @ (A1.T @ A1) ** d @ lam1
    t12 = lam1 @ (A1.T @ A2) ** d @ lam2
    t22 = lam2 @ (A2.T @ A2) ** d @ lam2
    return float(t11 - 2.0 * t12 + t22)


def model_norm2(lam, A, d: int) -> float:
    """||M||^2 = lam' [A'A]^d lam (Lemma 3.4)."""
    A = np.asarray(A, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    return float(lam @ (A.T @ A) ** d @ lam)
