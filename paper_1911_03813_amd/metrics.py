"""Quality measures of a finished decomposition (Section 4.2).

Host-side post-processing of solve results, used by the benchmark and by
applications: the relative error ||X - M|| / ||X|| from the objective and
alpha, and the similarity score of eq. (Score) between the true component
means of a mixture and the recovered factors.
"""

from __future__ import annotations

import math

import numpy as np


def relative_error(f: float, alpha: float) -> float:
    """sqrt(max(f, 0) / alpha): rounding may leave f slightly negative."""
    return math.sqrt(max(float(f), 0.0) / float(alpha)) if alpha > 0 else float("nan")


def similarity_score(means, factors) -> float:
    """eq. (Score): the best one-to-one pairing of true means with recovered
    factors by |cosine|, averaged over the smaller of the two sets (a
    rectangular assignment, solved exactly by scipy's Hungarian method)."""
    from scipy.optimize import linear_sum_assignment

    mu = np.asarray(means, dtype=np.float64)
    a = np.asarray(factors, dtype=np.float64)
    mu = mu / np.linalg.norm(mu, axis=0)
    a = a / np.linalg.norm(a, axis=0)
    sim = np.abs(mu.T @ a)
    i, j = linear_sum_assignment(-sim)
    return float(sim[i, j].sum()) / min(sim.shape)
