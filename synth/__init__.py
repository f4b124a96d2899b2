"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out.  It holds none of
the decomposition's arithmetic: no inner products, powers, objective or
gradient terms.  Both the CPU oracle and the GPU path take their inputs from
here, so that they see the same stored values.

Workloads follow the paper's synthetic data:

* observations drawn from a spherical Gaussian mixture, v ~ N(mu_j, sigma^2 I)
  with r components of equal share (Section 4.2); the component means are
  unit vectors, either independent random directions or "congruent" ones
  with pairwise cosine 0.5 as in the paper's own experiments;
* observations with i.i.d. U(0,1) entries (Section 4.1, Table 1);
* a random initial guess A0 ~ N(0,1) with normalised columns, and the
  Gaussian test matrix Omega ~ N(0,1) of the randomized-range-finder start
  (Section 4.2, eq. (rrf)); forming V*Omega is the method's work and is not
  done here.

Every generator is keyed by a tuple of integers through numpy's
SeedSequence, so an input is reproducible from its key alone.
"""

from __future__ import annotations

import numpy as np

ROOT_SEED = 191103813


def rng(*key: int) -> np.random.Generator:
    """A numpy Generator keyed by ROOT_SEED and the given integers."""
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, *[int(k) for k in key]]))


def unit_means(n: int, r: int, *key: int, congruent: bool = False) -> np.ndarray:
    """r unit-norm component means as the columns of an n x r array (fp64).

    congruent=False: mu_j = g_j / ||g_j|| with g_j ~ N(0, I_n).
    congruent=True:  ||mu_j|| = 1 and mu_j' mu_k = 0.5 for j != k (the paper's
    choice in Section 4.2).  Built as Q R with Q an n x r orthonormal basis
    (QR of a Gaussian matrix) and R the Cholesky factor of the target Gram
    matrix 0.5 I + 0.5 11'.  Needs r <= n.
    """
    g = rng(*key).standard_normal((n, r))
    if not congruent:
        return g / np.linalg.norm(g, axis=0, keepdims=True)
    if r > n:
        raise ValueError("congruent means need r <= n")
    q, _ = np.linalg.qr(g)
    gram = 0.5 * np.eye(r) + 0.5 * np.ones((r, r))
    R = np.linalg.cholesky(gram).T          # gram = R' R
    return q @ R


def gmm(n: int, r: int, p: int, sigma: float, *key: int, congruent: bool = False):
    """Spherical Gaussian-mixture observations (Section 4.2).

    Returns (V, nu, means): V is n x p fp64 in column-major (Fortran) order,
    column l being observation l; nu = 1/p; means is n x r.  Observations
    are assigned to components in contiguous blocks of (nearly) equal size:
    block j holds the observations with index in [j*p//r, (j+1)*p//r).
    """
    means = unit_means(n, r, *key, 0, congruent=congruent)
    g = rng(*key, 1)
    comp = (np.arange(p) * r) // p                  # contiguous equal shares
    noise = g.standard_normal((n, p))
    V = means[:, comp] + sigma * noise
    nu = np.full(p, 1.0 / p)
    return np.asfortranarray(V), nu, means


def uniform_obs(n: int, p: int, *key: int):
    """Observations with i.i.d. U(0,1) entries (Section 4.1); nu = 1/p."""
    V = rng(*key).random((n, p))
    return np.asfortranarray(V), np.full(p, 1.0 / p)


def gauss_factors(n: int, r: int, *key: int, normalise: bool = True) -> np.ndarray:
    """A0 ~ N(0,1)^{n x r}, columns scaled to unit norm when normalise."""
    a = rng(*key).standard_normal((n, r))
    if normalise:
        a = a / np.linalg.norm(a, axis=0, keepdims=True)
    return np.asfortranarray(a)


def gauss_weights(r: int, *key: int) -> np.ndarray:
    """A weight vector lambda ~ N(0,1)^r (used by evaluation tests)."""
    return rng(*key).standard_normal(r)


def omega(p: int, r: int, *key: int) -> np.ndarray:
    """Gaussian test matrix Omega ~ N(0,1)^{p x r} of the range-finder start."""
    return np.asfortranarray(rng(*key).standard_normal((p, r)))


# Named workload shapes -----------------------------------------------------
#: (d, n, r, p, sigma) of the small fp64 case, the mid-size case and the
#: large single-instance case.
SMALL = dict(d=3, n=10, r=3, p=750, sigma=1e-2)
MID = dict(d=4, n=100, r=20, p=5000, sigma=1e-2)
LARGE = dict(d=3, n=1000, r=100, p=100_000, sigma=1e-2)


def batch_shapes(count: int, *key: int):
    """Shapes of a grouped workload: n ~ U{16..256}, r ~ U{2..32}, p = 250 r,
    d ~ U{3,4}, sigma ~ U{1e-3, 1e-2}.  Returns a list of dicts."""
    g = rng(*key)
    out = []
    for _ in range(count):
        n = int(g.integers(16, 257))
        r = int(g.integers(2, 33))
        d = int(g.integers(3, 5))
        sigma = float(g.choice([1e-3, 1e-2]))
        out.append(dict(n=n, r=r, p=250 * r, d=d, sigma=sigma))
    return out


def poisson_arrivals(rate: float, count: int, *key: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    gaps = rng(*key).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)
