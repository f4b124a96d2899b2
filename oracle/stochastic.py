"""Stochastic objective and gradient, and Adam with the paper's schedule
(Section 5, Lemma 5.1, Table stoch).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Lemma 5.1: for X = (1/p) sum_l v_l^{(x)d} and s columns drawn uniformly with
replacement, X~ = (1/s) sum_k v_{i_k}^{(x)d} has E[X~ a^{d-1}] = X a^{d-1}.
Algorithm 2 then applies unchanged to the sampled columns with weights 1/s.
For general weights nu the same holds with sample k weighted p nu_{i_k} / s
(uniform indices, importance weight p nu_i): E[X~] = sum_l nu_l v_l^{(x)d}.
The shifted objective (alpha = 0) is -2 <X~, M> + ||M||^2, linear in X~, so
its value and gradient are unbiased too.

Indices come from Philox-4x32-10 (``oracle.philox``): sample k of draw t
under seed is word k mod 4 of the block with counter (k div 4, t low word,
t high word, stream) and key (seed low word, seed high word); the word x
maps to the index floor(x p / 2^32).  Training draws use stream 3 (draw t =
the number of gradient steps taken before it); the fixed set on which the
objective is estimated uses stream 4, draw 0.

Adam is Kingma & Ba's method (ICLR 2015, Algorithm 1): with gradient g,
m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, and the step
x <- x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) at step t.
The paper's schedule around it (Section 5): epochs of `epoch_len` steps;
after each epoch the objective is estimated on the fixed set; if the
estimate did not decrease, the learning rate drops from lr0 to lr1 and the
state of the prior epoch is restored; the second time, the method stops and
returns the prior epoch's iterate.  Reading taken where the paper is
silent: "the state of the prior epoch" is the whole optimiser state (x, m, v
and t) saved when that epoch's estimate was accepted; the first epoch is
compared with the estimate at the start; the draw counter is never reset,
so a restored state continues with fresh samples.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fg import fg_implicit
from .philox import MASK, philox4x32_10

STREAM_SAMPLE = 3
STREAM_ESTIMATE = 4


def sample_indices(s: int, p: int, seed: int, draw: int, stream: int = STREAM_SAMPLE) -> np.ndarray:
    """The s column indices of draw `draw` (int64, each in [0, p))."""
    nblk = (s + 3) // 4
    b = np.arange(nblk, dtype=np.uint64)
    t = np.uint64(draw)
    ctr = np.stack([b, np.full(nblk, t & MASK, dtype=np.uint64), np.full(nblk, t >> np.uint64(32), dtype=np.uint64),
                    np.full(nblk, stream, dtype=np.uint64)], axis=-1)
    sd = np.uint64(seed)
    key = np.broadcast_to(np.array([sd & MASK, sd >> np.uint64(32)], dtype=np.uint64), (nblk, 2))
    w = philox4x32_10(ctr, key).reshape(-1)[:s].astype(np.uint64)
    return ((w * np.uint64(p)) >> np.uint64(32)).astype(np.int64)


def sampled_data(V, nu, idx):
    """The sampled columns and their weights p nu_i / s (Lemma 5.1)."""
    V = np.asarray(V, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    p = V.shape[1]
    s = len(idx)
    return V[:, idx], p * nu[idx] / s


def stochastic_fg(V, nu, A, lam, d: int, idx):
    """Shifted objective and gradient (Algorithm 2, alpha = 0) on the
    sampled columns `idx`."""
    Vs, ws = sampled_data(V, nu, idx)
    return fg_implicit(Vs, ws, A, lam, d, 0.0, with_intermediates=False)


@dataclass
class AdamOpts:
    lr0: float = 0.01
    lr1: float = 0.001
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    epoch_len: int = 100
    max_epochs: int = 1000


@dataclass
class AdamResult:
    x: np.ndarray
    epochs: int
    steps: int                    # gradient steps taken (reverted ones included)
    converged: bool               # stopped by the second failed epoch
    trace: list = field(default_factory=list)   # estimate at the start and after each epoch


def adam(grad, estimate, x0, o: AdamOpts) -> AdamResult:
    """Adam with the paper's epoch schedule.  grad(x, draw) returns the
    stochastic gradient for draw number `draw`; estimate(x) the objective
    estimate on the fixed set."""
    x = np.array(x0, dtype=np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    t = 0
    lr = o.lr0
    draws = 0
    f_prev = estimate(x)
    trace = [f_prev]
    saved = (x.copy(), m.copy(), v.copy(), t)
    fails = 0
    epochs = 0
    converged = False
    while epochs < o.max_epochs:
        for _ in range(o.epoch_len):
            g = grad(x, draws)
            draws += 1
            t += 1
            m = o.beta1 * m + (1.0 - o.beta1) * g
            v = o.beta2 * v + (1.0 - o.beta2) * g * g
            mhat = m / (1.0 - o.beta1 ** t)
            vhat = v / (1.0 - o.beta2 ** t)
            x = x - lr * mhat / (np.sqrt(vhat) + o.eps)
        epochs += 1
        fe = estimate(x)
        trace.append(fe)
        if fe < f_prev:
            f_prev = fe
            saved = (x.copy(), m.copy(), v.copy(), t)
            continue
        x, m, v, t = saved[0].copy(), saved[1].copy(), saved[2].copy(), saved[3]
        fails += 1
        if fails == 1:
            lr = o.lr1
        else:
            converged = True
            break
    if not converged:
        x = saved[0].copy()       # the last accepted iterate
    return AdamResult(x, epochs, draws, converged, trace)


def pack(lam, A):
    return np.concatenate([np.asarray(lam, dtype=np.float64), np.asarray(A, dtype=np.float64).reshape(-1, order="F")])


def unpack(x, n, r):
    return x[:r].copy(), x[r:].reshape((n, r), order="F").copy()


def stochastic_solve(V, nu, d: int, lam0, A0, s: int, seed: int, o: AdamOpts, est_samples: int = 1000):
    """Adam on the stochastic shifted objective from one start (lam0, A0).
    Returns (lam, A, AdamResult)."""
    V = np.asarray(V, dtype=np.float64)
    n, p = V.shape
    r = np.asarray(A0).shape[1]
    est_idx = sample_indices(est_samples, p, seed, 0, STREAM_ESTIMATE)

    def grad(x, draw):
        lam, A = unpack(x, n, r)
        o_ = stochastic_fg(V, nu, A, lam, d, sample_indices(s, p, seed, draw))
        return pack(o_.g_lambda, o_.G_A)

    def estimate(x):
        lam, A = unpack(x, n, r)
        return float(stochastic_fg(V, nu, A, lam, d, est_idx).f)

    res = adam(grad, estimate, pack(lam0, A0), o)
    lam, A = unpack(res.x, n, r)
    return lam, A, res
