"""Pins of the stochastic objective and of Adam (oracle.stochastic).

* Lemma 5.1, exactly: averaging the sampled TTSVs X~ a^{d-1} over all p^s
  index tuples of a tiny case (each tuple has probability p^-s) gives the
  TTSVs of the explicitly formed X, for uniform and for general weights;
  the same for the shifted objective and its gradient, which are linear in
  X~.
* The index generator: indices in [0, p), the published Philox known-answer
  words mapped by floor(x p / 2^32), uniform counts.
* Adam: Kingma & Ba's bias correction makes a constant gradient g move x by
  lr g / (|g| + eps) at every step, exactly.
* The schedule: a scripted sequence of estimates drives the learning-rate
  drop, the restore of the prior epoch's state and the stop.
"""

import itertools
import json
import os

import numpy as np
import pytest

from oracle import tensor as T
from oracle.fg import fg_bruteforce, fg_implicit
from oracle.philox import philox4x32_10
from oracle.stochastic import (AdamOpts, adam, sample_indices, sampled_data, stochastic_fg, stochastic_solve,
                               STREAM_ESTIMATE)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _case(seed, n=3, p=3, r=2, d=3, uniform=True):
    g = np.random.default_rng(seed)
    V = g.standard_normal((n, p))
    nu = np.full(p, 1.0 / p) if uniform else g.uniform(0.2, 1.0, p)
    A = g.standard_normal((n, r))
    lam = g.standard_normal(r)
    return V, nu, A, lam, d


@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("p,s,d", [(3, 2, 3), (4, 3, 3), (3, 3, 4)])
def test_lemma_5_1_by_enumeration(uniform, p, s, d):
    V, nu, A, lam, d = _case(7 + p + s, n=3, p=p, d=d, uniform=uniform)
    X = T.kruskal(nu, V, d)
    want_Y = np.stack([T.ttsv_all_but_one(X, A[:, j]) for j in range(A.shape[1])], axis=1)
    full = fg_bruteforce(V, nu, A, lam, d, alpha=0.0)
    Y = np.zeros_like(want_Y)
    f = 0.0
    g = np.zeros_like(lam)
    G = np.zeros_like(A)
    for tup in itertools.product(range(p), repeat=s):
        Vs, ws = sampled_data(V, nu, np.array(tup))
        o = fg_implicit(Vs, ws, A, lam, d, 0.0)
        Y += o.Y
        f += o.f
        g += o.g_lambda
        G += o.G_A
    k = float(p ** s)
    np.testing.assert_allclose(Y / k, want_Y, rtol=1e-12, atol=1e-14)
    assert abs(f / k - full.f) <= 1e-12 * max(1.0, abs(full.f))
    np.testing.assert_allclose(g / k, full.g_lambda, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(G / k, full.G_A, rtol=1e-11, atol=1e-13)


def test_sample_weights_are_one_over_s_for_uniform_nu():
    V, nu, *_ = _case(1, p=50)
    _, ws = sampled_data(V, nu, np.array([3, 3, 49, 0]))
    np.testing.assert_allclose(ws, 0.25, rtol=1e-15)


def test_indices_from_the_published_vectors():
    # Philox-4x32-10 known answers (Salmon et al.): the words of a block map
    # to indices floor(x p / 2^32)
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for case in kat["cases"]:
        ctr = np.array([[int(x, 16) for x in case["counter"]]], dtype=np.uint64)
        key = np.array([[int(x, 16) for x in case["key"]]], dtype=np.uint64)
        w = philox4x32_10(ctr, key)[0]
        assert [int(x) for x in w] == [int(x, 16) for x in case["output"]]
    # and sample_indices applies that map to block (k div 4, draw, 0, stream)
    s, p, seed, draw = 8, 1000, 12345, 7
    idx = sample_indices(s, p, seed, draw)
    ctr = np.array([[b, draw, 0, 3] for b in range(2)], dtype=np.uint64)
    key = np.array([[seed, 0]] * 2, dtype=np.uint64)
    w = philox4x32_10(ctr, key).reshape(-1).astype(np.uint64)
    assert idx.tolist() == [int(x) * p >> 32 for x in w]


def test_indices_are_uniform_and_in_range():
    p = 37
    idx = np.concatenate([sample_indices(1000, p, 5, t) for t in range(40)])
    assert idx.min() >= 0 and idx.max() < p
    counts = np.bincount(idx, minlength=p)
    exp = len(idx) / p
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 80.0                       # 36 degrees of freedom: p-value ~ 5e-5
    assert not np.array_equal(sample_indices(10, p, 5, 0), sample_indices(10, p, 5, 1))
    assert not np.array_equal(sample_indices(10, p, 5, 0), sample_indices(10, p, 5, 0, STREAM_ESTIMATE))


def test_adam_constant_gradient_closed_form():
    o = AdamOpts(lr0=0.05, epoch_len=7, max_epochs=1)
    g0 = np.array([2.0, -0.5, 1e-3, 0.0])
    x0 = np.array([1.0, 1.0, 1.0, 1.0])
    # the estimate keeps decreasing, so the single epoch is accepted
    res = adam(lambda x, t: g0, lambda x: -float(np.sum(x0 - x)), x0, o)
    step = o.lr0 * g0 / (np.abs(g0) + o.eps)
    np.testing.assert_allclose(res.x, x0 - 7 * step, rtol=0, atol=1e-14)
    assert res.steps == 7 and res.epochs == 1 and not res.converged


def test_adam_first_step_on_a_quadratic():
    c = np.array([3.0, -2.0, 0.5])
    x0 = np.zeros(3)
    o = AdamOpts(lr0=0.1, epoch_len=1, max_epochs=1)
    res = adam(lambda x, t: x - c, lambda x: 0.5 * float(np.sum((x - c) ** 2)), x0, o)
    # m^ = g and v^ = g^2 after one step: the move is lr g / (|g| + eps),
    # lr sign(c - x0) up to eps
    g = x0 - c
    np.testing.assert_allclose(res.x, x0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.x, 0.1 * np.sign(c), rtol=0, atol=1e-8)


def test_schedule_drops_rate_restores_and_stops():
    # constant gradient 1: x decreases by lr per step (up to eps); the
    # scripted estimates fail after epoch 3 and after epoch 5
    script = iter([10.0, 9.0, 8.0, 8.5, 7.0, 7.5])
    seen = []

    def est(x):
        seen.append(float(x[0]))
        return next(script)

    o = AdamOpts(lr0=0.01, lr1=0.001, epoch_len=10, max_epochs=50)
    res = adam(lambda x, t: np.ones(1), est, np.zeros(1), o)
    assert res.converged and res.epochs == 5 and res.steps == 50
    assert res.trace == [10.0, 9.0, 8.0, 8.5, 7.0, 7.5]
    step0 = 0.01 / (1.0 + 1e-8)
    step1 = 0.001 / (1.0 + 1e-8)
    # epochs 1, 2 accepted at lr0; epoch 3 rejected (restored to after epoch 2);
    # epoch 4 at lr1 accepted; epoch 5 rejected: the answer is after epoch 4
    np.testing.assert_allclose(seen[2], -20 * step0, rtol=1e-12)
    np.testing.assert_allclose(seen[4], -20 * step0 - 10 * step1, rtol=1e-12)
    np.testing.assert_allclose(res.x[0], -20 * step0 - 10 * step1, rtol=1e-12)


def test_solve_decreases_the_full_objective():
    import synth
    n, r, p, d = 8, 2, 400, 3
    V, nu, means = synth.gmm(n, r, p, 1e-2, 91)
    A0 = synth.gauss_factors(n, r, 91, 5)
    lam0 = np.ones(r)
    o = AdamOpts(epoch_len=50, max_epochs=40)
    lam, A, res = stochastic_solve(V, nu, d, lam0, A0, 20, 3, o, est_samples=200)
    f0 = fg_implicit(V, nu, A0, lam0, d, 0.0).f
    f1 = fg_implicit(V, nu, A, lam, d, 0.0).f
    assert f1 < f0
    assert res.trace[0] > min(res.trace)
    assert stochastic_fg(V, nu, A, lam, d, np.arange(p)).f == pytest.approx(f1, rel=1e-12)
