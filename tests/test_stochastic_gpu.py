"""Parity of the stochastic objective (symtd_fg_sampled) and the device Adam
solver (symtd_solve_adam) with the oracle (oracle.stochastic), Section 5.

* The sampled indices are the oracle's bit for bit; the shifted objective
  and gradient on them match Algorithm 2 on the sampled columns (weights
  p nu_i / s) within 1e-12 (fp64) / 1e-5 (fp32) of the cancelling terms.
* Adam in fp64 follows the oracle's trajectory: the per-epoch estimates
  agree to 1e-9 and every lane takes the same accept / restore / stop
  decisions and the same number of steps.
"""

import numpy as np
import pytest

import synth
from helpers import TOL, compare_fg, gpu_available, make_case, stored, to_dev
from oracle.fg import fg_implicit
from oracle.stochastic import AdamOpts, sample_indices, sampled_data, stochastic_solve

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_1911_03813_amd as S


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    c = S.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("n,p,r,d,s,draw", [(37, 2003, 5, 3, 1, 0), (37, 2003, 5, 3, 7, 11), (64, 5000, 20, 4, 250, 3),
                                            (130, 777, 17, 3, 1000, 123456789012)])
def test_sampled_objective(ctx, kind, n, p, r, d, s, draw):
    dt = torch.float64 if kind == "f64" else torch.float32
    V, nu, A, lam = make_case(n, p, r, d, (90, n, s), 1e-2, kind)
    seed = 77 + s
    print(f"case sampled {kind} n={n} p={p} r={r} d={d} s={s} draw={draw}", flush=True)
    f, g, G, idx = S.symtd_fg_sampled(ctx, to_dev(V, dt), to_dev(nu, torch.float64), to_dev(A, dt),
                                      to_dev(lam, torch.float64), d, s, seed, draw, with_indices=True)
    torch.cuda.synchronize()
    want = sample_indices(s, p, seed, draw)
    assert np.array_equal(idx.cpu().numpy(), want)
    Vs, ws = sampled_data(V, nu, want)
    got = (float(f.cpu()[0]), g.cpu().numpy(), G.cpu().double().numpy())
    errs = compare_fg(got, Vs, ws, A, lam, d, 0.0, kind)
    assert max(errs) <= TOL[kind], errs


def test_sampled_objective_is_unbiased_in_the_mean(ctx):
    # the average over many draws approaches the full shifted objective
    n, p, r, d = 20, 3000, 4, 3
    V, nu, A, lam = make_case(n, p, r, d, (91,), 1e-1, "f64")
    Vd, nud, Ad, ld = to_dev(V, torch.float64), to_dev(nu, torch.float64), to_dev(A, torch.float64), \
        to_dev(lam, torch.float64)
    full = fg_implicit(V, nu, A, lam, d, 0.0)
    fs = []
    for t in range(400):
        f, g, G = S.symtd_fg_sampled(ctx, Vd, nud, Ad, ld, d, 50, 5, t)
        fs.append(float(f.cpu()[0]))
    fs = np.array(fs)
    se = fs.std() / np.sqrt(len(fs))
    assert abs(fs.mean() - full.f) <= 5 * se


def test_adam_follows_the_oracle(ctx):
    n, p, r, d, R = 12, 3000, 3, 3, 2
    V, nu, _ = synth.gmm(n, r, p, 5e-2, 92)
    A0 = np.concatenate([synth.gauss_factors(n, r, 92, 5 + k) for k in range(R)], axis=1)
    o = AdamOpts(lr0=0.01, lr1=0.001, epoch_len=25, max_epochs=14)
    s, se, seed = 40, 300, 21
    print("case adam fp64", flush=True)
    res = S.symtd_solve_adam(ctx, to_dev(V, torch.float64), to_dev(nu, torch.float64), d, r, samples=s,
                             est_samples=se, epoch_len=o.epoch_len, max_epochs=o.max_epochs, lr0=o.lr0, lr1=o.lr1,
                             restarts=R, seed=seed, A0=to_dev(A0, torch.float64), trace_len=o.max_epochs + 1)
    for k in range(R):
        lam_o, A_o, ro = stochastic_solve(V, nu, d, np.ones(r), A0[:, k * r:(k + 1) * r], s, seed, o, est_samples=se)
        tr = res["f_trace"][k][:len(ro.trace)]
        np.testing.assert_allclose(tr, np.array(ro.trace), rtol=1e-9, atol=0)
        assert res["epochs_restarts"][k] == ro.epochs
        assert res["steps_restarts"][k] == ro.steps
        assert res["exit_restarts"][k] == (2 if ro.converged else 3)
        f_o = fg_implicit(V, nu, A_o, lam_o, d, 0.0).f
        assert abs(res["f_restarts"][k] - f_o) <= 1e-8 * abs(f_o)
    best = int(np.argmin(res["f_restarts"]))
    assert res["best_restart"] == best
    f_chk = fg_implicit(V, nu, res["A"].cpu().numpy(), res["lam"].cpu().numpy(), d, 0.0).f
    assert abs(f_chk - res["f"]) <= 1e-12 * abs(f_chk)


def test_adam_fp32_recovers_the_means(ctx):
    # the regime of the paper's example (sigma = 0.1), scaled down: the
    # oracle's Adam reaches a similarity score of 0.999 from these starts
    n, r, p, d = 100, 5, 50_000, 3
    V, nu, means = synth.gmm(n, r, p, 1e-1, 93)
    Vs = stored(V, "f32")
    print("case adam fp32 mixture", flush=True)
    res = S.symtd_solve_adam(ctx, to_dev(Vs, torch.float32), to_dev(nu, torch.float64), d, r, samples=100,
                             est_samples=1000, epoch_len=100, max_epochs=200, restarts=4, seed=3, trace_len=201)
    tr = res["f_trace"][res["best_restart"]]
    tr = tr[np.isfinite(tr)]
    assert tr[-1] < tr[0]
    score = S.metrics.similarity_score(means, res["A"].cpu().double().numpy())
    print(f"  f {res['f']:.6f} score {score:.4f} epochs {res['epochs']} exit {res['exit_reason']}", flush=True)
    assert score > 0.99
    full = fg_implicit(Vs, nu, res["A"].cpu().double().numpy(), res["lam"].cpu().numpy(), d, 0.0).f
    assert abs(full - res["f"]) <= 1e-10 * abs(full)


def test_adam_rejects_bad_options(ctx):
    V = to_dev(np.ones((4, 10)), torch.float64)
    nu = to_dev(np.full(10, 0.1), torch.float64)
    for kw in (dict(samples=0), dict(epoch_len=0), dict(lr0=-1.0), dict(beta1=1.0), dict(restarts=0)):
        with pytest.raises(S.SymtdError):
            S.symtd_solve_adam(ctx, V, nu, 3, 2, **kw)
