"""Parity of the multi-model evaluation, the starts and the device L-BFGS solve
(through the C ABI) with the oracle (oracle.fg, oracle.solve, oracle.lbfgs).

The evaluation of several models side by side is compared element by element
with the oracle per model (1e-12 fp64 / 1e-5 fp32 of the cancelling terms).
The starts are compared with the oracle's Philox/Box-Muller draws.  The solve
is compared with the oracle's L-BFGS on the same data: the f trajectory
step by step while rounding has not yet separated the two runs, then the end
results (stop reason, final f / relative error, the model the result holds).
"""

import numpy as np
import pytest

import synth
from helpers import TOL, compare_fg, gpu_available, make_case, stored, to_dev
from oracle import lbfgs as L
from oracle.fg import fg_implicit
from oracle.metrics import score
from oracle.normx import normx_implicit
from oracle.philox import gaussian_matrix
from oracle.solve import INIT_GAUSS, INIT_RRF, solve, start

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


def dev_case(V, nu, kind):
    dt = torch.float64 if kind == "f64" else torch.float32
    return to_dev(V, dt), to_dev(nu, torch.float64)


# --- several models side by side ---------------------------------------------------

@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("n,p,r,models", [(40, 3000, 5, 3), (100, 5000, 20, 4), (17, 333, 1, 7)])
def test_fg_multi_matches_oracle(ctx, kind, n, p, r, models):
    dt = torch.float64 if kind == "f64" else torch.float32
    d = 3
    V, nu, _, _ = make_case(n, p, r, d, (20, n), kind=kind)
    As = [stored(synth.gauss_factors(n, r, 21, k), kind) for k in range(models)]
    lams = [synth.rng(22, k).standard_normal(r) for k in range(models)]
    alpha = normx_implicit(V, nu, d)
    print(f"case n={n} p={p} r={r} models={models} kind={kind}", flush=True)
    Vd, nud = dev_case(V, nu, kind)
    Ad = to_dev(np.hstack(As), dt)
    ld = to_dev(np.concatenate(lams), torch.float64)
    f, g, G = S.symtd_fg_multi(ctx, Vd, nud, Ad, ld, r, d, alpha)
    torch.cuda.synchronize()
    f, g, G = f.cpu().numpy(), g.cpu().numpy(), G.cpu().numpy().astype(np.float64)
    for k in range(models):
        cols = slice(k * r, (k + 1) * r)
        ef, eg, eG = compare_fg((f[k], g[cols], G[:, cols]), V, nu, As[k], lams[k], d, alpha, kind)
        assert ef <= TOL[kind] and eg <= TOL[kind] and eG <= TOL[kind], (k, ef, eg, eG)
        # and exactly what the single-model call gives for that model, when
        # both calls multiply their last column subtile in the same form (a
        # last subtile of 1..4 columns takes the narrow MFMA form, whose fp32
        # sums run in another order); otherwise the single call is checked
        # against the oracle in its own right
        f1, g1, G1 = S.symtd_fg(ctx, Vd, nud, to_dev(As[k], dt), to_dev(lams[k], torch.float64), d, alpha)
        torch.cuda.synchronize()
        f1, g1, G1 = f1.cpu().numpy()[0], g1.cpu().numpy(), G1.cpu().numpy().astype(np.float64)
        narrow = lambda cols_total: 1 <= cols_total % 16 <= 4
        if narrow(r) == narrow(r * models):
            assert f1 == f[k]
            assert np.array_equal(g1, g[cols])
            assert np.array_equal(G1, G[:, cols])
        else:
            e1 = compare_fg((f1, g1, G1), V, nu, As[k], lams[k], d, alpha, kind)
            assert max(e1) <= TOL[kind], e1


# --- starts --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("init", [INIT_GAUSS, INIT_RRF])
def test_starts_match_oracle(ctx, kind, init):
    n, p, r, d, R, seed = 30, 2000, 4, 3, 3, 77
    V, nu, _ = synth.gmm(n, r, p, 1e-2, 23)
    V = stored(V, kind)
    Vd, nud = dev_case(V, nu, kind)
    alpha = normx_implicit(V, nu, d)
    out = S.symtd_solve(ctx, Vd, nud, d, r, restarts=R, seed=seed, init=init, alpha=alpha, max_evals=1)
    assert out["exit_reason"] == 4 and out["iters"] == 0
    tol = TOL[kind]
    for k in range(R):
        if init == INIT_GAUSS:
            A_ref = gaussian_matrix(n, r, seed, k, 1)
        else:
            A_ref = V @ stored(gaussian_matrix(p, r, seed, k, 2), kind)   # Omega as the device stores it
        A_ref = A_ref / np.linalg.norm(A_ref, axis=0)
        f_ref = fg_implicit(V, nu, stored(A_ref, kind), np.ones(r), d, alpha, with_intermediates=False).f
        # f at every start (the evaluation's own rounding included)
        assert abs(out["f_restarts"][k] - f_ref) <= 10 * tol * alpha, (k, out["f_restarts"][k], f_ref)
        if k == out["best_restart"]:
            A = out["A"].cpu().numpy().astype(np.float64)
            print(f"start {k}: max |A - A_ref| = {np.max(np.abs(A - A_ref)):.2e}", flush=True)
            assert np.max(np.abs(A - A_ref)) <= tol, np.max(np.abs(A - A_ref))
            assert np.array_equal(out["lam"].cpu().numpy(), np.ones(r))
    # the oracle's own starts are the same draws
    for k in range(R):
        _, A_o = start(V, r, init, seed, k)
        if init == INIT_GAUSS:
            assert np.allclose(A_o, gaussian_matrix(n, r, seed, k, 1) / np.linalg.norm(gaussian_matrix(n, r, seed, k, 1), axis=0))


# --- solve ---------------------------------------------------------------------------

def test_trajectory_small_fp64(ctx):
    # d=3, n=10, r=3, p=750 Gaussian mixture (sigma=1e-2), Gaussian start, 200 iterations
    n, p, r, d, seed = 10, 750, 3, 3, 5
    V, nu, _ = synth.gmm(n, r, p, 1e-2, 1)
    Vd, nud = dev_case(V, nu, "f64")
    alpha = normx_implicit(V, nu, d)
    T = 201
    out = S.symtd_solve(ctx, Vd, nud, d, r, init=S.INIT_GAUSS, seed=seed, pgtol=0.0, ftol=0.0, max_iters=200,
                        trace_len=T)
    ref = solve(V, nu, d, r, alpha=alpha, restarts=1, init=INIT_GAUSS, seed=seed, pgtol=0.0, ftol=0.0,
                max_iters=200)
    run = ref.runs[0]
    hist = np.array(run.f_hist) * ref.scale
    tr = out["f_trace"][0]
    k = min(len(hist), int(np.sum(~np.isnan(tr))))
    dev = np.abs(tr[:k] - hist[:k]) / alpha
    first = int(np.argmax(dev > 1e-10)) if np.any(dev > 1e-10) else k
    print(f"gpu: {S.EXIT_NAMES[out['exit_reason']]} iters={out['iters']} evals={out['evals']} f={out['f']:.6e}; "
          f"oracle: {L.REASONS[run.reason]} iters={run.iters} evals={run.evals} f={ref.f:.6e}; "
          f"trajectories agree to 1e-10 alpha for {first} of {k} steps", flush=True)
    assert abs(out["alpha"] - alpha) <= 1e-13 * alpha
    assert first >= min(k, 40)
    assert out["exit_reason"] == run.reason
    assert abs(out["f"] - ref.f) <= 1e-8 * alpha


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_solve_mid(ctx, kind):
    # d=4, n=100, r=20, p=5000, randomized-range-finder starts, 2 restarts
    n, p, r, d, R, seed = 100, 5000, 20, 4, 2, 3
    V, nu, mu = synth.gmm(n, r, p, 1e-2, 2)
    V = stored(V, kind)
    Vd, nud = dev_case(V, nu, kind)
    alpha = normx_implicit(V, nu, d)
    out = S.symtd_solve(ctx, Vd, nud, d, r, restarts=R, seed=seed, init=S.INIT_RRF, pgtol=1e-6, max_iters=300,
                        trace_len=40)
    ref = solve(V, nu, d, r, alpha=alpha, restarts=R, init=INIT_RRF, seed=seed, pgtol=1e-6, max_iters=300)
    rel_ref = np.sqrt(max(ref.f, 0.0) / alpha)
    print(f"{kind}: gpu rel_err={out['rel_err']:.3e} iters={out['iters']} best={out['best_restart']} "
          f"({S.EXIT_NAMES[out['exit_reason']]}); oracle rel_err={rel_ref:.3e} iters={ref.runs[ref.best].iters} "
          f"best={ref.best} ({L.REASONS[ref.runs[ref.best].reason]})", flush=True)
    # the returned model evaluates (fp64 oracle) to the reported f
    A = out["A"].cpu().numpy().astype(np.float64)
    lam = out["lam"].cpu().numpy()
    f_chk = fg_implicit(V, nu, A, lam, d, alpha, with_intermediates=False).f
    tol = TOL[kind]
    assert abs(f_chk - out["f"]) <= 10 * tol * alpha
    # same quality of fit as the oracle's run (A-13: |rel_err difference| <= 1e-4)
    assert abs(out["rel_err"] - rel_ref) <= 1e-4
    if kind == "f64":
        # early trajectory of restart 0 step by step
        hist = np.array(ref.runs[0].f_hist[:40]) * ref.scale
        tr = out["f_trace"][0][:len(hist)]
        assert np.max(np.abs(tr - hist)) <= 1e-10 * alpha
        assert score(A, mu) > 0.9


def test_noiseless_mixture_recovers_means(ctx):
    n, r, p, d = 10, 3, 750, 3
    V, nu, mu = synth.gmm(n, r, p, 0.0, 64)
    Vd, nud = dev_case(V, nu, "f64")
    out = S.symtd_solve(ctx, Vd, nud, d, r, restarts=3, seed=1, init=S.INIT_RRF, pgtol=1e-10, ftol=0.0,
                        max_iters=3000)
    A = out["A"].cpu().numpy()
    assert out["rel_err"] < 1e-5
    assert score(A, mu) > 0.999
    # the oracle's solve from the same starts (eq. (rrf), Philox draws) ends
    # at the same score, and the library's score of eq. (Score) agrees with
    # the oracle's
    alpha = normx_implicit(V, nu, d)
    ref = solve(V, nu, d, r, alpha=alpha, restarts=3, init=INIT_RRF, seed=1, pgtol=1e-10, ftol=0.0, max_iters=3000)
    assert abs(score(ref.A, mu) - score(A, mu)) <= 1e-6
    assert abs(S.metrics.similarity_score(mu, A) - score(A, mu)) <= 1e-14


def test_exit_codes(ctx):
    n, p, r, d = 12, 600, 3, 3
    V, nu, _ = synth.gmm(n, r, p, 1e-2, 30)
    Vd, nud = dev_case(V, nu, "f64")
    alpha = normx_implicit(V, nu, d)
    out = S.symtd_solve(ctx, Vd, nud, d, r, max_iters=3, pgtol=0.0, ftol=0.0)
    assert out["exit_reason"] == L.MAX_ITERS and out["iters"] == 3
    ref = solve(V, nu, d, r, alpha=alpha, max_evals=5, pgtol=0.0, ftol=0.0)
    out = S.symtd_solve(ctx, Vd, nud, d, r, max_evals=5, pgtol=0.0, ftol=0.0)
    assert out["exit_reason"] == L.MAX_EVALS == ref.runs[0].reason
    assert out["evals"] == ref.runs[0].evals <= 5
    assert out["iters"] == ref.runs[0].iters
    # a non-finite objective at the start
    nu_bad = nu.copy()
    nu_bad[3] = np.inf
    out = S.symtd_solve(ctx, Vd, to_dev(nu_bad, torch.float64), d, r, alpha=0.0)
    assert out["exit_reason"] == L.NONFINITE and out["evals"] == 1


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_best_of_restarts(ctx, kind):
    n, p, r, d, R = 20, 1500, 4, 3, 5
    V, nu, _ = synth.gmm(n, r, p, 5e-2, 31)
    V = stored(V, kind)
    Vd, nud = dev_case(V, nu, kind)
    out = S.symtd_solve(ctx, Vd, nud, d, r, restarts=R, seed=9, init=S.INIT_GAUSS, pgtol=1e-6, max_iters=150)
    fr = out["f_restarts"]
    assert out["best_restart"] == int(np.argmin(fr))
    # the reported f is an fp64 evaluation at the best restart's final point:
    # in fp64 the same value the solve ended with, in fp32 within its tolerance
    if kind == "f64":
        assert out["f"] == fr.min()
    else:
        assert abs(out["f"] - fr.min()) <= 10 * TOL[kind] * out["alpha"]
    A = out["A"].cpu().numpy().astype(np.float64)
    f_chk = fg_implicit(V, nu, A, out["lam"].cpu().numpy(), d, out["alpha"], with_intermediates=False).f
    assert abs(f_chk - out["f"]) <= 1e-11 * out["alpha"]


def test_solve_bad_arguments(ctx):
    V, nu, _ = synth.gmm(6, 2, 50, 1e-2, 32)
    Vd, nud = dev_case(V, nu, "f64")
    for kw in ({"m": 0}, {"m": 9}, {"restarts": 0}, {"pgtol": -1.0}, {"max_iters": 0}):
        with pytest.raises(S.SymtdError) as e:
            S.symtd_solve(ctx, Vd, nud, 3, 2, **kw)
        assert e.value.status == -1
