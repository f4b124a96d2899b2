"""Parity of the noise-corrected moments (symtd_moment_stats,
symtd_fg_corrected, symtd_alpha_corrected and symtd_solve with sigma > 0)
with oracle.corrected.

* m and M2 against oracle.corrected.stats, relative to the sums of absolute
  terms: 1e-13 (both are summed in fp64 from the stored values).
* f, g_lambda and G_A of the corrected objective against
  oracle.corrected.fg_corrected, relative to the plain evaluation's
  cancelling terms plus the correction's absolute terms: 1e-12 in fp64,
  1e-5 in fp32, for d = 3 and 4 over ragged shapes.
* alpha_c against oracle.corrected.alpha_corrected, relative to alpha +
  2 |<X, Delta>|abs + ||Delta||^2: 1e-12.
* A corrected solve follows the oracle's L-BFGS on the corrected objective
  step by step, and on a Gaussian mixture its model is closer to the
  noiseless moment sum_j w_j mu_j^{(x)d} than the uncorrected solve's.
"""

import numpy as np
import pytest

import synth
from helpers import TOL, gpu_available, make_case, stored, to_dev
from oracle import corrected as Cr
from oracle import lbfgs as L
from oracle import tensor as T
from oracle.fg import magnitudes
from oracle.normx import normx_implicit
from oracle.solve import INIT_GAUSS, pack, start, unpack

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


def _dtype(kind):
    return torch.float64 if kind == "f64" else torch.float32


def corr_scales(A, m, M2, sigma, d):
    """Sums of the absolute terms of Delta a^d and Delta a^{d-1}, per column."""
    Aa = np.abs(A)
    t = np.sum(A * A, axis=0)
    s2 = sigma ** 2
    if d == 3:
        u = np.abs(m) @ Aa
        return 3 * s2 * u * t, s2 * (np.outer(np.abs(m), t) + 2 * Aa * u)
    Sa = np.abs(M2) + s2 * np.eye(len(m))
    SA = Sa @ Aa
    q = np.sum(Aa * SA, axis=0)
    return 6 * s2 * q * t + 3 * s2 * s2 * t * t, 3 * s2 * (SA * t + Aa * q) + 3 * s2 * s2 * Aa * t


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("n,p", [(7, 50), (75, 750), (33, 1000)])
def test_moment_stats(ctx, kind, n, p):
    V, nu, _ = synth.gmm(n, 3, p, 0.3, 61, n)
    V = stored(V, kind)
    print(f"case stats {kind} n={n} p={p}", flush=True)
    m, M2 = S.symtd_moment_stats(ctx, to_dev(V, _dtype(kind)), to_dev(nu, torch.float64))
    torch.cuda.synchronize()
    m_o, M2_o = Cr.stats(V, nu)
    ms = np.abs(V) @ nu
    Ms = (np.abs(V) * nu) @ np.abs(V).T
    assert np.all(np.abs(m.cpu().numpy() - m_o) <= 1e-13 * ms)
    assert np.all(np.abs(M2.cpu().numpy() - M2_o) <= 1e-13 * Ms)


CASES = [(6, 50, 2, (1,)), (10, 750, 3, (2,)), (20, 300, 7, (3,)), (17, 100, 33, (4,)), (75, 750, 5, (6,))]


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("n,p,r,key", CASES)
def test_fg_corrected(ctx, kind, d, n, p, r, key):
    V, nu, A, lam = make_case(n, p, r, d, key + (d,), sigma=0.2, kind=kind)
    sigma = 0.2
    dt = _dtype(kind)
    alpha = 0.75
    print(f"case fg_corrected {kind} d={d} n={n} p={p} r={r}", flush=True)
    Vd, nud = to_dev(V, dt), to_dev(nu, torch.float64)
    m, M2 = S.symtd_moment_stats(ctx, Vd, nud, second=(d == 4))
    f, g, G = S.symtd_fg_corrected(ctx, Vd, nud, to_dev(A, dt), to_dev(lam, torch.float64), d, sigma, m, M2,
                                   alpha=alpha)
    torch.cuda.synchronize()
    m_o, M2_o = Cr.stats(V, nu)
    ref = Cr.fg_corrected(V, nu, A, lam, d, sigma, alpha, m_o, M2_o)
    mag = magnitudes(V, nu, A, lam, d, alpha)
    fa, pa = corr_scales(A, m_o, M2_o, sigma, d)
    f_scale = mag.f_scale + 2 * float(np.abs(lam) @ fa)
    g_scale = mag.g_scale + 2 * fa
    G_scale = mag.G_scale + 2 * d * np.abs(lam) * pa.max(axis=0)
    ef = abs(float(f.cpu()[0]) - ref.f) / f_scale
    eg = np.max(np.abs(g.cpu().numpy() - ref.g_lambda) / g_scale)
    eG = np.max(np.abs(G.cpu().double().numpy() - ref.G_A) / G_scale[None, :])
    print(f"  errors f {ef:.2e} g {eg:.2e} G {eG:.2e}", flush=True)
    assert max(ef, eg, eG) <= TOL[kind]


def test_fg_corrected_sigma_zero_is_fg(ctx):
    V, nu, A, lam = make_case(10, 300, 4, 3, (8,))
    Vd, nud, Ad, ld = to_dev(V, torch.float64), to_dev(nu, torch.float64), to_dev(A, torch.float64), to_dev(
        lam, torch.float64)
    m, _ = S.symtd_moment_stats(ctx, Vd, nud, second=False)
    a = S.symtd_fg_corrected(ctx, Vd, nud, Ad, ld, 3, 0.0, m, None, alpha=1.0)
    b = S.symtd_fg(ctx, Vd, nud, Ad, ld, 3, alpha=1.0)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("n,p", [(6, 50), (20, 1000), (50, 3001)])
def test_alpha_corrected(ctx, kind, d, n, p):
    V, nu, _ = synth.gmm(n, 3, p, 0.3, 71, n, d)
    V = stored(V, kind)
    sigma = 0.3
    dt = _dtype(kind)
    print(f"case alpha_corrected {kind} d={d} n={n} p={p}", flush=True)
    Vd, nud = to_dev(V, dt), to_dev(nu, torch.float64)
    m, M2 = S.symtd_moment_stats(ctx, Vd, nud, second=(d == 4))
    alpha = normx_implicit(V, nu, d)
    got = S.symtd_alpha_corrected(ctx, Vd, nud, d, sigma, m, M2, alpha)
    m_o, M2_o = Cr.stats(V, nu)
    want = Cr.alpha_corrected(V, nu, d, sigma, alpha, m_o, M2_o)
    fa, _ = corr_scales(V, m_o, M2_o, sigma, d)
    scale = alpha + 2 * float(nu @ fa) + Cr.delta_norm2(m_o, M2_o, sigma, d)
    assert abs(got - want) <= 1e-12 * scale


def test_entry_errors(ctx):
    V, nu, A, lam = make_case(6, 40, 2, 3, (9,))
    Vd, nud, Ad, ld = to_dev(V, torch.float64), to_dev(nu, torch.float64), to_dev(A, torch.float64), to_dev(
        lam, torch.float64)
    m, M2 = S.symtd_moment_stats(ctx, Vd, nud)
    with pytest.raises(S.SymtdError):
        S.symtd_fg_corrected(ctx, Vd, nud, Ad, ld, 5, 0.1, m, M2)          # order 5
    with pytest.raises(S.SymtdError):
        S.symtd_fg_corrected(ctx, Vd, nud, Ad, ld, 4, 0.1, m, None)        # d = 4 without M2
    with pytest.raises(S.SymtdError):
        S.symtd_fg_corrected(ctx, Vd, nud, Ad, ld, 3, -0.1, m, M2)         # negative sigma
    with pytest.raises(S.SymtdError):
        S.symtd_solve(ctx, Vd, nud, 2, 2, sigma=0.1)                       # order 2
    with pytest.raises(S.SymtdError):
        S.symtd_solve_batched(ctx, [dict(V=Vd, nu=nud, d=3, r=2, sigma=0.1)])
    # the context stays usable
    f, _, _ = S.symtd_fg_corrected(ctx, Vd, nud, Ad, ld, 3, 0.1, m, M2)
    torch.cuda.synchronize()
    assert np.isfinite(float(f.cpu()[0]))


def _oracle_corrected_solve(V, nu, d, r, sigma, alpha_c, lam0, A0, **kw):
    n = V.shape[0]
    m_o, M2_o = Cr.stats(V, nu)

    def fun(x):
        lam, A = unpack(x, n, r)
        o = Cr.fg_corrected(V, nu, A, lam, d, sigma, alpha_c, m_o, M2_o)
        return o.f / alpha_c, np.concatenate([o.g_lambda, o.G_A.reshape(-1, order="F")]) / alpha_c

    return L.lbfgs(fun, pack(lam0, A0), **kw)


@pytest.mark.parametrize("d", [3, 4])
def test_corrected_solve_trajectory(ctx, d):
    # d = 3/4, n = 8, r = 3, p = 600 Gaussian mixture, sigma = 0.3, Gaussian start, 150 iterations
    n, p, r, seed, sigma = 8, 600, 3, 4, 0.3
    V, nu, _ = synth.gmm(n, r, p, sigma, 81, d)
    Vd, nud = to_dev(V, torch.float64), to_dev(nu, torch.float64)
    alpha = normx_implicit(V, nu, d)
    alpha_c = Cr.alpha_corrected(V, nu, d, sigma, alpha)
    print(f"case corrected solve d={d}", flush=True)
    out = S.symtd_solve(ctx, Vd, nud, d, r, init=S.INIT_GAUSS, seed=seed, pgtol=0.0, ftol=0.0, max_iters=150,
                        trace_len=151, sigma=sigma)
    lam0, A0 = start(V, r, INIT_GAUSS, seed, 0)
    run = _oracle_corrected_solve(V, nu, d, r, sigma, alpha_c, lam0, A0, pgtol=0.0, ftol=0.0, max_iters=150)
    assert abs(out["alpha"] - alpha_c) <= 1e-12 * alpha
    hist = np.array(run.f_hist) * alpha_c
    tr = out["f_trace"][0]
    k = min(len(hist), int(np.sum(~np.isnan(tr))))
    dev = np.abs(tr[:k] - hist[:k]) / alpha_c
    first = int(np.argmax(dev > 1e-10)) if np.any(dev > 1e-10) else k
    print(f"  gpu f={out['f']:.6e} oracle f={run.f * alpha_c:.6e}; agree for {first} of {k} steps", flush=True)
    assert first >= min(k, 30)
    # the reported f is the corrected objective at the returned model, in fp64
    lam = out["lam"].cpu().numpy()
    A = out["A"].cpu().numpy()
    ref = Cr.fg_corrected(V, nu, A, lam, d, sigma, alpha_c)
    assert abs(out["f"] - ref.f) <= 1e-11 * alpha_c
    M = T.kruskal(lam, A, d)
    Xc = T.kruskal(nu, V, d) - Cr.delta_tensor(*Cr.stats(V, nu), sigma, d)
    assert abs(out["f"] - T.inner(Xc - M, Xc - M)) <= 1e-10 * alpha_c


@pytest.mark.parametrize("d", [3, 4])
def test_correction_recovers_the_clean_moment(ctx, d):
    # Gaussian mixture n = 10, r = 3, p = 40000, sigma = 0.5: the rank-r model
    # fitted to the corrected moment is closer to sum_j w_j mu_j^{(x)d}
    n, r, p, sigma = 10, 3, 40000, 0.5
    V, nu, means = synth.gmm(n, r, p, sigma, 91, d)
    comp = (np.arange(p) * r) // p
    w = np.bincount(comp, minlength=r) / p
    C = T.kruskal(w, means, d)
    Vd, nud = to_dev(V, torch.float64), to_dev(nu, torch.float64)
    err = {}
    for s in (0.0, sigma):
        out = S.symtd_solve(ctx, Vd, nud, d, r, restarts=4, seed=3, pgtol=1e-8, max_iters=2000, sigma=s)
        M = T.kruskal(out["lam"].cpu().numpy(), out["A"].cpu().numpy(), d)
        err[s] = np.sqrt(T.inner(M - C, M - C) / T.inner(C, C))
    print(f"  d={d} relative distance to the clean moment: plain {err[0.0]:.3e} corrected {err[sigma]:.3e}",
          flush=True)
    assert err[sigma] < 0.25 * err[0.0]


@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("n,p,r", [(1, 1, 1), (4, 3, 2), (4096, 40, 2)])
def test_corrected_edge_shapes(ctx, d, n, p, r):
    # one covariate and one observation; the largest n the correction takes
    V, nu, A, lam = make_case(n, p, r, d, (n, p, d), sigma=0.2)
    sigma = 0.4
    print(f"case corrected edge d={d} n={n} p={p} r={r}", flush=True)
    Vd, nud = to_dev(V, torch.float64), to_dev(nu, torch.float64)
    m, M2 = S.symtd_moment_stats(ctx, Vd, nud, second=(d == 4))
    f, g, G = S.symtd_fg_corrected(ctx, Vd, nud, to_dev(A, torch.float64), to_dev(lam, torch.float64), d, sigma,
                                   m, M2, alpha=0.5)
    torch.cuda.synchronize()
    m_o, M2_o = Cr.stats(V, nu)
    ref = Cr.fg_corrected(V, nu, A, lam, d, sigma, 0.5, m_o, M2_o)
    mag = magnitudes(V, nu, A, lam, d, 0.5)
    fa, pa = corr_scales(A, m_o, M2_o, sigma, d)
    assert abs(float(f.cpu()[0]) - ref.f) <= 1e-12 * (mag.f_scale + 2 * float(np.abs(lam) @ fa))
    assert np.all(np.abs(g.cpu().numpy() - ref.g_lambda) <= 1e-12 * (mag.g_scale + 2 * fa))
    G_scale = mag.G_scale + 2 * d * np.abs(lam) * pa.max(axis=0)
    assert np.all(np.abs(G.cpu().numpy() - ref.G_A) <= 1e-12 * G_scale[None, :])
    alpha = normx_implicit(V, nu, d)
    got = S.symtd_alpha_corrected(ctx, Vd, nud, d, sigma, m, M2, alpha)
    want = Cr.alpha_corrected(V, nu, d, sigma, alpha, m_o, M2_o)
    fv, _ = corr_scales(V, m_o, M2_o, sigma, d)
    assert abs(got - want) <= 1e-12 * (alpha + 2 * float(nu @ fv) + Cr.delta_norm2(m_o, M2_o, sigma, d))


def test_corrected_refuses_large_n(ctx):
    V, nu, A, lam = make_case(4097, 8, 1, 3, (77,))
    Vd, nud = to_dev(V, torch.float64), to_dev(nu, torch.float64)
    m, _ = S.symtd_moment_stats(ctx, Vd, nud, second=False)
    with pytest.raises(S.SymtdError):
        S.symtd_fg_corrected(ctx, Vd, nud, to_dev(A, torch.float64), to_dev(lam, torch.float64), 3, 0.1, m, None)
    with pytest.raises(S.SymtdError):
        S.symtd_solve(ctx, Vd, nud, 3, 1, sigma=0.1)
