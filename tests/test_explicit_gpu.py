"""Parity of the explicit route (Algorithm 1) with the oracle.

* symtd_form_moment against the explicitly formed X = sum_l nu_l v_l^{(x)d}
  (oracle.tensor.kruskal), entry by entry, relative to the sum of the
  entry's absolute terms: 1e-13 in fp64, 2^-23 (one fp32 rounding) in fp32.
* symtd_fg_explicit against oracle.fg.fg_explicit on the same stored X,
  relative to the explicit route's cancelling terms
  (oracle.fg.magnitudes_explicit): 1e-12 for fp64, 1e-5 for fp32; shapes
  over d = 2 .. 5, ragged n and r (more than one 16-column subtile), and
  the first scenario of Table 1.
* The explicit and implicit evaluations of the same data agree.
"""

import numpy as np
import pytest

import synth
from helpers import TOL, compare_fg, gpu_available, make_case, stored, to_dev
from oracle import tensor as T
from oracle.fg import fg_explicit, magnitudes_explicit

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
@pytest.mark.parametrize("n,p,d", [(3, 9, 2), (7, 50, 3), (5, 30, 4), (4, 17, 5), (75, 750, 3)])
def test_form_moment(ctx, kind, n, p, d):
    dt = torch.float64 if kind == "f64" else torch.float32
    V, nu = synth.uniform_obs(n, p, 100, n, d)
    V = stored(V, kind)
    print(f"case moment {kind} n={n} p={p} d={d}", flush=True)
    X = S.symtd_form_moment(ctx, to_dev(V, dt), to_dev(nu, torch.float64), d)
    torch.cuda.synchronize()
    got = X.cpu().double().numpy().reshape((n,) * d)
    want = T.kruskal(nu, V, d)
    scale = T.kruskal(np.abs(nu), np.abs(V), d)
    tol = 1e-13 if kind == "f64" else 2.0 ** -23
    assert np.all(np.abs(got - want) <= tol * scale)
    # symmetric to rounding: an entry and its transpose are accumulated in
    # different product orders
    assert np.all(np.abs(got - np.swapaxes(got, 0, d - 1)) <= 2 * tol * scale)


CASES = [(6, 50, 3, 2, (1,)), (10, 750, 3, 3, (2,)), (20, 300, 7, 4, (3,)), (17, 100, 33, 3, (4,)),
         (5, 40, 2, 5, (5,)), (75, 750, 5, 3, (6,)), (40, 400, 18, 3, (7,))]


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("n,p,r,d,key", CASES)
def test_fg_explicit(ctx, kind, n, p, r, d, key):
    dt = torch.float64 if kind == "f64" else torch.float32
    V, nu = synth.uniform_obs(n, p, 101, *key)
    V = stored(V, kind)
    A = stored(synth.gauss_factors(n, r, 102, *key), kind)
    lam = synth.rng(103, *key).standard_normal(r)
    print(f"case explicit {kind} n={n} p={p} r={r} d={d}", flush=True)
    X = S.symtd_form_moment(ctx, to_dev(V, dt), to_dev(nu, torch.float64), d)
    Xh = X.cpu().double().numpy().reshape((n,) * d)
    alpha = float(np.sum(Xh * Xh))
    f, g, G = S.symtd_fg_explicit(ctx, X, n, d, to_dev(A, dt), to_dev(lam, torch.float64), alpha)
    torch.cuda.synchronize()
    ref = fg_explicit(Xh, A, lam, d, alpha)
    mag = magnitudes_explicit(Xh, A, lam, d, alpha)
    ef = abs(float(f.cpu()[0]) - ref.f) / mag.f_scale
    eg = float(np.max(np.abs(g.cpu().numpy() - ref.g_lambda) / mag.g_scale))
    eG = float(np.max(np.abs(G.cpu().double().numpy() - ref.G_A) / mag.G_scale[None, :]))
    print(f"  errors f={ef:.2e} g={eg:.2e} G={eG:.2e}", flush=True)
    assert max(ef, eg, eG) <= TOL[kind], (ef, eg, eG)


def test_explicit_equals_implicit(ctx):
    # Table 1's first scenario: d=3, n=75, p=750, r=5, uniform observations
    n, p, r, d = 75, 750, 5, 3
    V, nu = synth.uniform_obs(n, p, 104)
    A = synth.gauss_factors(n, r, 104, 5)
    lam = np.ones(r)
    Vd, nud, Ad, ld = to_dev(V, torch.float64), to_dev(nu, torch.float64), to_dev(A, torch.float64), \
        to_dev(lam, torch.float64)
    X = S.symtd_form_moment(ctx, Vd, nud, d)
    ex = S.symtd_fg_explicit(ctx, X, n, d, Ad, ld, 0.0)
    im = S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 0.0)
    torch.cuda.synchronize()
    got = (float(ex[0].cpu()[0]), ex[1].cpu().numpy(), ex[2].cpu().numpy())
    errs = compare_fg(got, V, nu, A, lam, d, 0.0, "f64")
    assert max(errs) <= 1e-11, errs
    assert abs(float(ex[0].cpu()[0]) - float(im[0].cpu()[0])) <= 1e-12 * abs(float(im[0].cpu()[0]))
