"""Pins of the noise-corrected moments (oracle.corrected).

* The Gaussian moment identity the correction rests on, exactly: for a
  component mean mu (and for a two-component mixture), the moment
  E[(mu + sigma g)^{(x)d}] computed by tensor-product Gauss-Hermite
  quadrature (exact for these degrees) equals mu^{(x)d} + Delta with the
  population statistics m = E[v], M2 = E[v v'], for d = 3 and d = 4.
* The contractions Delta a^d, Delta a^{d-1}, the closed form of
  ||Delta||^2 and <X, Delta> against the explicit tensor Delta.
* The corrected objective with alpha_c is ||X - Delta - M||^2 itself, and
  its gradient is the brute-force derivative of that norm.
"""

import numpy as np
import pytest

from oracle import corrected as Cr
from oracle import tensor as T


@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("n", [2, 3])
def test_gaussian_moment_identity(d, n):
    g = np.random.default_rng(10 + n + d)
    mu = g.standard_normal(n)
    sigma = 0.37
    want = Cr.gaussian_moment(mu, sigma, d)
    M2 = np.outer(mu, mu) + sigma ** 2 * np.eye(n)
    got = T.outer_power(mu, d) + Cr.delta_tensor(mu, M2, sigma, d)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d", [3, 4])
def test_mixture_moment_identity(d):
    g = np.random.default_rng(20 + d)
    n, sigma = 2, 0.5
    mus = g.standard_normal((n, 2))
    w = np.array([0.3, 0.7])
    want = sum(w[j] * Cr.gaussian_moment(mus[:, j], sigma, d) for j in range(2))
    clean = sum(w[j] * T.outer_power(mus[:, j], d) for j in range(2))
    m = mus @ w
    M2 = (mus * w) @ mus.T + sigma ** 2 * np.eye(n)
    np.testing.assert_allclose(clean + Cr.delta_tensor(m, M2, sigma, d), want, rtol=1e-12, atol=1e-13)


def _case(seed, n=3, p=9, r=2):
    g = np.random.default_rng(seed)
    V = g.standard_normal((n, p))
    nu = g.uniform(0.1, 1.0, p)
    A = g.standard_normal((n, r))
    lam = g.standard_normal(r)
    return V, nu, A, lam


@pytest.mark.parametrize("d", [3, 4])
def test_contractions_and_constants(d):
    V, nu, A, lam = _case(30 + d)
    sigma = 0.3
    m, M2 = Cr.stats(V, nu)
    D = Cr.delta_tensor(m, M2, sigma, d)
    full, part = Cr.delta_contractions(A, m, M2, sigma, d)
    for j in range(A.shape[1]):
        assert full[j] == pytest.approx(T.ttsv_all(D, A[:, j]), rel=1e-12, abs=1e-13)
        np.testing.assert_allclose(part[:, j], T.ttsv_all_but_one(D, A[:, j]), rtol=1e-12, atol=1e-13)
    assert Cr.delta_norm2(m, M2, sigma, d) == pytest.approx(T.inner(D, D), rel=1e-12)
    X = T.kruskal(nu, V, d)
    assert Cr.x_dot_delta(V, nu, m, M2, sigma, d) == pytest.approx(T.inner(X, D), rel=1e-12)


@pytest.mark.parametrize("d", [3, 4])
def test_corrected_objective_is_the_corrected_norm(d):
    V, nu, A, lam = _case(40 + d)
    sigma = 0.25
    m, M2 = Cr.stats(V, nu)
    X = T.kruskal(nu, V, d)
    D = Cr.delta_tensor(m, M2, sigma, d)
    M = T.kruskal(lam, A, d)
    R = X - D - M
    alpha_c = Cr.alpha_corrected(V, nu, d, sigma, T.inner(X, X))
    assert alpha_c == pytest.approx(T.inner(X - D, X - D), rel=1e-12)
    o = Cr.fg_corrected(V, nu, A, lam, d, sigma, alpha_c)
    assert o.f == pytest.approx(T.inner(R, R), rel=1e-11, abs=1e-12)
    g = np.array([-2.0 * T.inner(R, T.outer_power(A[:, j], d)) for j in range(A.shape[1])])
    G = np.stack([-2.0 * d * lam[j] * T.ttsv_all_but_one(R, A[:, j]) for j in range(A.shape[1])], axis=1)
    np.testing.assert_allclose(o.g_lambda, g, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(o.G_A, G, rtol=1e-11, atol=1e-12)


def test_sigma_zero_is_the_plain_objective():
    from oracle.fg import fg_implicit
    V, nu, A, lam = _case(50)
    for d in (3, 4):
        a = Cr.fg_corrected(V, nu, A, lam, d, 0.0, 1.5)
        b = fg_implicit(V, nu, A, lam, d, 1.5)
        assert a.f == b.f
        assert np.array_equal(a.g_lambda, b.g_lambda) and np.array_equal(a.G_A, b.G_A)


def test_corrected_fit_recovers_the_clean_moment():
    # Gaussian mixture n = 10, r = 3, p = 40000, sigma = 0.5, d = 3: the rank-r
    # fit of X - Delta lies far closer to sum_j w_j mu_j^{(x)3} than the fit of X
    from oracle import lbfgs as L
    from oracle.normx import normx_implicit
    from oracle.solve import INIT_RRF, pack, solve, start, unpack
    import synth
    n, r, p, sigma, d = 10, 3, 40000, 0.5, 3
    V, nu, means = synth.gmm(n, r, p, sigma, 91, d)
    w = np.bincount((np.arange(p) * r) // p, minlength=r) / p
    C = T.kruskal(w, means, d)
    alpha = normx_implicit(V, nu, d)
    m, M2 = Cr.stats(V, nu)
    ac = Cr.alpha_corrected(V, nu, d, sigma, alpha, m, M2)
    plain = solve(V, nu, d, r, alpha=alpha, restarts=2, seed=3, pgtol=1e-8, max_iters=2000)
    best = None
    for k in range(2):
        def fun(x):
            lam, A = unpack(x, n, r)
            o = Cr.fg_corrected(V, nu, A, lam, d, sigma, ac, m, M2)
            return o.f / ac, np.concatenate([o.g_lambda, o.G_A.reshape(-1, order="F")]) / ac
        run = L.lbfgs(fun, pack(*start(V, r, INIT_RRF, 3, k)), pgtol=1e-8, max_iters=2000)
        best = run if best is None or run.f < best.f else best

    def dist(lam, A):
        M = T.kruskal(lam, A, d)
        return np.sqrt(T.inner(M - C, M - C) / T.inner(C, C))

    e_plain = dist(plain.lam, plain.A)
    e_corr = dist(*unpack(best.x, n, r))
    assert e_corr < 0.1 and e_plain > 0.5
