"""Pins of the oracle's generator, starts and L-BFGS driver (CPU only).

Each check ties the oracle to something other than itself: the generator's
published known-answer vectors, distribution tests of the normals, the
dense BFGS inverse update, closed-form optima (a convex quadratic, the
Rosenbrock function, Eckart-Young for d = 2, an exactly representable
mixture) and the strong Wolfe conditions themselves.
"""

import json
import os

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import lbfgs as L
from oracle.fg import fg_implicit
from oracle.metrics import rel_err, score
from oracle.normx import normx_implicit
from oracle.philox import gaussian_matrix, normals, philox4x32_10, uniform_from_word
from oracle.solve import INIT_GAUSS, INIT_RRF, objective, pack, solve, start, unpack

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- generator -----------------------------------------------------------------

def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as fh:
        kat = json.load(fh)
    for case in kat["cases"]:
        ctr = np.array([[int(w, 16) for w in case["counter"]]], dtype=np.uint64)
        key = np.array([[int(w, 16) for w in case["key"]]], dtype=np.uint64)
        out = philox4x32_10(ctr, key)[0]
        assert [f"{int(w):08x}" for w in out] == case["output"]


def test_uniform_map_open_interval():
    u = uniform_from_word(np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint64))
    assert u[0] == 0.5 / 2**32 and u[-1] == 1.0 - 0.5 / 2**32
    assert np.all((u > 0) & (u < 1))


def test_normals_distribution():
    z = normals(400_000, seed=1234, restart=3, stream=2)
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    d, _ = stats.kstest(z, "norm")
    assert d < 1.95 / np.sqrt(n)          # 0.1% critical value of the KS statistic
    # the two normals of one Box-Muller pair are uncorrelated, and so are the pairs
    zz = z.reshape(-1, 4)
    for a, b in ((0, 1), (2, 3), (0, 2), (1, 3)):
        assert abs(np.corrcoef(zz[:, a], zz[:, b])[0, 1]) < 5.0 / np.sqrt(zz.shape[0])
    # fourth moment of a standard normal is 3
    assert abs(np.mean(z**4) - 3.0) < 0.05


def test_streams_differ():
    a = normals(64, 7, 0, 1)
    b = normals(64, 7, 1, 1)
    c = normals(64, 7, 0, 2)
    e = normals(64, 8, 0, 1)
    assert not np.allclose(a, b) and not np.allclose(a, c) and not np.allclose(a, e)
    assert np.array_equal(normals(10, 7, 0, 1), a[:10])            # prefix property
    G = gaussian_matrix(5, 3, 7, 0, 1)
    assert np.array_equal(G.T.reshape(-1), normals(15, 7, 0, 1))   # column-major numbering


# --- starts ----------------------------------------------------------------------

def test_starts_unit_columns():
    V, nu, _ = synth.gmm(20, 4, 400, 1e-2, 50)
    for kind in (INIT_GAUSS, INIT_RRF):
        lam, A = start(V, 4, kind, 11, 2)
        assert np.array_equal(lam, np.ones(4))
        assert np.allclose(np.linalg.norm(A, axis=0), 1.0, atol=1e-14)


def test_rrf_rank_one():
    # a rank-one V = v c': every column of V Omega is a multiple of v
    v = synth.rng(51).standard_normal(9)
    c = synth.rng(52).standard_normal(300)
    V = np.outer(v, c)
    _, A = start(V, 3, INIT_RRF, 5, 0)
    vh = v / np.linalg.norm(v)
    for j in range(3):
        assert abs(abs(A[:, j] @ vh) - 1.0) < 1e-13


# --- L-BFGS pieces ---------------------------------------------------------------

def test_two_loop_equals_dense_bfgs():
    rg = synth.rng(60)
    N, k = 12, 5
    Q = rg.standard_normal((N, N))
    Q = Q @ Q.T + N * np.eye(N)
    S = [rg.standard_normal(N) for _ in range(k)]
    Y = [Q @ s for s in S]            # curvature pairs of a convex quadratic (s'y > 0)
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    H = gamma * np.eye(N)
    for s, y in zip(S, Y):            # explicit BFGS inverse updates, oldest first
        rho = 1.0 / (y @ s)
        E = np.eye(N) - rho * np.outer(s, y)
        H = E @ H @ E.T + rho * np.outer(s, s)
    g = rg.standard_normal(N)
    assert np.allclose(L.two_loop(g, S, Y, gamma), H @ g, rtol=1e-12, atol=1e-13)


def test_cubic_min_exact():
    # c(t) = t^3 - 6 t^2 + 9 t + 1 has its local minimum at t = 3
    c = lambda t: t**3 - 6 * t**2 + 9 * t + 1
    dc = lambda t: 3 * t**2 - 12 * t + 9
    for a, b in ((2.0, 4.0), (4.0, 2.0), (1.5, 3.5), (2.5, 10.0)):
        assert abs(L.cubic_min(a, c(a), dc(a), b, c(b), dc(b)) - 3.0) < 1e-12


def rosen(x):
    f = 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
    g = np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200.0 * (x[1] - x[0] ** 2)])
    return f, g


@pytest.mark.parametrize("seed", range(6))
def test_line_search_strong_wolfe(seed):
    rg = synth.rng(70, seed)
    x = rg.uniform(-2, 2, 2)
    f0, g0 = rosen(x)
    d = -g0 if seed % 2 == 0 else -g0 / np.linalg.norm(g0) * rg.uniform(0.01, 5)
    dphi0 = float(g0 @ d)

    def phi(a):
        f, g = rosen(x + a * d)
        return f, float(g @ d), g

    a1 = min(1.0, 1.0 / np.sqrt(-dphi0)) if seed % 2 == 0 else 1.0
    a, fa, _, ev = L.line_search(phi, f0, dphi0, a1)
    assert a is not None and ev <= L.MAXLS
    fa2, da, _ = phi(a)
    assert fa2 <= f0 + L.C1 * a * dphi0
    assert abs(da) <= -L.C2 * dphi0


def test_lbfgs_convex_quadratic():
    rg = synth.rng(61)
    N = 40
    Q = rg.standard_normal((N, N))
    Q = Q @ Q.T / N + 0.1 * np.eye(N)
    xs = rg.standard_normal(N)
    # f = (x - x*)' Q (x - x*) / 2: minimum 0 at x*, so f is resolved down to the tolerance
    res = L.lbfgs(lambda x: (0.5 * (x - xs) @ Q @ (x - xs), Q @ (x - xs)), np.zeros(N), pgtol=1e-11, ftol=0.0)
    assert res.reason == L.PGTOL
    assert np.allclose(res.x, xs, rtol=0, atol=1e-9)
    assert all(res.f_hist[i + 1] < res.f_hist[i] for i in range(len(res.f_hist) - 1))


def test_lbfgs_rosenbrock():
    res = L.lbfgs(rosen, np.array([-1.2, 1.0]), pgtol=1e-10, ftol=0.0)
    assert res.reason == L.PGTOL
    assert np.allclose(res.x, [1.0, 1.0], atol=1e-8)


def test_lbfgs_exit_codes():
    x0 = np.array([-1.2, 1.0])
    r = L.lbfgs(rosen, x0, max_iters=3)
    assert r.reason == L.MAX_ITERS and r.iters == 3
    r = L.lbfgs(rosen, x0, max_evals=5, pgtol=0.0, ftol=0.0)
    assert r.reason == L.MAX_EVALS and r.evals <= 5
    r = L.lbfgs(lambda x: (np.nan, x), x0)
    assert r.reason == L.NONFINITE and r.evals == 1
    r = L.lbfgs(rosen, np.array([1.0, 1.0]))
    assert r.reason == L.PGTOL and r.iters == 0
    r = L.lbfgs(rosen, x0, pgtol=0.0, ftol=1e-3)
    assert r.reason == L.FTOL


# --- the decomposition objective and solve --------------------------------------

def test_objective_packing_central_difference():
    # the gradient of phi(x) matches central differences in a lambda and an A coordinate
    V, nu, _ = synth.gmm(7, 3, 90, 1e-1, 62)
    r, d = 3, 3
    alpha = normx_implicit(V, nu, d)
    lam, A = start(V, r, INIT_RRF, 3, 0)
    lam = lam * np.array([0.5, 1.0, 1.5])
    fun = objective(V, nu, d, r, alpha)
    x = pack(lam, A)
    _, g = fun(x)
    for i in (1, r + 2, r + 7 * 1 + 4, len(x) - 1):
        h = 1e-6
        e = np.zeros_like(x)
        e[i] = h
        fd = (fun(x + e)[0] - fun(x - e)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i]))
    lam2, A2 = unpack(x, 7, r)
    assert np.array_equal(lam2, lam) and np.array_equal(A2, A)


def test_solve_d2_eckart_young():
    # d = 2: X = V D_nu V' is PSD; the best rank-r fit leaves the smallest eigenvalues
    rg = synth.rng(63)
    n, p, r = 6, 40, 2
    V = rg.standard_normal((n, p))
    nu = np.full(p, 1.0 / p)
    X = (V * nu) @ V.T
    theta = np.sort(np.linalg.eigvalsh(X))[::-1]
    fstar = float(np.sum(theta[r:] ** 2))
    alpha = normx_implicit(V, nu, 2)
    assert abs(alpha - np.sum(theta**2)) <= 1e-13 * alpha
    res = solve(V, nu, 2, r, alpha=alpha, restarts=3, init=INIT_RRF, seed=9, pgtol=1e-12, ftol=0.0,
                max_iters=2000)
    assert abs(res.f - fstar) <= 1e-9 * alpha


def test_solve_noiseless_mixture():
    # sigma = 0: X = sum_j (1/r) mu_j^{(x)3} exactly, so the fit reaches f ~ 0 and recovers the means
    n, r, p, d = 10, 3, 750, 3
    V, nu, mu = synth.gmm(n, r, p, 0.0, 64)
    alpha = normx_implicit(V, nu, d)
    res = solve(V, nu, d, r, alpha=alpha, restarts=3, init=INIT_RRF, seed=1, pgtol=1e-10, ftol=0.0,
                max_iters=3000)
    assert rel_err(res.f, alpha) < 1e-5
    assert score(res.A, mu) > 0.999


def test_solve_best_of_restarts():
    V, nu, _ = synth.gmm(8, 4, 400, 5e-2, 65)
    alpha = normx_implicit(V, nu, 3)
    res = solve(V, nu, 3, 3, alpha=alpha, restarts=4, init=INIT_GAUSS, seed=2, pgtol=1e-6, max_iters=300)
    assert res.best == int(np.argmin(res.f_restarts))
    assert res.f == min(res.f_restarts)
    # the returned model evaluates to the reported f
    o = fg_implicit(V, nu, res.A, res.lam, 3, alpha, with_intermediates=False)
    assert abs(o.f - res.f) <= 1e-12 * alpha
