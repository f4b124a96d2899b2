"""Pins of the CPU oracle against facts other than itself (runs on the CPU).

Each test names the passage of the paper, or the mathematical fact, that
fixes the expected value.  Together they are chosen so that a plausible slip
anywhere in the oracle (a dropped term, a wrong sign, power or index, a
transposed operand) fails at least one of them.
"""

import itertools
import json
import os

import numpy as np
import pytest

import synth
from oracle import tensor as T
from oracle.fg import fg_bruteforce, fg_implicit, grad_paper_explicit, magnitudes
from oracle.metrics import model_dist2, model_norm2, rel_err, score, score_bruteforce
from oracle.normx import normx_explicit, normx_implicit

HERE = os.path.dirname(os.path.abspath(__file__))


def _case(n, p, r, d, key, gmm=False):
    if gmm:
        V, nu, _ = synth.gmm(n, r, p, 0.1, 7, *key)
    else:
        V = synth.rng(1, *key).standard_normal((n, p))
        nu = synth.rng(2, *key).random(p) + 0.1          # arbitrary positive weights
    A = synth.rng(3, *key).standard_normal((n, r))
    lam = synth.rng(4, *key).standard_normal(r)
    return V, nu, A, lam


# --- tensor primitives against their definitions ---------------------------

def test_outer_power_entries():
    # eq. (outer_product): (a^{(x)3})_{ijk} = a_i a_j a_k, by an explicit loop
    a = np.array([1.5, -2.0, 0.25])
    t = T.outer_power(a, 3)
    for i, j, k in itertools.product(range(3), repeat=3):
        assert t[i, j, k] == a[i] * a[j] * a[k]


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_lemma_3_1_and_3_2(d):
    # Lemma 3.1: <a^{(x)d}, b^{(x)d}> = <a,b>^d ; Lemma 3.2: b^{(x)d} a^{d-1} = <a,b>^{d-1} b
    g = synth.rng(11, d)
    for n in (1, 2, 4, 6):
        a, b = g.standard_normal(n), g.standard_normal(n)
        ip = T.inner(T.outer_power(a, d), T.outer_power(b, d))
        assert np.isclose(ip, (a @ b) ** d, rtol=1e-12, atol=1e-14)
        S = T.outer_power(b, d)
        assert np.allclose(T.ttsv_all_but_one(S, a), (a @ b) ** (d - 1) * b, rtol=1e-12, atol=1e-14)
        assert np.isclose(T.ttsv_all(S, a), (a @ b) ** d, rtol=1e-12, atol=1e-14)


# --- Algorithm 2 against brute force on explicit tensors -------------------

@pytest.mark.parametrize("n,p,r,d", [(3, 5, 2, 2), (4, 7, 3, 3), (5, 9, 4, 3), (3, 6, 2, 4),
                                     (4, 5, 3, 5), (2, 3, 1, 6), (6, 11, 5, 3)])
@pytest.mark.parametrize("gmm", [False, True])
def test_implicit_matches_bruteforce(n, p, r, d, gmm):
    V, nu, A, lam = _case(n, p, r, d, (n, p, r, d), gmm=gmm)
    alpha = normx_explicit(V, nu, d)
    imp = fg_implicit(V, nu, A, lam, d, alpha)
    bf = fg_bruteforce(V, nu, A, lam, d)
    mag = magnitudes(V, nu, A, lam, d, alpha)
    assert abs(imp.f - bf.f) <= 1e-12 * mag.f_scale
    assert np.all(np.abs(imp.g_lambda - bf.g_lambda) <= 1e-12 * mag.g_scale)
    assert np.all(np.abs(imp.G_A - bf.G_A) <= 1e-12 * mag.G_scale[None, :])
    # the gradient as printed in eqs. (gradl)/(gradb) is the same derivative
    g, G = grad_paper_explicit(V, nu, A, lam, d)
    assert np.all(np.abs(g - bf.g_lambda) <= 1e-12 * mag.g_scale)
    assert np.all(np.abs(G - bf.G_A) <= 1e-12 * mag.G_scale[None, :])


def test_w_two_ways():
    # Lemma 3.5 with Lemma 3.2: w_j = a_j'y_j equals sum_l nu_l <v_l, a_j>^d
    V, nu, A, lam = _case(40, 300, 6, 3, (5,))
    out = fg_implicit(V, nu, A, lam, 3)
    w2 = nu @ (V.T @ A) ** 3
    assert np.allclose(out.w, w2, rtol=1e-12, atol=1e-13 * np.abs(nu) @ np.abs(V.T @ A) ** 3)


def test_golden_worked_example():
    with open(os.path.join(HERE, "golden", "worked_example_d3.json")) as fh:
        ex = json.load(fh)
    V = np.array(ex["V"]); A = np.array(ex["A"])
    out = fg_implicit(V, np.array(ex["nu"]), A, np.array(ex["lambda"]), ex["d"], ex["alpha"])
    assert out.f == pytest.approx(ex["f"], abs=1e-14)
    assert np.allclose(out.g_lambda, ex["g_lambda"], atol=1e-13)
    assert np.allclose(out.G_A, ex["G_A"], atol=1e-13)
    assert normx_implicit(V, np.array(ex["nu"]), ex["d"]) == pytest.approx(ex["alpha"], abs=1e-15)


# --- special cases and closed forms ----------------------------------------

@pytest.mark.parametrize("d", [2, 3, 4])
def test_exact_solution_zero(d):
    # r = p, A = V, lambda = nu reproduces X exactly: f = 0 and g = 0
    V, nu, _, _ = _case(7, 5, 5, d, (9, d))
    alpha = normx_implicit(V, nu, d)
    out = fg_implicit(V, nu, V.copy(), nu.copy(), d, alpha)
    mag = magnitudes(V, nu, V, nu, d, alpha)
    assert abs(out.f) <= 1e-13 * mag.f_scale
    assert np.all(np.abs(out.g_lambda) <= 1e-13 * mag.g_scale)
    assert np.all(np.abs(out.G_A) <= 1e-13 * mag.G_scale[None, :])


def test_gmm_sigma0_exact():
    # sigma = 0: X = (1/r) sum_j mu_j^{(x)d}, so A = means, lambda = 1/r is exact
    n, r, p, d = 12, 4, 400, 3
    V, nu, means = synth.gmm(n, r, p, 0.0, 21)
    alpha = normx_implicit(V, nu, d)
    out = fg_implicit(V, nu, means, np.full(r, 1.0 / r), d, alpha)
    assert abs(out.f) <= 1e-14 * alpha
    assert np.max(np.abs(out.G_A)) <= 1e-13


@pytest.mark.parametrize("d", [2, 3, 5])
def test_rank_one_closed_form(d):
    # p = r = 1: f = nu^2 |v|^{2d} - 2 nu lam (v'a)^d + lam^2 |a|^{2d}
    g = synth.rng(31, d)
    v, a = g.standard_normal(6), g.standard_normal(6)
    nu, lam = 0.7, -1.3
    expect = nu**2 * (v @ v) ** d - 2 * nu * lam * (v @ a) ** d + lam**2 * (a @ a) ** d
    out = fg_implicit(v[:, None], np.array([nu]), a[:, None], np.array([lam]), d,
                      normx_implicit(v[:, None], np.array([nu]), d))
    assert out.f == pytest.approx(expect, rel=1e-13)
    # and the derivatives of the same closed form
    dlam = -2 * nu * (v @ a) ** d + 2 * lam * (a @ a) ** d
    da = -2 * nu * lam * d * (v @ a) ** (d - 1) * v + lam**2 * 2 * d * (a @ a) ** (d - 1) * a
    assert out.g_lambda[0] == pytest.approx(dlam, rel=1e-12)
    assert np.allclose(out.G_A[:, 0], da, rtol=1e-12, atol=1e-12 * np.abs(da).max())


def test_d2_eckart_young():
    # d = 2: X = V D_nu V' is a PSD matrix; the best rank-r model is its top-r
    # eigenpairs (Eckart-Young), leaving f = sum of the other squared eigenvalues
    n, p, r = 9, 30, 3
    V = synth.rng(41).standard_normal((n, p))
    nu = synth.rng(42).random(p) + 0.05
    X = V @ np.diag(nu) @ V.T
    theta, Q = np.linalg.eigh(X)
    alpha = normx_implicit(V, nu, 2)
    assert alpha == pytest.approx(np.sum(theta**2), rel=1e-12)
    out = fg_implicit(V, nu, Q[:, -r:], theta[-r:], 2, alpha)
    assert out.f == pytest.approx(np.sum(theta[:-r] ** 2), rel=1e-9, abs=1e-12 * alpha)
    # it is a stationary point
    mag = magnitudes(V, nu, Q[:, -r:], theta[-r:], 2, alpha)
    assert np.all(np.abs(out.g_lambda) <= 1e-12 * mag.g_scale)
    assert np.all(np.abs(out.G_A) <= 1e-12 * mag.G_scale[None, :])


def test_optimal_lambda_zero_gradient():
    # for fixed A, f is quadratic in lambda with Hessian 2 B^{d}; its minimiser
    # solves B^{d} lambda = w, where g_lambda vanishes
    V, nu, A, _ = _case(8, 50, 4, 3, (51,))
    out0 = fg_implicit(V, nu, A, np.zeros(4), 3)
    lam_star = np.linalg.solve((A.T @ A) ** 3, out0.w)
    out = fg_implicit(V, nu, A, lam_star, 3)
    assert np.max(np.abs(out.g_lambda)) <= 1e-10 * np.max(np.abs(out0.w))


# --- derivatives of f ------------------------------------------------------

def test_lambda_central_difference_exact():
    # f is a quadratic in lambda, so a central difference with a large step is exact
    V, nu, A, lam = _case(6, 40, 3, 3, (61,))
    out = fg_implicit(V, nu, A, lam, 3)
    for j in range(3):
        e = np.zeros(3); e[j] = 1.0
        fd = (fg_implicit(V, nu, A, lam + e, 3).f - fg_implicit(V, nu, A, lam - e, 3).f) / 2.0
        assert fd == pytest.approx(out.g_lambda[j], rel=1e-12, abs=1e-13 * abs(out.f))


@pytest.mark.parametrize("d", [2, 3, 4])
def test_complex_step_gradient(d):
    # f is a real polynomial in A: Im f(A + i h E) / h = <G_A, E> to rounding
    V, nu, A, lam = _case(7, 30, 4, d, (71, d))
    out = fg_implicit(V, nu, A, lam, d)
    h = 1e-30
    for k in range(3):
        E = synth.rng(72, d, k).standard_normal(A.shape)
        fc = fg_implicit(V, nu, A + 1j * h * E, lam, d, with_intermediates=False).f
        assert np.imag(fc) / h == pytest.approx(np.sum(out.G_A * E), rel=1e-12)
    # and for lambda
    e = synth.rng(73, d).standard_normal(4)
    fc = fg_implicit(V, nu, A.astype(complex), lam + 1j * h * e, d, with_intermediates=False).f
    assert np.imag(fc) / h == pytest.approx(out.g_lambda @ e, rel=1e-12)


def test_central_difference_gradient():
    V, nu, A, lam = _case(5, 20, 3, 3, (81,))
    out = fg_implicit(V, nu, A, lam, 3)
    h = 1e-6
    for (i, j) in [(0, 0), (4, 2), (2, 1)]:
        E = np.zeros_like(A); E[i, j] = h
        fd = (fg_implicit(V, nu, A + E, lam, 3).f - fg_implicit(V, nu, A - E, lam, 3).f) / (2 * h)
        assert fd == pytest.approx(out.G_A[i, j], rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("d", [3, 4])
def test_column_identity(d):
    # a_j'(G_A)_{:,j} = d lambda_j (g_lambda)_j, from lines 3-9 of Algorithm 2
    V, nu, A, lam = _case(10, 60, 5, d, (91, d))
    out = fg_implicit(V, nu, A, lam, d)
    mag = magnitudes(V, nu, A, lam, d)
    lhs = np.sum(A * out.G_A, axis=0)
    assert np.all(np.abs(lhs - d * lam * out.g_lambda) <= 1e-12 * d * np.abs(lam) * mag.g_scale)


@pytest.mark.parametrize("d", [3, 4])
def test_gauges(d):
    V, nu, A, lam = _case(8, 40, 4, d, (101, d))
    alpha = normx_implicit(V, nu, d)
    f0 = fg_implicit(V, nu, A, lam, d, alpha).f
    c = np.array([2.0, 0.5, 3.0, -1.5])
    # scaling gauge: a_j -> c_j a_j, lambda_j -> c_j^{-d} lambda_j
    f1 = fg_implicit(V, nu, A * c, lam * c ** (-d), d, alpha).f
    assert f1 == pytest.approx(f0, rel=1e-12)
    # permutation of the components
    perm = [2, 0, 3, 1]
    assert fg_implicit(V, nu, A[:, perm], lam[perm], d, alpha).f == pytest.approx(f0, rel=1e-12)
    # sign of a_j: for odd d it flips the sign of component j, so f changes
    # unless lambda_j flips too
    s = np.array([-1.0, 1.0, 1.0, 1.0])
    f_sign = fg_implicit(V, nu, A * s, lam * s ** d, d, alpha).f
    assert f_sign == pytest.approx(f0, rel=1e-12)


# --- ||X||^2 -----------------------------------------------------------------

@pytest.mark.parametrize("n,p,d", [(3, 4, 2), (4, 9, 3), (3, 7, 4), (5, 6, 3), (2, 5, 6)])
def test_normx_implicit_vs_explicit(n, p, d):
    V, nu, _, _ = _case(n, p, 1, d, (111, n, p, d))
    assert normx_implicit(V, nu, d, block=3) == pytest.approx(normx_explicit(V, nu, d), rel=1e-12)


def test_normx_orthonormal():
    # orthonormal columns: V'V = I, so ||X||^2 = sum_l nu_l^2 for every d
    Q, _ = np.linalg.qr(synth.rng(121).standard_normal((20, 8)))
    nu = synth.rng(122).random(8)
    for d in (2, 3, 4, 7):
        assert normx_implicit(Q, nu, d) == pytest.approx(np.sum(nu**2), rel=1e-12)


# --- metrics -----------------------------------------------------------------

def test_score_assignment_vs_bruteforce():
    g = synth.rng(131)
    for r, rh in [(3, 3), (3, 5), (5, 3), (4, 6), (6, 2)]:
        M = g.standard_normal((10, r)); A = g.standard_normal((10, rh))
        assert score(M, A) == pytest.approx(score_bruteforce(M, A), rel=1e-12)


def test_score_exact_recovery():
    M = synth.unit_means(15, 5, 141)
    A = M[:, [3, 1, 4, 0, 2]] * np.array([2.0, -1.0, 0.3, 5.0, -7.0])
    assert score(M, A) == pytest.approx(1.0, abs=1e-14)
    assert score_bruteforce(M, A) == pytest.approx(1.0, abs=1e-14)


def test_model_distance_explicit():
    g = synth.rng(151)
    for d in (2, 3, 4):
        A1, A2 = g.standard_normal((4, 3)), g.standard_normal((4, 2))
        l1, l2 = g.standard_normal(3), g.standard_normal(2)
        D = T.kruskal(l1, A1, d) - T.kruskal(l2, A2, d)
        assert model_dist2(l1, A1, l2, A2, d) == pytest.approx(T.inner(D, D), rel=1e-11)
        assert model_norm2(l1, A1, d) == pytest.approx(T.inner(T.kruskal(l1, A1, d), T.kruskal(l1, A1, d)), rel=1e-12)


def test_rel_err():
    assert rel_err(4.0, 16.0) == 0.5
    assert rel_err(-1e-18, 1.0) == 0.0


def test_congruent_means():
    M = synth.unit_means(30, 6, 161, congruent=True)
    G = M.T @ M
    assert np.allclose(np.diag(G), 1.0, atol=1e-14)
    assert np.allclose(G[~np.eye(6, dtype=bool)], 0.5, atol=1e-14)
