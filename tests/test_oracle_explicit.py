"""Pins of Algorithm 1 (oracle.fg.fg_explicit) and of its comparison scales.

Algorithm 1 on an explicitly formed X = sum_l nu_l v_l^{(x)d} must give the
definition's f, g_lambda and G_A (brute-force differentiation of ||X - M||^2,
eqs. (optFunc), (gradl), (gradb)) and agree with Algorithm 2 (the paper
states the two are mathematically identical, Section 3.4); a symmetric X
that is not of moment form is handled too (checked against the brute-force
derivative of ||X - M||^2 with that X).  The explicit scales are recomputed
from their definition by loops, and are tight enough that a relative 1e-11
change of an output fails the 1e-12 bar.
"""

import itertools

import numpy as np
import pytest

from oracle import tensor as T
from oracle.fg import fg_bruteforce, fg_explicit, fg_implicit, magnitudes_explicit


def _case(seed, n=4, p=7, r=3, d=3):
    g = np.random.default_rng(seed)
    V = g.standard_normal((n, p))
    nu = g.uniform(0.1, 1.0, p)
    A = g.standard_normal((n, r))
    lam = g.standard_normal(r)
    return V, nu, A, lam, d


@pytest.mark.parametrize("seed,n,d,r", [(0, 4, 3, 3), (1, 3, 4, 2), (2, 5, 2, 4), (3, 2, 5, 2)])
def test_explicit_equals_definition_and_implicit(seed, n, d, r):
    V, nu, A, lam, d = _case(seed, n=n, d=d, r=r)
    X = T.kruskal(nu, V, d)
    alpha = T.inner(X, X)
    ex = fg_explicit(X, A, lam, d, alpha)
    bf = fg_bruteforce(V, nu, A, lam, d)
    im = fg_implicit(V, nu, A, lam, d, alpha)
    scale = abs(alpha) + abs(im.w @ lam) + abs(lam @ im.u)
    for o in (bf, im):
        assert abs(ex.f - o.f) <= 1e-12 * scale
        np.testing.assert_allclose(ex.g_lambda, o.g_lambda, rtol=1e-10, atol=1e-12 * scale)
        np.testing.assert_allclose(ex.G_A, o.G_A, rtol=1e-10, atol=1e-12 * scale)


def test_explicit_on_a_symmetric_tensor_not_of_moment_form():
    # symmetrise a random tensor; brute force differentiates ||X - M||^2 directly
    g = np.random.default_rng(9)
    n, d, r = 3, 3, 2
    Z = g.standard_normal((n,) * d)
    X = sum(np.transpose(Z, pm) for pm in itertools.permutations(range(d))) / 6.0
    A = g.standard_normal((n, r))
    lam = g.standard_normal(r)
    M = T.kruskal(lam, A, d)
    R = X - M
    f = T.inner(R, R)
    gl = np.array([-2.0 * T.inner(R, T.outer_power(A[:, j], d)) for j in range(r)])
    G = np.stack([-2.0 * d * lam[j] * T.ttsv_all_but_one(R, A[:, j]) for j in range(r)], axis=1)
    ex = fg_explicit(X, A, lam, d, T.inner(X, X))
    assert abs(ex.f - f) <= 1e-12 * (1 + abs(f))
    np.testing.assert_allclose(ex.g_lambda, gl, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(ex.G_A, G, rtol=1e-11, atol=1e-12)


def _scales_by_loops(X, A, lam, d, alpha):
    n, r = A.shape
    idx = list(itertools.product(range(n), repeat=d - 1))
    yabs = np.array([[sum(abs(X[(i,) + t]) * np.prod([abs(A[k, j]) for k in t]) for t in idx) for j in range(r)]
                     for i in range(n)])
    y = np.array([[sum(X[(i,) + t] * np.prod([A[k, j] for k in t]) for t in idx) for j in range(r)]
                  for i in range(n)])
    w = np.array([sum(A[i, j] * y[i, j] for i in range(n)) for j in range(r)])
    wabs = np.array([sum(abs(A[i, j]) * yabs[i, j] for i in range(n)) for j in range(r)])
    b = A.T @ A
    u = np.array([sum(b[j, k] ** d * lam[k] for k in range(r)) for j in range(r)])
    f_scale = abs(alpha) + abs(lam @ u) + 2 * abs(w @ lam)
    g_scale = np.array([2 * (wabs[j] + sum(abs(b[j, k]) ** d * abs(lam[k]) for k in range(r))) for j in range(r)])
    G_scale = np.array([2 * d * abs(lam[j]) * (max(yabs[:, j]) + max(
        sum(abs(A[i, k]) * abs(lam[k]) * abs(b[k, j]) ** (d - 1) for k in range(r)) for i in range(n)))
        for j in range(r)])
    return f_scale, g_scale, G_scale


@pytest.mark.parametrize("seed,d", [(4, 3), (5, 4)])
def test_explicit_scales_by_definition_and_tightness(seed, d):
    V, nu, A, lam, d = _case(seed, n=3, d=d, r=2)
    X = T.kruskal(nu, V, d)
    alpha = 0.7
    mag = magnitudes_explicit(X, A, lam, d, alpha)
    f_s, g_s, G_s = _scales_by_loops(X, A, lam, d, alpha)
    assert abs(mag.f_scale - f_s) <= 1e-13 * f_s
    np.testing.assert_allclose(mag.g_scale, g_s, rtol=1e-13)
    np.testing.assert_allclose(mag.G_scale, G_s, rtol=1e-13)
    ref = fg_explicit(X, A, lam, d, alpha)
    ratio = np.abs(ref.G_A) / mag.G_scale[None, :]
    assert 1e-11 * ratio.max() > 1e-12
    assert 1e-11 * np.max(np.abs(ref.g_lambda) / mag.g_scale) > 1e-12
