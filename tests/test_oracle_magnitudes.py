"""Pins of oracle.fg.magnitudes, the comparison scales of every parity test.

Each scale is the sum of the absolute values of the terms that cancel in
f, g_lambda or G_A (Algorithm 2, with w and u as in Lemmas 3.4 and 3.5).
Here they are recomputed from that definition with explicit Python loops
over every index, and the scales are shown to be tight enough that a
relative perturbation of 1e-11 in one output element fails the fp64 bar of
1e-12 (so a scale inflated by a slip, a sum for a max or a wrong power,
would be caught)."""

import numpy as np
import pytest

from oracle.fg import fg_implicit, magnitudes


def _case(seed, n=4, p=6, r=3, d=3):
    g = np.random.default_rng(seed)
    V = g.standard_normal((n, p))
    nu = g.uniform(0.1, 1.0, p) * g.choice([-1.0, 1.0], p)
    A = g.standard_normal((n, r))
    lam = g.standard_normal(r)
    return V, nu, A, lam, d, float(g.uniform(0.5, 2.0))


def _scales_by_loops(V, nu, A, lam, d, alpha):
    n, p = V.shape
    r = A.shape[1]
    z = [[sum(V[i, l] * A[i, j] for i in range(n)) for j in range(r)] for l in range(p)]
    b = [[sum(A[i, j] * A[i, k] for i in range(n)) for k in range(r)] for j in range(r)]
    # the cancelling terms of f: alpha, lambda'u = ||M||^2 and 2 w'lambda = 2 <X, M>
    w = [sum(nu[l] * z[l][j] ** d for l in range(p)) for j in range(r)]
    u = [sum(b[j][k] ** d * lam[k] for k in range(r)) for j in range(r)]
    f_scale = abs(alpha) + abs(sum(lam[j] * u[j] for j in range(r))) + 2 * abs(sum(w[j] * lam[j] for j in range(r)))
    # g_lambda[j] = -2 (w_j - u_j): every term of both sums, in absolute value
    g_scale = [2 * (sum(abs(nu[l]) * abs(z[l][j]) ** d for l in range(p))
                    + sum(abs(b[j][k]) ** d * abs(lam[k]) for k in range(r))) for j in range(r)]
    # G_A[:, j] = -2 d lambda_j (y_j - sum_k a_k lambda_k c_kj): the largest
    # absolute-term sum over the rows of each of the two parts
    G_scale = []
    for j in range(r):
        yabs = max(sum(abs(V[i, l]) * abs(nu[l]) * abs(z[l][j]) ** (d - 1) for l in range(p)) for i in range(n))
        mabs = max(sum(abs(A[i, k]) * abs(lam[k]) * abs(b[k][j]) ** (d - 1) for k in range(r)) for i in range(n))
        G_scale.append(2 * d * abs(lam[j]) * (yabs + mabs))
    return f_scale, np.array(g_scale), np.array(G_scale)


@pytest.mark.parametrize("seed,d", [(0, 3), (1, 4), (2, 2), (3, 5)])
def test_scales_match_their_definition(seed, d):
    V, nu, A, lam, d, alpha = _case(seed, d=d)
    mag = magnitudes(V, nu, A, lam, d, alpha)
    f_s, g_s, G_s = _scales_by_loops(V, nu, A, lam, d, alpha)
    assert abs(mag.f_scale - f_s) <= 1e-13 * f_s
    np.testing.assert_allclose(mag.g_scale, g_s, rtol=1e-13, atol=0)
    np.testing.assert_allclose(mag.G_scale, G_s, rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 4])
def test_scales_bound_the_outputs_tightly(seed):
    V, nu, A, lam, d, alpha = _case(seed)
    ref = fg_implicit(V, nu, A, lam, d, alpha)
    mag = magnitudes(V, nu, A, lam, d, alpha)
    # each output is at most its scale (triangle inequality) ...
    assert abs(ref.f) <= mag.f_scale
    assert np.all(np.abs(ref.g_lambda) <= mag.g_scale)
    assert np.all(np.abs(ref.G_A) <= mag.G_scale[None, :])
    # ... and a relative 1e-11 change of the largest output element fails
    # the 1e-12 bar: the scales are not vacuously large
    tol = 1e-12
    assert 1e-11 * abs(ref.f) / mag.f_scale > tol
    j = int(np.argmax(np.abs(ref.g_lambda) / mag.g_scale))
    assert 1e-11 * abs(ref.g_lambda[j]) / mag.g_scale[j] > tol
    ratio = np.abs(ref.G_A) / mag.G_scale[None, :]
    i, j = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    G = ref.G_A.copy()
    G[i, j] *= 1 + 1e-11
    assert np.max(np.abs(G - ref.G_A) / mag.G_scale[None, :]) > tol


def test_scales_at_an_exact_fit_are_the_cancelling_sizes():
    # at A = V, lambda = nu (r = p) f = g = 0 exactly, but the scales keep the
    # size of the cancelling terms: f_scale = 4 alpha and g_scale = 4 w
    V, nu, _, _, d, _ = _case(5, n=5, p=3, r=3)
    nu = np.abs(nu)
    alpha = float(nu @ (V.T @ V) ** d @ nu)
    mag = magnitudes(V, nu, V, nu, d, alpha)
    assert abs(mag.f_scale - 4 * alpha) <= 1e-13 * alpha
    w = ((V.T @ V) ** d) @ nu
    if d % 2 == 1:
        w = (np.abs(V.T @ V) ** d) @ nu
    np.testing.assert_allclose(mag.g_scale, 4 * w, rtol=1e-13)
