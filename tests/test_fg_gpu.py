"""Parity of symtd_fg (the HIP path, through the C ABI) with the fp64 oracle.

Every case compares f, g_lambda and G_A element by element with
oracle.fg.fg_implicit on the same stored inputs, relative to the magnitudes
of the terms that cancel (oracle.fg.magnitudes): 1e-12 for fp64 products,
1e-5 for fp32 products.
"""

import numpy as np
import pytest

import synth
from helpers import TOL, compare_fg, gpu_available, make_case, stored, to_dev
from oracle.normx import normx_implicit

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


def run_fg(ctx, V, nu, A, lam, d, alpha, kind, ldv_pad=0):
    dt = torch.float64 if kind == "f64" else torch.float32
    n, p = V.shape
    if ldv_pad:
        big = to_dev(np.vstack([V, np.zeros((ldv_pad, p))]), dt)
        Vd = big[:n, :]
    else:
        Vd = to_dev(V, dt)
    f, g, G = S.symtd_fg(ctx, Vd, to_dev(nu, torch.float64), to_dev(A, dt), to_dev(lam, torch.float64), d, alpha)
    torch.cuda.synchronize()
    return float(f.cpu()[0]), g.cpu().numpy(), G.cpu().numpy().astype(np.float64)


def check(ctx, n, p, r, d, key, kind, sigma=1e-2, alpha=None, ldv_pad=0):
    V, nu, A, lam = make_case(n, p, r, d, key, sigma, kind)
    if alpha is None:
        alpha = normx_implicit(V, nu, d) if p <= 20000 else 0.0
    print(f"case n={n} p={p} r={r} d={d} kind={kind} ldv_pad={ldv_pad}", flush=True)
    got = run_fg(ctx, V, nu, A, lam, d, alpha, kind, ldv_pad)
    ef, eg, eG = compare_fg(got, V, nu, A, lam, d, alpha, kind)
    print(f"  errors f={ef:.2e} g_lambda={eg:.2e} G_A={eG:.2e}", flush=True)
    tol = TOL[kind]
    assert ef <= tol and eg <= tol and eG <= tol, (ef, eg, eG)
    return ef, eg, eG


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_small_config(ctx, kind):
    # d=3, n=10, r=3, p=750 (Gaussian mixture, sigma=1e-2)
    check(ctx, 10, 750, 3, 3, (1,), kind)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_mid_config(ctx, kind):
    # d=4, n=100, r=20, p=5000
    check(ctx, 100, 5000, 20, 4, (2,), kind)


@pytest.mark.parametrize("n,p,r,d", [
    (1, 1, 1, 3), (1, 7, 2, 2), (3, 1, 1, 4), (5, 17, 16, 3), (17, 33, 5, 2),
    (31, 129, 17, 5), (64, 256, 32, 3), (130, 1000, 33, 4), (257, 4099, 7, 6),
    (96, 3000, 112, 3), (40, 2000, 129, 3), (200, 6000, 100, 3),
])
@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_shape_sweep(ctx, n, p, r, d, kind):
    # ragged sizes that are not multiples of any tile, several column groups
    check(ctx, n, p, r, d, (3, n, p, r, d), kind)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_unaligned_leading_dimension(ctx, kind):
    # ldv = n + 1 takes the scalar-load path
    check(ctx, 50, 1500, 9, 3, (4,), kind, ldv_pad=1)
    check(ctx, 64, 700, 20, 4, (5,), kind, ldv_pad=3)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 8, 11, 16])   # 16: the largest order the library takes
def test_orders(ctx, d):
    check(ctx, 48, 2500, 12, d, (6, d), "f64")
    check(ctx, 48, 2500, 12, d, (6, d), "f32")


@pytest.mark.parametrize("r", [1, 2, 3, 4, 18, 35, 52, 100, 116, 5, 21])
def test_narrow_last_subtile(ctx, r):
    # fp64: a last column subtile with r mod 16 in 1..4 factor columns runs on
    # the 4x4x4 form in both products (r = 116: the second column group is that
    # subtile alone); r = 5 and 21 take the 16x16x4 form throughout
    check(ctx, 70, 3000, r, 3, (12, r), "f64")
    check(ctx, 33, 1001, r, 4, (13, r), "f64")


def test_exact_solution(ctx):
    # r = p, A = V, lambda = nu: f = 0 and the gradient vanishes
    n, p, d = 12, 40, 3
    V = synth.rng(7).standard_normal((n, p))
    nu = np.full(p, 1.0 / p)
    alpha = normx_implicit(V, nu, d)
    f, g, G = run_fg(ctx, V, nu, V.copy(), nu.copy(), d, alpha, "f64")
    assert abs(f) <= 1e-12 * alpha
    assert np.max(np.abs(g)) <= 1e-12 * alpha
    assert np.max(np.abs(G)) <= 1e-10 * alpha


def test_large_config_fp32(ctx):
    # d=3, n=1000, r=100, p=100000 (the large single-instance shape), in the
    # launch configuration the benchmark times; full element-wise comparison
    check(ctx, 1000, 100_000, 100, 3, (8,), "f32", alpha=0.0)


def test_large_config_fp64(ctx):
    check(ctx, 1000, 100_000, 100, 3, (8,), "f64", alpha=0.0)


@pytest.mark.parametrize("waves,splits", [(1, 1), (2, 3), (3, 7), (7, 2), (64, 5), (1000, 100)])
@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_work_splits(ctx, waves, splits, kind):
    # every split of the first product over waves (with partial hand-offs
    # between neighbours) and of the second over observation ranges gives the
    # same result to rounding
    try:
        S.symtd_set_tuning(ctx, S.TUNE_G1_BLOCKS, waves)
        S.symtd_set_tuning(ctx, S.TUNE_G2_SPLITS, splits)
        check(ctx, 70, 3000, 40, 3, (10, waves), kind)
        check(ctx, 33, 777, 9, 4, (11, waves), kind)
    finally:
        S.symtd_set_tuning(ctx, S.TUNE_G1_BLOCKS, 0)
        S.symtd_set_tuning(ctx, S.TUNE_G2_SPLITS, 0)


def test_deterministic(ctx):
    V, nu, A, lam = make_case(300, 20000, 40, 3, (9,), kind="f32")
    a = run_fg(ctx, V, nu, A, lam, 3, 0.0, "f32")
    b = run_fg(ctx, V, nu, A, lam, 3, 0.0, "f32")
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_bad_arguments(ctx):
    V = to_dev(np.ones((4, 5)), torch.float64)
    nu = to_dev(np.ones(5), torch.float64)
    A = to_dev(np.ones((4, 2)), torch.float64)
    lam = to_dev(np.ones(2), torch.float64)
    with pytest.raises(S.SymtdError) as e:
        S.symtd_fg(ctx, V, nu, A, lam, 1)
    assert e.value.status == -1 and "order" in str(e.value)
    with pytest.raises(S.SymtdError):
        S.symtd_fg(ctx, V, nu, A, lam, 3, prec=S.PREC_FP32)   # fp64 storage with fp32 products


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("n,p,r,models", [(300, 20000, 40, 1), (37, 3000, 5, 3), (130, 9000, 17, 4),
                                          (1000, 30000, 100, 1)])
def test_alternating_inputs(ctx, kind, n, p, r, models):
    """Two different factor sets evaluated in turn, three times each: every
    call gives the bits of that set's first call.  The closing kernel's last
    column block of each model writes f on an arrival counter that must be
    back at zero after every launch; a stale f would show the other set's
    value."""
    d = 3
    dt = torch.float64 if kind == "f64" else torch.float32
    V, nu, _ = synth.gmm(n, r, p, 1e-2, 61, n)
    V = stored(V, kind)
    Vd, nud = to_dev(V, dt), to_dev(nu, torch.float64)
    sets = []
    for k in range(2):
        A = stored(synth.gauss_factors(n, r * models, 62, n, k), kind)
        lam = synth.gauss_factors(r * models, 1, 63, n, k)[:, 0] + 0.5
        sets.append((to_dev(A, dt), to_dev(lam, torch.float64)))
    print(f"case n={n} p={p} r={r} models={models} kind={kind}", flush=True)

    def once(k):
        f, g, G = S.symtd_fg_multi(ctx, Vd, nud, sets[k][0], sets[k][1], r, d, 1.5)
        torch.cuda.synchronize()
        return f.cpu().numpy(), g.cpu().numpy(), G.cpu().numpy()

    first = [once(0), once(1)]
    assert not np.array_equal(first[0][0], first[1][0])
    for _ in range(3):
        for k in range(2):
            got = once(k)
            for x, y in zip(got, first[k]):
                assert np.array_equal(x, y)
