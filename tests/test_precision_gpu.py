"""Parity of the fp16 and bf16x3 product paths (data handles) with the fp64
oracle.  Errors are relative to the cancelling terms (oracle.fg.magnitudes),
per quantity (f, g_lambda, G_A), and the bound of each is set per shape from
a CPU model of the path's operand roundings (tests/lowprec_model.py):

* bf16x3: a tenth of the error of a single bf16 plane (no hi/lo split);
* fp16:   four times the model of the path itself (W prescaled by 2^s);

both at least 1e-7.  tests/test_lowprec_model.py shows on the CPU that the
model of a path without the split, or without the prescale, fails these
bounds at the shapes where the feature matters.  The oracle evaluates the
stored fp32 inputs; the 16-bit rounding of V, A and W is part of the path's
error.  The header's worst-case bounds (bf16x3 2 (d+1) 3 2^-16, fp16
2 (d+1) 2 2^-11) are checked as well.
"""

import numpy as np
import pytest

import lowprec_model as LPM
from helpers import gpu_available, make_case, to_dev
from oracle.fg import fg_implicit, magnitudes
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


def run(ctx, n, p, r, d, key, prec, sigma=1e-2, alpha=None):
    V, nu, A, lam = make_case(n, p, r, d, key, sigma, "f32")
    if alpha is None:
        alpha = normx_implicit(V, nu, d) if p <= 20000 else 0.0
    print(f"case n={n} p={p} r={r} d={d} prec={prec}", flush=True)
    data = S.Data(ctx, to_dev(V, torch.float32), to_dev(nu, torch.float64), prec)
    f, g, G = data.fg(to_dev(A, torch.float32), to_dev(lam, torch.float64), d, alpha)
    torch.cuda.synchronize()
    got = (float(f.cpu()[0]), g.cpu().numpy(), G.cpu().numpy().astype(np.float64))
    data.close()
    ref = fg_implicit(V, nu, A, lam, d, alpha)
    mag = magnitudes(V, nu, A, lam, d, alpha)
    err = np.array([abs(got[0] - ref.f) / mag.f_scale,
                    np.max(np.abs(got[1] - ref.g_lambda) / mag.g_scale),
                    np.max(np.abs(got[2] - ref.G_A) / mag.G_scale[None, :])])
    kind = "bf16x3" if prec == S.PREC_BF16X3 else "fp16"
    bound, e_model = LPM.bounds(V, nu, A, lam, d, alpha, kind, ref, mag)
    fmt = lambda v: "/".join(f"{x:.2e}" for x in v)  # noqa: E731
    print(f"  errors f/g/G {fmt(err)}  bound {fmt(bound)}  model ({'bf16' if kind == 'bf16x3' else kind}) "
          f"{fmt(e_model)}", flush=True)
    assert np.all(err <= bound), (err, bound)
    assert np.all(err <= S.prec_bound(prec, d))
    return err


PRECS = ["bf16x3", "fp16"]


def prec_of(name):
    return S.PREC_BF16X3 if name == "bf16x3" else S.PREC_FP16


@pytest.mark.parametrize("name", PRECS)
def test_small_and_mid(ctx, name):
    run(ctx, 10, 750, 3, 3, (1,), prec_of(name))
    run(ctx, 100, 5000, 20, 4, (2,), prec_of(name))


@pytest.mark.parametrize("n,p,r,d", [
    (1, 1, 1, 3), (3, 7, 2, 2), (17, 33, 5, 3), (64, 129, 16, 3), (130, 1000, 33, 4),
    (257, 4099, 7, 3), (96, 3000, 112, 3), (40, 2000, 129, 3), (200, 6000, 100, 3),
])
@pytest.mark.parametrize("name", PRECS)
def test_shape_sweep(ctx, name, n, p, r, d):
    run(ctx, n, p, r, d, (3, n, p, r, d), prec_of(name))


@pytest.mark.parametrize("name", PRECS)
def test_large(ctx, name):
    # d=3, n=1000, r=100, p=100000: the large single-instance shape
    run(ctx, 1000, 100_000, 100, 3, (8,), prec_of(name), alpha=0.0)


def test_fp32_handle_forwards(ctx):
    V, nu, A, lam = make_case(50, 1500, 9, 3, (4,), 1e-2, "f32")
    Vd, nud = to_dev(V, torch.float32), to_dev(nu, torch.float64)
    Ad, ld = to_dev(A, torch.float32), to_dev(lam, torch.float64)
    data = S.Data(ctx, Vd, nud, S.PREC_FP32)
    a = data.fg(Ad, ld, 3, 0.5)
    b = S.symtd_fg(ctx, Vd, nud, Ad, ld, 3, 0.5)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    data.close()


@pytest.mark.parametrize("name", PRECS)
@pytest.mark.parametrize("n,p,r", [(130, 9000, 17), (1000, 30000, 100)])
def test_alternating_inputs(ctx, name, n, p, r):
    """Two different factor sets evaluated in turn on one data handle: every
    call gives the bits of that set's first call (the closing kernel's
    arrival counter is back at zero after every launch)."""
    V, nu, A0, lam0 = make_case(n, p, r, 3, (9, n), 1e-2, "f32")
    _, _, A1, lam1 = make_case(n, p, r, 3, (10, n), 1e-2, "f32")
    print(f"case n={n} p={p} r={r} prec={name}", flush=True)
    data = S.Data(ctx, to_dev(V, torch.float32), to_dev(nu, torch.float64), prec_of(name))
    sets = [(to_dev(A0, torch.float32), to_dev(lam0, torch.float64)),
            (to_dev(A1, torch.float32), to_dev(lam1, torch.float64))]
    try:
        def once(k):
            out = data.fg(sets[k][0], sets[k][1], 3, 2.0)
            torch.cuda.synchronize()
            return [x.cpu().numpy() for x in out]

        first = [once(0), once(1)]
        assert not np.array_equal(first[0][0], first[1][0])
        for _ in range(3):
            for k in range(2):
                for x, y in zip(once(k), first[k]):
                    assert np.array_equal(x, y)
    finally:
        data.close()
