"""Parity of symtd_normX (||X||^2 on fp64 matrix cores) with the oracle."""

import numpy as np
import pytest

import synth
from helpers import gpu_available, stored, to_dev
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


def gpu_alpha(ctx, V, nu, d, kind):
    dt = torch.float64 if kind == "f64" else torch.float32
    a = S.symtd_normX(ctx, to_dev(V, dt), to_dev(nu, torch.float64), d)
    torch.cuda.synchronize()
    return float(a.cpu()[0])


@pytest.mark.parametrize("n,p,d", [(1, 1, 3), (10, 750, 3), (7, 129, 2), (33, 300, 4), (100, 5000, 4),
                                   (257, 1000, 5), (1000, 4000, 3), (40, 600, 11), (40, 600, 16),
                                   # 2 to 6 steps of 16 covariates: every exit of the three-deep load ring
                                   (17, 300, 3), (48, 200, 3), (49, 200, 3), (64, 130, 4), (80, 250, 4),
                                   (96, 260, 3)])
@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_normx_parity(ctx, n, p, d, kind):
    print(f"case n={n} p={p} d={d} kind={kind}", flush=True)
    V, nu, _ = synth.gmm(n, 3, p, 1e-1, 11, n, p)
    V = stored(V, kind)
    ref = normx_implicit(V, nu, d)
    got = gpu_alpha(ctx, V, nu, d, kind)
    # all terms are positive for even d; for odd d compare against the sum of |terms|
    scale = normx_implicit(np.abs(V), nu, d)
    assert abs(got - ref) <= 1e-12 * scale, (got, ref)


def test_normx_duplicated_columns(ctx):
    # X is unchanged when every observation is split into two copies of half weight
    V, nu, _ = synth.gmm(200, 5, 3000, 1e-2, 12)
    a1 = gpu_alpha(ctx, V, nu, 3, "f64")
    a2 = gpu_alpha(ctx, np.hstack([V, V]), np.concatenate([nu, nu]) / 2, 3, "f64")
    assert a2 == pytest.approx(a1, rel=1e-12)


def test_normx_full_shape(ctx):
    # the benchmark's data set (d=3, n=1000, p=1e5, fp32 storage) against the
    # oracle's value stored by tests/golden/make_normx_full.py
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "normx_gmm_n1000_p1e5_d3.json")) as fh:
        g = json.load(fh)
    w = g["workload"]
    print(f"case normx full shape n={w['n']} p={w['p']} d={w['d']}", flush=True)
    V, nu, _ = synth.gmm(w["n"], w["r"], w["p"], w["sigma"], w["synth_key"])
    got = gpu_alpha(ctx, V, nu, w["d"], "f32")
    assert abs(got - g["value"]) <= 1e-12 * g["scale_abs"], (got, g["value"])
