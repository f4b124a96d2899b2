"""Pins of the 16-bit rounding model (tests/lowprec_model.py) and proof that
the per-shape bounds the GPU parity tests use can tell the fp16 and bf16x3
paths from their broken variants: a single bf16 plane (no hi/lo split) and
fp16 without the power-of-two prescale of W."""

import numpy as np
import pytest

import lowprec_model as L
from helpers import make_case
from oracle.fg import fg_implicit, magnitudes
from oracle.normx import normx_implicit


def test_bf16_rounding_is_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                        # bf16 spacing in [1, 2)
    assert L.bf16(one + ulp / 2)[()] == one                  # tie, to the even neighbour 1
    assert L.bf16(one + 3 * ulp / 2)[()] == one + 2 * ulp    # tie, to the even neighbour 1 + 2 ulp
    assert L.bf16(one + ulp / 2 + 2.0 ** -20)[()] == one + ulp
    assert L.bf16(-(one + ulp / 2 + 2.0 ** -20))[()] == -(one + ulp)
    assert L.bf16(3.0)[()] == 3.0
    # the largest relative rounding error is half a unit in the last place
    x = np.random.default_rng(0).uniform(-8, 8, 100_000).astype(np.float32).astype(np.float64)
    assert np.max(np.abs(L.bf16(x) - x) / np.abs(x)) <= 2.0 ** -8


def test_fp16_keeps_subnormals():
    assert L.fp16(2.0 ** -20)[()] == 2.0 ** -20               # subnormal in binary16
    assert L.fp16(2.0 ** -26)[()] == 0.0                      # below half the smallest subnormal
    assert L.fp16(1.0 + 2.0 ** -11)[()] == 1.0                # tie to even
    assert L.fp16(1.0 + 3 * 2.0 ** -11)[()] == 1.0 + 2.0 ** -9


def test_split_carries_sixteen_bits():
    x = np.random.default_rng(1).standard_normal(100_000).astype(np.float32).astype(np.float64)
    hi, lo = L._split(x)
    assert np.array_equal(hi, L.bf16(x))
    rel = np.abs(hi + lo - x) / np.abs(x)
    assert np.max(rel) <= 2.0 ** -16
    assert np.max(np.abs(hi - x) / np.abs(x)) > 2.0 ** -10    # one plane alone is much coarser


def test_wscale_brings_nu_into_one_two():
    for nu_max in (1e-5, 1.0 / 750, 0.3, 1.0, 7.5):
        s = L.wscale_of(np.array([nu_max / 3, nu_max]))
        assert 1.0 <= s * nu_max < 2.0
        assert np.log2(s) == np.round(np.log2(s))


def test_exact_inputs_have_no_model_error():
    # values with few significant bits (and, with d = 2, W = nu z too) are
    # stored exactly by both formats, so every model equals the oracle up to
    # fp64 rounding
    rng = np.random.default_rng(2)
    n, p, r, d = 6, 9, 2, 2
    V = rng.integers(-3, 4, (n, p)) / 4.0
    A = rng.integers(-3, 4, (n, r)) / 2.0
    nu = np.full(p, 0.25)
    lam = np.array([0.5, -1.0])
    ref = fg_implicit(V, nu, A, lam, d, 1.0)
    mag = magnitudes(V, nu, A, lam, d, 1.0)
    for mode in L.MODES:
        assert np.all(L.model_errors(V, nu, A, lam, d, 1.0, mode, ref, mag) <= 1e-15), mode


# shapes of the GPU parity sweep where the broken variants must fail
DISCRIMINATING = [(100, 5000, 20, 4, (2,)), (257, 4099, 7, 3, (3, 257, 4099, 7, 3)),
                  (200, 6000, 100, 3, (3, 200, 6000, 100, 3))]


def _case(n, p, r, d, key):
    V, nu, A, lam = make_case(n, p, r, d, key, 1e-2, "f32")
    alpha = normx_implicit(V, nu, d)
    return V, nu, A, lam, alpha, fg_implicit(V, nu, A, lam, d, alpha), magnitudes(V, nu, A, lam, d, alpha)


@pytest.mark.parametrize("n,p,r,d,key", DISCRIMINATING)
def test_bf16x3_bound_rejects_single_plane(n, p, r, d, key):
    V, nu, A, lam, alpha, ref, mag = _case(n, p, r, d, key)
    bound, e_plain = L.bounds(V, nu, A, lam, d, alpha, "bf16x3", ref, mag)
    e_split = L.model_errors(V, nu, A, lam, d, alpha, "bf16x3", ref, mag)
    assert np.any(e_plain > bound), (e_plain, bound)          # no split: fails
    assert np.all(e_split <= 0.5 * bound), (e_split, bound)   # the split: passes with room


@pytest.mark.parametrize("n,p,r,d,key", [c for c in DISCRIMINATING if c[1] >= 5000])
def test_fp16_bound_rejects_unscaled_w(n, p, r, d, key):
    V, nu, A, lam, alpha, ref, mag = _case(n, p, r, d, key)
    bound, e_path = L.bounds(V, nu, A, lam, d, alpha, "fp16", ref, mag)
    e_noscale = L.model_errors(V, nu, A, lam, d, alpha, "fp16_noscale", ref, mag)
    assert np.any(e_noscale > bound), (e_noscale, bound)
    assert np.all(e_path <= bound)
