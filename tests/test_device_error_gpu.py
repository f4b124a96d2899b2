"""Device-side errors of asynchronous evaluations surface as SYMTD_EDEVICE.

The first product splits slabs between neighbouring blocks (stream-K); the
block finishing a shared slab waits, bounded by a spin limit, for its
neighbour's partial.  SYMTD_TUNE_FAULT_HANDOFF makes every such wait watch
for a flag value no block writes, so each runs out a small spin limit and
gives up, as it would if a partial never arrived; every kernel still exits
normally.  The call itself returns at once (it is asynchronous); the
give-up must then be reported by symtd_check and by the next call, after
which evaluations are correct again.
"""

import numpy as np
import pytest

from helpers import TOL, compare_fg, gpu_available, make_case, to_dev

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_1911_03813_amd as S


@pytest.fixture()
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    c = S.Context(0)
    yield c
    c.close()


def _inputs(kind, dt):
    # 391 slabs of 128 observations over 256 blocks: many slabs are shared
    n, p, r, d = 200, 50_000, 20, 3
    V, nu, A, lam = make_case(n, p, r, d, (40,), 1e-2, kind)
    dev = (to_dev(V, dt), to_dev(nu, torch.float64), to_dev(A, dt), to_dev(lam, torch.float64))
    return (V, nu, A, lam, d), dev


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_give_up_is_reported_then_cleared(ctx, kind):
    dt = torch.float64 if kind == "f64" else torch.float32
    (V, nu, A, lam, d), (Vd, nud, Ad, ld) = _inputs(kind, dt)
    print(f"case give-up {kind}: n={V.shape[0]} p={V.shape[1]}", flush=True)
    S.symtd_set_tuning(ctx, S.TUNE_SPIN_LIMIT, 64)
    S.symtd_set_tuning(ctx, S.TUNE_FAULT_HANDOFF, 1)
    S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 1.0)            # returns before the device has run it
    S.symtd_set_tuning(ctx, S.TUNE_FAULT_HANDOFF, 0)
    with pytest.raises(S.SymtdError) as e:
        S.symtd_check(ctx)
    assert e.value.status == -4
    assert "hand-off" in str(e.value)
    S.symtd_check(ctx)                                  # the record was cleared
    S.symtd_set_tuning(ctx, S.TUNE_SPIN_LIMIT, 0)
    out = S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 1.0)
    S.symtd_check(ctx)
    got = (float(out[0].cpu()[0]), out[1].cpu().numpy(), out[2].cpu().double().numpy())
    errs = compare_fg(got, V, nu, A, lam, d, 1.0, kind)
    assert max(errs) <= TOL[kind], errs


def test_next_call_reports_the_give_up(ctx):
    (V, nu, A, lam, d), (Vd, nud, Ad, ld) = _inputs("f32", torch.float32)
    S.symtd_set_tuning(ctx, S.TUNE_SPIN_LIMIT, 64)
    S.symtd_set_tuning(ctx, S.TUNE_FAULT_HANDOFF, 1)
    S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 1.0)
    S.symtd_set_tuning(ctx, S.TUNE_FAULT_HANDOFF, 0)
    S.symtd_set_tuning(ctx, S.TUNE_SPIN_LIMIT, 0)
    torch.cuda.synchronize()                            # the device has recorded the give-up
    with pytest.raises(S.SymtdError) as e:
        S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 1.0)        # refused, nothing launched
    assert e.value.status == -4
    out = S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 1.0)      # and the call after it is correct
    torch.cuda.synchronize()
    got = (float(out[0].cpu()[0]), out[1].cpu().numpy(), out[2].cpu().double().numpy())
    assert max(compare_fg(got, V, nu, A, lam, d, 1.0, "f32")) <= TOL["f32"]


def test_sixteen_bit_product_reports_the_give_up(ctx):
    (V, nu, A, lam, d), (Vd, nud, Ad, ld) = _inputs("f32", torch.float32)
    data = S.Data(ctx, Vd, nud, S.PREC_FP16)
    try:
        S.symtd_set_tuning(ctx, S.TUNE_SPIN_LIMIT, 64)
        S.symtd_set_tuning(ctx, S.TUNE_FAULT_HANDOFF, 1)
        data.fg(Ad, ld, d, 1.0)
        S.symtd_set_tuning(ctx, S.TUNE_FAULT_HANDOFF, 0)
        S.symtd_set_tuning(ctx, S.TUNE_SPIN_LIMIT, 0)
        with pytest.raises(S.SymtdError):
            S.symtd_check(ctx)
        data.fg(Ad, ld, d, 1.0)
        S.symtd_check(ctx)
    finally:
        data.close()
