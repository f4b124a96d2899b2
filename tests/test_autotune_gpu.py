"""The tuning table on the device: a table entry sets an evaluation's launch
shape exactly as the equivalent context override does (the same bits), an
instance of the grouped evaluation gives the same bits alone and in a mix
under a fixed table, tuned shapes keep parity with the oracle, and the
autotuners return shapes from their candidate sets."""

import numpy as np
import pytest

from helpers import TOL, compare_fg, gpu_available, make_case, to_dev

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_1911_03813_amd as S
    from paper_1911_03813_amd import autotune as AT


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    c = S.Context(0)
    AT.clear()
    yield c
    AT.clear()
    c.close()


def _bits(out):
    torch.cuda.synchronize()
    return [x.cpu().clone() for x in out]


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_table_entry_acts_like_the_override(ctx, kind):
    dt = torch.float64 if kind == "f64" else torch.float32
    n, p, r, d = 200, 50_000, 20, 3
    case = make_case(n, p, r, d, (110,), 1e-2, kind)
    Vd, nud, Ad, ld = to_dev(case[0], dt), to_dev(case[1], torch.float64), to_dev(case[2], dt), \
        to_dev(case[3], torch.float64)
    AT.clear()
    base = _bits(S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 0.5))
    prec = S.PREC_FP64 if kind == "f64" else S.PREC_FP32
    AT.put(dict(kind=AT.KIND_FG, prec=prec, n_bucket=AT.bucket(n), p_bucket=AT.bucket(p), r_bucket=AT.bucket(r),
                v0=64, v1=7, us=0.0))
    tuned = _bits(S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 0.5))
    assert all(torch.equal(x, y) for x, y in zip(tuned, _bits(S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 0.5))))
    AT.clear()
    S.symtd_set_tuning(ctx, S.TUNE_G1_BLOCKS, 64)
    S.symtd_set_tuning(ctx, S.TUNE_G2_SPLITS, 7)
    forced = _bits(S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 0.5))
    S.symtd_set_tuning(ctx, S.TUNE_G1_BLOCKS, 0)
    S.symtd_set_tuning(ctx, S.TUNE_G2_SPLITS, 0)
    assert all(torch.equal(x, y) for x, y in zip(tuned, forced))
    assert all(torch.equal(x, y) for x, y in zip(base, _bits(S.symtd_fg(ctx, Vd, nud, Ad, ld, d, 0.5))))
    got = (float(tuned[0][0]), tuned[1].numpy(), tuned[2].double().numpy())
    assert max(compare_fg(got, *case, d, 0.5, kind)) <= TOL[kind]


def test_grouped_alone_equals_mix_under_a_table(ctx):
    shapes = [(60, 2000, 4, 3), (120, 1500, 6, 4), (33, 700, 3, 3)]
    items, host = [], []
    for k, (n, p, r, d) in enumerate(shapes):
        case = make_case(n, p, r, d, (111, k), 1e-2, "f32")
        Vd, nud = to_dev(case[0], torch.float32), to_dev(case[1], torch.float64)
        Ad, ld = to_dev(case[2], torch.float32), to_dev(case[3], torch.float64)
        items.append(dict(V=Vd, nu=nud, A=Ad, lam=ld, r=r, d=d, alpha=0.25))
        host.append((case, d))
    AT.clear()
    default = [_bits(o) for o in S.symtd_fg_batched(ctx, items)]
    # a table entry for the first instance's bucket: 4-block splits
    n, p, r, d = shapes[0]
    AT.put(dict(kind=AT.KIND_GROUPED, prec=S.PREC_FP32, n_bucket=AT.bucket(n), p_bucket=AT.bucket(p),
                r_bucket=AT.bucket(r), v0=4, v1=0, us=0.0))
    mix = [_bits(o) for o in S.symtd_fg_batched(ctx, items)]
    alone = _bits(S.symtd_fg_batched(ctx, items[:1])[0])
    assert all(torch.equal(x, y) for x, y in zip(mix[0], alone))
    for k in (1, 2):     # instances of other buckets keep their default shape
        assert all(torch.equal(x, y) for x, y in zip(mix[k], default[k]))
    for out, (case, dd) in zip(mix, host):
        got = (float(out[0][0]), out[1].numpy(), out[2].double().numpy())
        assert max(compare_fg(got, *case, dd, 0.25, "f32")) <= TOL["f32"]
    AT.clear()


def test_tuners_pick_from_their_candidates(ctx):
    AT.clear()
    n, p, r, d = 100, 5000, 20, 4
    case = make_case(n, p, r, d, (112,), 1e-2, "f64")
    e = AT.tune_fg(ctx, to_dev(case[0], torch.float64), to_dev(case[1], torch.float64),
                   to_dev(case[2], torch.float64), to_dev(case[3], torch.float64), d, reps=3)
    assert e["kind"] == AT.KIND_FG and e["v0"] >= 1 and e["v1"] >= 1 and e["us"] > 0
    assert e["n_bucket"] == AT.bucket(n) and e["p_bucket"] == AT.bucket(p) and e["r_bucket"] == AT.bucket(r)
    g = AT.tune_grouped(ctx, to_dev(case[0].astype(np.float32), torch.float32), to_dev(case[1], torch.float64), d,
                        40, copies=8, reps=2)
    assert g["kind"] == AT.KIND_GROUPED and g["v0"] in (4, 8, 16, 32, 64)
    assert len(AT.entries()) == 2
    AT.clear()
