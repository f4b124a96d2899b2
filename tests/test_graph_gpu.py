"""Evaluations captured in a graph and replayed.

The first product's hand-off between neighbouring blocks is tagged with a
launch epoch that the device itself advances, so replays of a captured
evaluation (where every launch argument is frozen) never take a flag left
by the previous replay for their own.  Every replay, with eager
evaluations of other inputs in between, must give the eager result's bits;
this holds for symtd_fg and for symtd_fg_noalloc, the entry point meant for
capture.
"""

import numpy as np
import pytest

from helpers import gpu_available, make_case, to_dev

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


def _dev(case, dt):
    V, nu, A, lam = case
    return to_dev(V, dt), to_dev(nu, torch.float64), to_dev(A, dt), to_dev(lam, torch.float64)


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("noalloc", [False, True])
def test_replays_equal_eager(ctx, kind, noalloc):
    dt = torch.float64 if kind == "f64" else torch.float32
    # 391 slabs over 256 blocks: shared slabs, so the hand-off runs
    n, p, r, d = 200, 50_000, 20, 3
    print(f"case graph {kind} noalloc={noalloc}", flush=True)
    Vd, nud, Ad, ld = _dev(make_case(n, p, r, d, (80,), 1e-2, kind), dt)
    _, _, A2, l2 = _dev(make_case(n, p, r, d, (81,), 1e-2, kind), dt)
    fg = S.symtd_fg_noalloc if noalloc else S.symtd_fg
    out = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty(r, dtype=torch.float64, device="cuda"),
           S.colmajor(torch.empty(n, r, dtype=dt, device="cuda")))
    other = tuple(torch.empty_like(x) for x in out)
    fg(ctx, Vd, nud, Ad, ld, d, 0.5, out=out)
    torch.cuda.synchronize()
    ref = [x.clone() for x in out]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fg(ctx, Vd, nud, Ad, ld, d, 0.5, out=out)       # warm on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fg(ctx, Vd, nud, Ad, ld, d, 0.5, out=out)
    for k in range(6):
        for x in out:
            x.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(out, ref):
            assert torch.equal(x, y), k
        # eager work between replays: another evaluation on the same context
        fg(ctx, Vd, nud, A2, l2, d, 0.5, out=other)
        torch.cuda.synchronize()
    S.symtd_check(ctx)
    assert not torch.equal(other[0], ref[0])
    del g
