"""symtd_fg_noalloc, the entry point that allocates nothing: called through
the C ABI, its results are the bits of symtd_fg (the same kernels on the
library's fixed scratch array) and within the oracle's tolerance, on two
calls in a row, the second with a smaller input; a workspace beyond the
fixed array is refused with SYMTD_EINVAL."""

import numpy as np
import pytest

from helpers import TOL, compare_fg, gpu_available, make_case, to_dev

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
def test_noalloc_equals_fg_two_calls(ctx, kind):
    dt = torch.float64 if kind == "f64" else torch.float32
    # the mid-size workload first, then a smaller, ragged one on the same array
    for (n, p, r, d, key) in [(100, 5000, 20, 4, (60,)), (37, 1001, 9, 3, (61,))]:
        print(f"case noalloc {kind} n={n} p={p} r={r} d={d}", flush=True)
        case = make_case(n, p, r, d, key, 1e-2, kind)
        Vd, nud, Ad, ld = _dev(case, dt)
        alpha = 1.5
        a = S.symtd_fg_noalloc(ctx, Vd, nud, Ad, ld, d, alpha)
        torch.cuda.synchronize()
        a = [x.cpu().clone() for x in a]
        b = S.symtd_fg(ctx, Vd, nud, Ad, ld, d, alpha)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y.cpu())
        got = (float(a[0][0]), a[1].numpy(), a[2].double().numpy())
        errs = compare_fg(got, *case, d, alpha, kind)
        assert max(errs) <= TOL[kind], errs


def test_noalloc_refuses_a_workspace_beyond_the_array(ctx):
    # d=3, n=1000, p=1e5, r=100 in fp32 needs about 81 MB of workspace
    n, p, r = 1000, 100_000, 100
    V = S.colmajor(torch.zeros(n, p, dtype=torch.float32, device="cuda"))
    A = S.colmajor(torch.zeros(n, r, dtype=torch.float32, device="cuda"))
    nu = torch.full((p,), 1.0 / p, dtype=torch.float64, device="cuda")
    lam = torch.ones(r, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SymtdError) as e:
        S.symtd_fg_noalloc(ctx, V, nu, A, lam, 3, 0.0)
    assert e.value.status == -1
    assert "scratch" in str(e.value)
