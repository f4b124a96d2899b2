"""Checkpoint and resume of symtd_solve (through the C ABI).

A solve paused after some evaluation steps, its state saved to host memory
and continued from it (with another polling cadence, and once across two
pauses) must end exactly where the uninterrupted solve ends: the same model
bits, the same per-restart figures and the same f traces.  Only the step
count may differ, by the idle steps that run after every restart has
stopped and before the next poll.  A state is refused for another problem
or other options.
"""

import numpy as np
import pytest

import synth
from helpers import gpu_available, stored, to_dev

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


def problem(kind, n=30, r=4, p=1200, sigma=1e-2, key=71):
    dt = torch.float64 if kind == "f64" else torch.float32
    V, nu, _ = synth.gmm(n, r, p, sigma, key)
    V = stored(V, kind)
    return to_dev(V, dt), to_dev(nu, torch.float64)


def same_end(a, b):
    assert torch.equal(a["A"], b["A"]) and torch.equal(a["lam"], b["lam"])
    for k in ("f", "alpha", "iters", "evals", "exit_reason", "best_restart"):
        assert a[k] == b[k], k
    for k in ("f_restarts", "iters_restarts", "evals_restarts", "exit_restarts"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["f_trace"], b["f_trace"], equal_nan=True)


@pytest.mark.parametrize("kind,noise", [("f64", 0.0), ("f32", 0.0), ("f64", 0.05)])
def test_pause_resume_equals_uninterrupted(ctx, kind, noise):
    Vd, nud = problem(kind)
    d, r = 3, 4
    kw = dict(restarts=3, seed=5, pgtol=1e-7, max_iters=400, trace_len=60, sigma=noise)
    print(f"case pause/resume {kind} sigma={noise}", flush=True)
    full = S.symtd_solve(ctx, Vd, nud, d, r, check_every=8, **kw)
    assert full["exit_reason"] != S.EXIT_RUNNING and full["steps"] > 40
    first = S.symtd_solve(ctx, Vd, nud, d, r, check_every=8, pause_after=13, **kw)
    assert first["paused"] and first["steps"] == 13 and first["exit_reason"] == S.EXIT_RUNNING
    state = first["state"]
    # continue with another polling cadence
    rest = S.symtd_solve(ctx, Vd, nud, d, r, check_every=5, state=state, **kw)
    assert not rest["paused"] and rest["steps"] >= full["steps"] - 8
    same_end(rest, full)
    # two pauses in a row
    second = S.symtd_solve(ctx, Vd, nud, d, r, check_every=3, pause_after=31, state=state, **kw)
    assert second["paused"] and second["steps"] == 31
    last = S.symtd_solve(ctx, Vd, nud, d, r, state=second["state"], **kw)
    same_end(last, full)


def test_pause_after_the_end_changes_nothing(ctx):
    Vd, nud = problem("f64", key=72)
    kw = dict(restarts=2, seed=1, pgtol=1e-5, max_iters=60, trace_len=20)
    full = S.symtd_solve(ctx, Vd, nud, 3, 4, check_every=4, **kw)
    late = S.symtd_solve(ctx, Vd, nud, 3, 4, check_every=4, pause_after=full["steps"] + 100, **kw)
    assert not late["paused"] and late["state"] is None
    same_end(late, full)


def test_resume_refuses_another_problem_or_options(ctx):
    Vd, nud = problem("f64", key=73)
    kw = dict(restarts=2, seed=3, pgtol=1e-7, max_iters=300)
    first = S.symtd_solve(ctx, Vd, nud, 3, 4, pause_after=10, **kw)
    assert first["paused"]
    state = first["state"]
    bad = [dict(kw, restarts=3), dict(kw, seed=4), dict(kw, pgtol=1e-6), dict(kw, max_iters=301),
           dict(kw, trace_len=5), dict(kw, pause_after=10), dict(kw, pause_after=4)]
    for opts in bad:
        with pytest.raises(S.SymtdError) as e:
            S.symtd_solve(ctx, Vd, nud, 3, 4, state=state, **opts)
        assert e.value.status == -1 and "saved state" in str(e.value), opts
    # another rank or order
    for d, r in ((4, 4), (3, 5)):
        with pytest.raises(S.SymtdError) as e:
            S.symtd_solve(ctx, Vd, nud, d, r, state=state, **kw)
        assert e.value.status == -1
    # a truncated state (the binding checks the length before the library reads it)
    with pytest.raises(S.SymtdError) as e:
        S.symtd_solve(ctx, Vd, nud, 3, 4, state=state[:-8], **kw)
    assert e.value.status == -1 and "bytes" in str(e.value)
    # a corrupted header
    broken = bytearray(state)
    broken[0] ^= 0xFF
    with pytest.raises(S.SymtdError) as e:
        S.symtd_solve(ctx, Vd, nud, 3, 4, state=bytes(broken), **kw)
    assert e.value.status == -1
    # the batched form refuses pausing
    with pytest.raises(S.SymtdError) as e:
        S.symtd_solve_batched(ctx, [dict(V=Vd, nu=nud, d=3, r=4, pause_after=5)])
    assert e.value.status == -1
