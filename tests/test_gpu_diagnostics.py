"""Device diagnostics (conserved totals, max |div B|; eq. 6 and 8) through
the C ABI against numpy sums and the oracle's discrete divergence, their
determinism, and checkpoint/resume: N steps, read back, a fresh context,
M more steps equal N + M steps bit for bit."""

import numpy as np
import pytest
import torch

from oracle.bweno import divergence
from paper_1006_2146_amd import ader, workloads

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _ref_totals(U, B, dx):
    vol = dx[0] * dx[1] * dx[2]
    t = np.zeros(8)
    t[:5] = U.sum(axis=(1, 2, 3)) * vol
    if B is not None:
        t[5:] = B.sum(axis=(1, 2, 3)) * vol
    return t


def _close(got, ref, scale, tol=1e-13):
    return np.all(np.abs(got - ref) <= tol * np.maximum(np.abs(scale), 1e-300))


@pytest.mark.parametrize("shape", [(9, 14, 21), (64, 64, 64), (1, 1, 1), (3, 1, 40)])
def test_euler_totals(shape):
    U = workloads.random_smooth(shape, seed=5)
    lengths = (1.0, 0.8, 1.3)
    dx = (lengths[0] / shape[2], lengths[1] / shape[1], lengths[2] / shape[0])
    with ader.Solver(shape, lengths=lengths) as s:
        s.set_state(U)
        say("euler totals", shape)
        tot, div = s.diagnostics()
        ref = _ref_totals(U, None, dx)
        scale = np.abs(U).sum(axis=(1, 2, 3)) * dx[0] * dx[1] * dx[2]
        assert _close(tot[:5], ref[:5], scale), (tot, ref)
        assert np.all(tot[5:] == 0.0) and div == 0.0
        # the same bits for another launch shape of the rest of the library
        shapes = ader.ader_get_launch(s.ctx)
        ader.ader_set_launch(s.ctx, {k: (64, 1) for k in shapes})
        tot2, _ = s.diagnostics()
        assert np.array_equal(tot, tot2)
        # conservation over steps (eq. 6 on a periodic mesh)
        for _ in range(3):
            s.step_cfl(0.3)
        tot3, _ = s.diagnostics()
        assert _close(tot3[:5], tot[:5], scale, 2e-13), (tot3 - tot)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_mhd_totals_and_div_b(order):
    shape = (10, 12, 14)
    U, B = workloads.mhd_random_field(shape, seed=order, p0=1.0)
    dx = (1.0 / 14, 1.0 / 12, 1.0 / 10)
    with ader.Solver(shape, gamma=G53, order=order, system=ader.ADER_MHD) as s:
        s.set_state(U, B)
        say("mhd diagnostics", order)
        tot, div = s.diagnostics()
        ref = _ref_totals(U, B, dx)
        vol = dx[0] * dx[1] * dx[2]
        scale = np.concatenate([np.abs(U).sum(axis=(1, 2, 3)), np.abs(B).sum(axis=(1, 2, 3))]) * vol
        # the fluid starts at rest: its momentum totals are sums of round-off,
        # compared on the scale of the mass and energy totals
        scale = np.maximum(scale, 1e-3 * scale.max())
        assert _close(tot, ref, scale), (tot, ref)
        assert div == np.abs(divergence(B, dx)).max()
        for _ in range(2):
            s.step_cfl(0.3)
        Ug, Bg = s.get_state()
        tot1, div1 = s.diagnostics()
        assert div1 == np.abs(divergence(Bg, dx)).max()
        assert div1 <= 1e-12 * np.abs(Bg).max() / min(dx)
        assert _close(tot1, tot, scale, 2e-13), tot1 - tot
        assert _close(tot1, _ref_totals(Ug, Bg, dx), scale)


def test_batch_diagnostics_per_problem():
    shapes = [(5, 7, 9), (1, 1, 1), (16, 16, 33), (2, 9, 1)]
    states = [workloads.mhd_random_field(sh, seed=40 + q, p0=1.0) for q, sh in enumerate(shapes)]
    with ader.BatchSolver(shapes, gamma=G53, system=ader.ADER_MHD) as b:
        for q, (U, B) in enumerate(states):
            b.set_state(q, U, B)
        say("batch diagnostics")
        tot, div = b.diagnostics()
        for q, ((U, B), sh) in enumerate(zip(states, shapes)):
            dx = (1.0 / sh[2], 1.0 / sh[1], 1.0 / sh[0])
            vol = dx[0] * dx[1] * dx[2]
            scale = np.concatenate([np.abs(U).sum(axis=(1, 2, 3)),
                                    np.abs(B).sum(axis=(1, 2, 3))]) * vol
            assert _close(tot[q], _ref_totals(U, B, dx), scale), q
            assert div[q] == np.abs(divergence(B, dx)).max(), q


def test_diagnostics_errors():
    with ader.Solver((4, 4, 4)) as s:
        assert ader.load().ader_diagnostics(s.ctx, None, None) == ader.ADER_ESEQ
    assert ader.load().ader_diagnostics(None, None, None) == ader.ADER_EINVAL


@pytest.mark.parametrize("system", ["euler", "mhd"])
@pytest.mark.parametrize("precision", [ader.ADER_FP64, ader.ADER_MIXED])
def test_checkpoint_resume_bitwise(system, precision):
    # N steps, read the state back, a fresh context from it, M more steps:
    # the same bits as N + M steps in one context (eager and graph-replayed)
    mhd = system == "mhd"
    shape = (9, 10, 11)
    kw = dict(order=3, precision=precision)
    if mhd:
        U0, B0 = workloads.mhd_random_field(shape, seed=9, p0=1.0)
        kw.update(gamma=G53, system=ader.ADER_MHD)
    else:
        U0, B0 = workloads.random_smooth(shape, seed=9), None
    N, M = 3, 4
    with ader.Solver(shape, **kw) as s:
        s.set_state(U0, B0)
        for _ in range(N + M):
            s.step_cfl(0.3)
        ref = s.get_state()
    stream = torch.cuda.Stream()
    with ader.Solver(shape, stream=stream.cuda_stream, **kw) as s:
        ader.ader_set_graph(s.ctx, True)
        s.set_state(U0, B0)
        for _ in range(N):
            s.step_cfl(0.3)
        mid = s.get_state()
    say("resume", system, precision)
    with ader.Solver(shape, **kw) as s:
        if mhd:
            s.set_state(*mid)
        else:
            s.set_state(mid)
        for _ in range(M):
            s.step_cfl(0.3)
        out = s.get_state()
    if mhd:
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
    else:
        assert np.array_equal(out, ref)
