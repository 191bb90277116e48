"""ader_diagnostics_noalloc, the diagnostics entry point that allocates
nothing (its scratch is a fixed device array of the library), against
ader_diagnostics through the C ABI: the same bits on two calls in a row,
the second with a smaller input, and its size limit."""

import ctypes

import numpy as np
import pytest

from paper_1006_2146_amd import ader, workloads

pytestmark = pytest.mark.gpu


def _noalloc(ctx, n):
    lib = ader.load()
    fn = lib.ader_diagnostics_noalloc
    fn.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                   ctypes.POINTER(ctypes.c_double)]
    fn.restype = ctypes.c_int
    tot = np.full((n, 8), np.nan)
    div = np.full(n, np.nan)
    rc = fn(ctx, tot.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            div.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, tot, div


def test_noalloc_equals_diagnostics_on_two_calls():
    # call 1: an MHD batch of three problems (several tiles each); call 2: a
    # smaller Euler problem, so stale rows of the first call would show
    shapes = [(20, 24, 33), (9, 5, 4), (16, 16, 16)]
    states = [workloads.mhd_random_field(sh, seed=60 + q, p0=1.0) for q, sh in enumerate(shapes)]
    with ader.BatchSolver(shapes, gamma=5.0 / 3.0, system=ader.ADER_MHD) as b:
        for q, (U, B) in enumerate(states):
            b.set_state(q, U, B)
        b.step_cfl(0.3)
        ref_tot, ref_div = b.diagnostics()
        rc, tot, div = _noalloc(b.ctx, len(shapes))
        assert rc == ader.ADER_OK
        assert np.array_equal(tot, ref_tot) and np.array_equal(div, ref_div)
    with ader.Solver((6, 7, 5)) as s:
        s.set_state(workloads.random_smooth((6, 7, 5), seed=3))
        s.step_cfl(0.3)
        ref_tot, ref_div = s.diagnostics()
        rc, tot, div = _noalloc(s.ctx, 1)
        assert rc == ader.ADER_OK
        assert np.array_equal(tot[0], ref_tot) and div[0] == ref_div == 0.0


def test_noalloc_limits():
    # more problems than the fixed scratch holds results for: rejected
    with ader.BatchSolver([(1, 1, 1)] * 4097) as b:
        rc, _, _ = _noalloc(b.ctx, 4097)
        assert rc == ader.ADER_EINVAL
    with ader.Solver((4, 4, 4)) as s:
        rc, _, _ = _noalloc(s.ctx, 1)
        assert rc == ader.ADER_ESEQ
