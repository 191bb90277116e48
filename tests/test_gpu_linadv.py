"""The linear-advection test system (ADER_LINADV) on the GPU through the C
ABI: exact translation by one zone at unit Courant number along each axis
and in both directions for any data (the property of the scheme with the
linear flux F_d(u) = a_d u and the upwind limit of eq. 56), FP64 parity with
the oracle's linear-advection step for an oblique velocity, batch = solo
bitwise, conservation, and the argument checks."""

import numpy as np
import pytest

from oracle import OracleConfig
from oracle import linadv as oracle_linadv
from paper_1006_2146_amd import ader

pytestmark = pytest.mark.gpu

CASES = [(2, "modal"), (2, "nodal"), (3, "modal"), (3, "nodal"), (4, "modal"), (4, "nodal")]
FORM = {"modal": ader.ADER_MODAL, "nodal": ader.ADER_NODAL}


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _solver(shape, order, form, lengths=(1.0, 1.0, 1.0)):
    return ader.Solver(shape, lengths=lengths, order=order, form=FORM[form],
                       system=ader.ADER_LINADV)


@pytest.mark.parametrize("order,form", CASES)
def test_exact_translation_at_unit_courant(order, form):
    rng = np.random.default_rng(order)
    n = (6, 5, 8)
    lengths = (1.0, 0.7, 1.3)
    dx = (lengths[0] / n[2], lengths[1] / n[1], lengths[2] / n[0])
    U = rng.uniform(0.5, 1.5, size=(5,) + n)
    with _solver(n, order, form, lengths) as s:
        for axis, speed in ((0, 3.0), (1, -2.0), (2, 0.5)):
            say("translation", order, form, axis, speed)
            a = [0.0, 0.0, 0.0]
            a[axis] = speed
            s.set_advection(a)
            s.set_state(U)
            s.step_cfl(1.0)
            dt = s.dt()
            assert abs(dt - dx[axis] / abs(speed)) <= 1e-15 * dt
            ref = np.roll(U, 1 if speed > 0 else -1, axis=3 - axis)
            assert np.abs(s.get_state() - ref).max() <= 1e-13


@pytest.mark.parametrize("order,form", CASES)
def test_parity_oblique_velocity(order, form):
    rng = np.random.default_rng(10 + order)
    n = (7, 9, 10)
    lengths = (1.0, 0.9, 1.2)
    a = (0.7, -0.4, 0.3)
    cfg = OracleConfig(order=order, form=form, lengths=lengths)
    U = rng.uniform(0.5, 1.5, size=(5,) + n)
    with _solver(n, order, form, lengths) as s:
        s.set_advection(a)
        s.set_state(U)
        for it in range(2):
            say("linadv parity", order, form, "step", it)
            dt = s.compute_dt(0.4)
            assert abs(dt - oracle_linadv.compute_dt(U, cfg, 0.4, a)) <= 1e-14 * dt
            s.step(dt)
            Ug = s.get_state()
            Uo = oracle_linadv.step(U, dt, cfg, a)
            err = np.abs(Ug - Uo).sum(axis=(1, 2, 3)) / np.abs(Uo).sum(axis=(1, 2, 3))
            mx = np.abs(Ug - Uo).max() / np.abs(Uo).max()
            assert np.all(err <= 1e-12) and mx <= 1e-12, (it, err, mx)
            tot, _ = s.diagnostics()
            vol = lengths[0] * lengths[1] * lengths[2] / (n[0] * n[1] * n[2])
            assert np.all(np.abs(tot[:5] - U.sum(axis=(1, 2, 3)) * vol)
                          <= 1e-13 * np.abs(U).sum(axis=(1, 2, 3)) * vol)
            U = Ug


def test_batch_equals_solo():
    shapes = [(5, 7, 9), (1, 1, 1), (8, 3, 4)]
    rng = np.random.default_rng(3)
    states = [rng.uniform(0.5, 1.5, size=(5,) + sh) for sh in shapes]
    a = (-0.5, 0.8, 0.2)
    with ader.BatchSolver(shapes, order=3, system=ader.ADER_LINADV) as b:
        b.set_advection(a)
        for q, U in enumerate(states):
            b.set_state(q, U)
        for _ in range(2):
            b.step_cfl(0.4)
        got = [b.get_state(q) for q in range(len(shapes))]
    for q, (sh, U) in enumerate(zip(shapes, states)):
        with ader.Solver(sh, order=3, system=ader.ADER_LINADV) as s:
            s.set_advection(a)
            s.set_state(U)
            for _ in range(2):
                s.step_cfl(0.4)
            assert np.array_equal(s.get_state(), got[q]), q


def test_linadv_errors():
    with ader.Solver((4, 4, 4)) as s:
        with pytest.raises(ader.AderError) as e:
            s.set_advection((1.0, 0.0, 0.0))
        assert e.value.code == ader.ADER_EUNSUPPORTED
    with ader.Solver((4, 4, 4), system=ader.ADER_LINADV) as s:
        for bad in ((0.0, 0.0, 0.0), (np.nan, 1.0, 0.0)):
            with pytest.raises(ader.AderError) as e:
                s.set_advection(bad)
            assert e.value.code == ader.ADER_EINVAL
        with pytest.raises(ader.AderError) as e:
            s.set_source(np.eye(5), None)
        assert e.value.code == ader.ADER_EUNSUPPORTED
        s.set_state(np.ones((5, 4, 4, 4)))
        # FP64 and the ADER scheme only
        ader.ader_set_precision(s.ctx, ader.ADER_MIXED)
        with pytest.raises(ader.AderError) as e:
            s.step(1e-3)
        assert e.value.code == ader.ADER_EUNSUPPORTED
        ader.ader_set_precision(s.ctx, ader.ADER_FP64)
        ader.ader_set_scheme(s.ctx, ader.ADER_SCHEME_SSPRK)
        with pytest.raises(ader.AderError) as e:
            s.step(1e-3)
        assert e.value.code == ader.ADER_EUNSUPPORTED
