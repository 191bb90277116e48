"""Pins of the oracle's linear-advection step (the scheme of Sec. II with
F_d(u) = a_d u and the upwind limit of eq. 56): exact translation by one
zone at unit Courant number along each axis and in both directions, for any
data; constant states; conservation; independence of the five components;
design order on a smooth wave against its exact zone averages."""

import numpy as np
import pytest

from oracle import OracleConfig
from oracle import linadv

CASES = [(2, 'modal'), (2, 'nodal'), (3, 'modal'), (3, 'nodal'), (4, 'modal'), (4, 'nodal')]


@pytest.mark.parametrize("order,form", CASES)
@pytest.mark.parametrize("axis,speed", [(0, 3.0), (1, -2.0), (2, 0.5)])
def test_exact_translation_at_unit_courant(order, form, axis, speed):
    # at |a_d| dt = dx_d the upwind face flux is the face-side average over
    # the step of the upwind zone's exact translate, which integrates to its
    # zone average: each zone takes its upwind neighbour's average
    rng = np.random.default_rng(order + 10 * axis)
    n = (6, 5, 8)
    U = rng.uniform(0.5, 1.5, size=(5,) + n)
    lengths = (1.0, 0.7, 1.3)
    cfg = OracleConfig(order=order, form=form, lengths=lengths)
    dx = cfg.spacing(n)
    a = [0.0, 0.0, 0.0]
    a[axis] = speed
    dt = dx[axis] / abs(speed)
    assert abs(linadv.compute_dt(U, cfg, 1.0, a) - dt) <= 1e-15 * dt
    Un = linadv.step(U, dt, cfg, a)
    ref = np.roll(U, 1 if speed > 0 else -1, axis=3 - axis)
    assert np.abs(Un - ref).max() <= 1e-13


@pytest.mark.parametrize("order,form", CASES)
def test_constant_state_conservation_and_independence(order, form):
    cfg = OracleConfig(order=order, form=form)
    a = (0.8, -0.5, 0.3)
    c = np.array([1.0, -2.0, 0.5, 3.0, 7.0])
    U = np.broadcast_to(c[:, None, None, None], (5, 4, 5, 6)).copy()
    assert np.array_equal(linadv.step(U, 0.05, cfg, a), U)
    rng = np.random.default_rng(order)
    U = rng.uniform(0.5, 1.5, size=(5, 5, 6, 7))
    dt = linadv.compute_dt(U, cfg, 0.4, a)
    Un = linadv.step(U, dt, cfg, a)
    assert np.all(np.abs(Un.sum(axis=(1, 2, 3)) - U.sum(axis=(1, 2, 3))) <= 1e-13 * U.sum())
    # each component advects alone: changing the others leaves it unchanged
    V = U.copy()
    V[1:] = rng.uniform(0.5, 1.5, size=V[1:].shape)
    assert np.abs(linadv.step(V, dt, cfg, a)[0] - Un[0]).max() <= 1e-15


def _wave_error(n, order, form, T=0.25):
    cfg = OracleConfig(order=order, form=form)
    x = np.arange(n) / n
    h = 1.0 / n

    def avg(t):
        v = (np.cos(2 * np.pi * (x - t)) - np.cos(2 * np.pi * (x + h - t))) / (2 * np.pi * h)
        return np.broadcast_to(v, (5, 1, 1, n)).copy()

    U = avg(0.0)
    a = (1.0, 0.0, 0.0)
    t = 0.0
    while t < T - 1e-12:
        dt = min(linadv.compute_dt(U, cfg, 0.5, a), T - t)
        U = linadv.step(U, dt, cfg, a)
        t += dt
    return np.abs(U - avg(T)).mean()


@pytest.mark.parametrize("order,form,floor", [(2, 'modal', 1.5), (3, 'modal', 2.7),
                                              (4, 'modal', 3.7), (4, 'nodal', 3.7)])
def test_design_order_on_a_smooth_wave(order, form, floor):
    e1, e2 = _wave_error(32, order, form), _wave_error(64, order, form)
    assert np.log2(e1 / e2) > floor, (e1, e2)
