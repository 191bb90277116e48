"""Pins of the positivity handling: the check of the paper's scheme (the
default) and the opt-in scaling safeguard (see oracle/positivity.py)."""

import numpy as np
import pytest

from oracle import basis, faces, positivity
from oracle.physics import primitives


def _zone_poly(order, rng, amp):
    ls = basis.N_SPATIAL[order]
    w = np.zeros((ls, 5, 1))
    w[0, :, 0] = [1.0, 0.3, -0.2, 0.1, 2.0]
    w[1:, :, 0] = amp * rng.normal(size=(ls - 1, 5))
    return w


def _check_values(w, order, form):
    uh = np.zeros((basis.N_SPACETIME[order],) + w.shape[1:])
    uh[:w.shape[0]] = w
    return [basis.evaluate(uh, order, p) for p in positivity.spatial_check_points(order, form)]


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_average_nodes_are_the_weighted_ones(order):
    # compose (D.4)/(D.9)/(D.14) with the exact face integral: exactly the
    # listed facial nodes carry a nonzero weight
    n = len(faces.FACE_NODES[order])
    weights = []
    for j in range(n):
        unit = [None] + [1.0 if k == j else 0.0 for k in range(n)]
        weights.append(faces.face_average_of_modes(faces.FACE_RULE[order](unit), order))
    nz = [j + 1 for j, w in enumerate(weights) if abs(w) > 1e-14]
    assert nz == positivity.FACE_AVERAGE_NODES[order]
    assert abs(sum(weights) - 1.0) < 1e-14


@pytest.mark.parametrize("order", [2, 3, 4])
def test_limiter_inactive_on_positive_polynomials(order):
    rng = np.random.default_rng(order)
    w = _zone_poly(order, rng, 0.01)
    out = positivity.limit_spatial(w, order, 'modal', 1.4)
    assert np.array_equal(out, w)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_limiter_restores_positivity_tightly(order):
    rng = np.random.default_rng(10 + order)
    hits = 0
    for _ in range(20):
        w = _zone_poly(order, rng, 1.5)
        out = positivity.limit_spatial(w, order, 'modal', 1.4)
        assert np.array_equal(out[0], w[0])                 # zone average kept
        ratio = out[1:] / np.where(w[1:] == 0, 1, w[1:])
        theta = ratio.ravel()[np.argmax(np.abs(w[1:]).ravel())]
        assert np.allclose(out[1:], theta * w[1:], rtol=1e-13, atol=0)
        vals = [v for v in _check_values(out, order, 'modal')]
        rho = np.array([v[0, 0] for v in vals])
        p = np.array([primitives(v, 1.4)[2][0] for v in vals])
        p_bar = primitives(w[0], 1.4)[2][0]
        eps_r = positivity.EPS_REL * w[0, 0, 0]
        eps_p = positivity.EPS_REL * p_bar
        assert rho.min() >= eps_r * (1 - 1e-6)
        assert p.min() >= eps_p * (1 - 1e-4) - 1e-14
        if theta < 1.0:
            hits += 1
            # the largest admissible theta: one check point sits on a bound
            tight = min(rho.min() / eps_r, p.min() / eps_p)
            assert abs(tight - 1.0) < 1e-3
    assert hits > 5


@pytest.mark.parametrize("order", [2, 3, 4])
def test_check_mode_reports_exactly_nonpositive_points(order):
    # the check raises where some check point has rho <= 0 or P <= 0 and
    # returns the polynomial unchanged (the same object) otherwise
    rng = np.random.default_rng(20 + order)
    w = _zone_poly(order, rng, 0.01)
    assert positivity.safeguard_spatial(w, order, 'modal', 1.4, 'check') is w
    w[:, 1:4] = 0.0     # at rest, so only rho decides
    vals = _check_values(w, order, 'modal')
    # move the zone average so that the lowest check point has rho slightly
    # below / above zero
    r_min = min(v[0, 0] for v in vals)
    for shift, raises in ((r_min + 1e-9, True), (r_min - 1e-9, False)):
        v = w.copy()
        v[0, 0, 0] -= shift
        if raises:
            with pytest.raises(positivity.NonPhysical):
                positivity.check_spatial(v, order, 'modal', 1.4)
        else:
            positivity.check_spatial(v, order, 'modal', 1.4)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_check_mode_pressure(order):
    # lowering the total energy until the pressure at the worst check point
    # crosses zero flips the check
    rng = np.random.default_rng(40 + order)
    w = _zone_poly(order, rng, 0.01)
    vals = _check_values(w, order, 'modal')
    pmin = min(float(primitives(v, 1.4)[2][0]) for v in vals)
    v = w.copy()
    v[0, 4, 0] -= pmin / 0.4 * 0.999
    positivity.check_spatial(v, order, 'modal', 1.4)
    v[0, 4, 0] -= pmin / 0.4 * 0.002
    with pytest.raises(positivity.NonPhysical):
        positivity.check_spatial(v, order, 'modal', 1.4)


def test_unknown_mode_rejected():
    w = _zone_poly(3, np.random.default_rng(0), 0.01)
    with pytest.raises(ValueError):
        positivity.safeguard_spatial(w, 3, 'modal', 1.4, 'clip')
