"""Pins of the oracle's face-side quantities (Sec. V, Appendix D)."""

import numpy as np
import pytest

from oracle import basis, faces
from tests import indep


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_mode_order(order):
    assert faces.FACE_MODES[order] == indep.face_modes(order)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_rules_exact_on_face_span(order):
    # (D.4), (D.9), (D.14) recover every mode of a polynomial in (D.2)/(D.7)/(D.12)
    rng = np.random.default_rng(order)
    n = len(faces.FACE_MODES[order])
    for _ in range(4):
        c = rng.normal(size=n)
        fv = [None] + [indep.face_value(c, order, p) for p in faces.FACE_NODES[order]]
        m = faces.FACE_RULE[order](fv)
        assert np.allclose(m[1:], c, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_rule_transverse_symmetry(order):
    # swapping the two transverse coordinates maps the node set to itself and
    # leaves the face average of any nodal data unchanged
    nodes = faces.FACE_NODES[order]
    idx = {tuple(map(float, p)): i for i, p in enumerate(nodes)}
    perm = [idx[(float(p[1]), float(p[0]), float(p[2]))] for p in nodes]
    rng = np.random.default_rng(5)
    v = rng.normal(size=len(nodes))
    a = faces.face_average_of_modes(faces.FACE_RULE[order]([None] + list(v)), order)
    b = faces.face_average_of_modes(faces.FACE_RULE[order]([None] + list(v[perm])), order)
    assert abs(a - b) < 1e-14


def _gl_face_average(coeffs, order, d, s, edge=None):
    """Numerical space-time average of the zone polynomial over one face side
    (or one edge of it) by Gauss-Legendre quadrature."""
    xs, ws = indep.gauss(5, -0.5, 0.5)
    ts, wt = indep.gauss(5, 0.0, 1.0)
    tr = faces.transverse_axes(d)
    tot = 0.0
    for i, (a, wa) in enumerate(zip(xs, ws)):
        for j, (b, wb) in enumerate(zip(xs, ws)):
            for t, w3 in zip(ts, wt):
                p = [0.0, 0.0, 0.0]
                p[d] = 0.5 * s
                p[tr[0]], p[tr[1]] = a, b
                wgt = wa * wb * w3
                if edge is not None:
                    which, sign = edge
                    p[tr[which]] = 0.5 * sign
                    wgt = (wb if which == 0 else wa) * w3
                    if (which == 0 and i > 0) or (which == 1 and j > 0):
                        continue
                tot += wgt * indep.st_value(coeffs, order, (p[0], p[1], p[2], t))
    return tot


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_and_edge_averages_of_u(order):
    # eq. (54), (55), (57) against direct quadrature
    rng = np.random.default_rng(20 + order)
    L = basis.N_SPACETIME[order]
    c = rng.normal(size=L)
    uh = c[:, None]
    for d in range(3):
        for s in (-1, 1):
            p = [0.0, 0.0, 0.0]
            p[d] = 0.5 * s
            ub = indep.st_value(c, order, (p[0], p[1], p[2], 0.5))
            assert abs(faces.barycentre_state(uh, order, d, s)[0] - ub) < 1e-14
            ref = _gl_face_average(c, order, d, s)
            assert abs(faces.face_average_u(uh, order, d, s)[0] - ref) < 1e-13
            tr = faces.transverse_axes(d)
            for which in (0, 1):
                for sign in (-1, 1):
                    ref = _gl_face_average(c, order, d, s, edge=(which, sign))
                    got = faces.edge_average_u(uh, order, d, s, tr[which], sign)[0]
                    assert abs(got - ref) < 1e-13


def _w(c, k):
    return c[k - 1]


def test_closed_forms_third_order_match():
    # eq. (61), (62), (63) (x-faces) against the oracle's direct integrals
    rng = np.random.default_rng(3)
    c = rng.normal(size=15)
    w = lambda k: _w(c, k)  # noqa: E731
    ubp = w(1) + 0.5 * (w(2) + w(11)) + 0.25 * (w(12) + w(13)) + (2 * w(5) - w(6) - w(7)) / 12
    ubm = ubp - w(2) - 0.5 * w(13)
    q1 = (w(6) + w(7) + w(12)) / 12
    up, um = ubp + q1, ubm + q1
    q2 = 0.5 * w(3) + 0.25 * (w(8) + w(14))
    uh = c[:, None]
    assert abs(faces.barycentre_state(uh, 3, 0, 1)[0] - ubp) < 1e-14
    assert abs(faces.barycentre_state(uh, 3, 0, -1)[0] - ubm) < 1e-14
    assert abs(faces.face_average_u(uh, 3, 0, 1)[0] - up) < 1e-14
    assert abs(faces.face_average_u(uh, 3, 0, -1)[0] - um) < 1e-14
    assert abs(faces.edge_average_u(uh, 3, 0, 1, 1, 1)[0] - (up + w(6) / 6 + q2)) < 1e-14


def test_closed_forms_fourth_order_match():
    # eq. (64), (65), (66) (x-faces)
    rng = np.random.default_rng(4)
    c = rng.normal(size=35)
    w = lambda k: _w(c, k)  # noqa: E731
    q1 = (w(1) + 0.5 * w(21) + 0.25 * w(22) + 0.125 * w(23)
          + (4 * w(5) - 2 * w(6) - 2 * w(7) + 2 * w(30) - w(31) - w(32)) / 24)
    q2 = 0.5 * w(2) + 0.05 * w(11) + 0.25 * w(24) + 0.125 * w(27) - (w(16) + w(18)) / 24
    ubp, ubm = q1 + q2, q1 - q2
    up = ubp + (2 * w(6) + 2 * w(7) + w(16) + w(18) + 2 * w(22) + 3 * w(23) + w(27)
                + w(31) + w(32)) / 24
    um = ubm + (2 * w(6) + 2 * w(7) - w(16) - w(18) + 2 * w(22) + 3 * w(23) - w(27)
                + w(31) + w(32)) / 24
    q3 = (w(3) + 0.5 * (w(8) + w(25)) + 0.25 * w(33) + 0.1 * w(12)
          + (w(14) + 2 * w(28)) / 6)
    upy = up + (2 * w(6) + w(16) + w(31)) / 12 + 0.5 * q3
    uh = c[:, None]
    assert abs(faces.barycentre_state(uh, 4, 0, 1)[0] - ubp) < 1e-14
    assert abs(faces.barycentre_state(uh, 4, 0, -1)[0] - ubm) < 1e-14
    assert abs(faces.face_average_u(uh, 4, 0, 1)[0] - up) < 1e-14
    assert abs(faces.face_average_u(uh, 4, 0, -1)[0] - um) < 1e-14
    assert abs(faces.edge_average_u(uh, 4, 0, 1, 1, 1)[0] - upy) < 1e-14
    assert abs(faces.edge_average_u(uh, 4, 0, 1, 1, -1)[0] - (upy - q3)) < 1e-14


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_flux_average_closed_forms(order):
    # (D.5), (D.10), (D.15): <f> and the edge averages from the face modes
    rng = np.random.default_rng(40 + order)
    n = len(faces.FACE_MODES[order])
    m = [None] + list(rng.normal(size=n))
    if order == 2:
        fx = m[1] + 0.5 * m[4]
        fy = fx + 0.5 * m[2]
    elif order == 3:
        fx = m[1] + 0.5 * m[7] + m[8] / 3
        q4 = 0.5 * m[2] + 0.25 * m[9]
        fy = fx + q4 + m[4] / 6
    else:
        fx = m[1] + 0.5 * m[11] + m[12] / 3 + 0.25 * m[13]
        q5 = fx + (2 * m[4] + m[18]) / 12
        q6 = 0.5 * m[2] + 0.05 * m[7] + 0.25 * m[14] + m[16] / 6
        fy = q5 + q6
    assert abs(faces.face_average_of_modes(m, order) - fx) < 1e-14
    assert abs(faces.edge_average_of_modes(m, order, 0, 1) - fy) < 1e-14


@pytest.mark.parametrize("order", [2, 3, 4])
def test_facial_flux_exact_for_polynomial_flux(order):
    # with a linear flux and u in the span, <F> equals the exact face average
    rng = np.random.default_rng(60 + order)
    L = basis.N_SPACETIME[order]
    c = rng.normal(size=L)
    uh = c[:, None]
    lin = lambda u, axis: 2.5 * u  # noqa: E731
    for d in range(3):
        for s in (-1, 1):
            pk = faces.face_side_packet(uh, order, d, s, 1.4, flux_fn=lin, edges=True)
            assert abs(pk['f'][0] - 2.5 * _gl_face_average(c, order, d, s)) < 1e-12
            for (which, sign), val in pk['f_edge'].items():
                ref = 2.5 * _gl_face_average(c, order, d, s, edge=(which, sign))
                assert abs(val[0] - ref) < 1e-12
