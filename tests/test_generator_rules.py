"""Pins of the GPU side's own derivation (the kernel-code generator
csrc/gen_scheme.py), made apart from the oracle: the generator's composed
predictor weights (the nodal-to-modal flux rules eq. (33), (40)-(42),
(49)-(51) with the evolution equations (30), (36), (45)) against the
Galerkin weak form of the space-time predictor derived in rationals, and
its App. D face and edge weights (eq. (D.4)-(D.15), (57)) against the exact
averages of a face polynomial, and the generated predictor's steps (modal
and nodal, App. A-C) exact for linear advection of data in the span.  Fluxes are random polynomials of the span
the rules are exact on, evaluated with the independent basis of
tests/indep.py; a misprint that the generator and the oracle shared would
fail here."""

import importlib.util
import os

import numpy as np
import pytest

from tests import indep
from tests.test_oracle_predictor import _galerkin_matrices

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gen():
    path = os.path.join(ROOT, "paper_1006_2146_amd", "csrc", "gen_scheme.py")
    spec = importlib.util.spec_from_file_location("gen_scheme_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


GEN = _gen()


@pytest.mark.parametrize("order", [2, 3, 4])
def test_mode_order_matches_eq_14_16(order):
    assert [tuple(m) for m in GEN.mode_list(order)] == [tuple(m) for m in indep.st_modes(order)]


@pytest.mark.parametrize("order", [2, 3, 4])
def test_predictor_weights_match_galerkin(order):
    # the weights applied to the nodal values of flux polynomials of the
    # space-time span give the evolutionary modes the weak form gives
    E = [np.array(e.tolist(), dtype=np.float64) for e in _galerkin_matrices(order)]
    W = GEN.evolution_weights(order, 'modal')
    nodes = [tuple(float(c) for c in p) for p in GEN.pred_nodes(order, 'modal')]
    L = len(indep.st_modes(order))
    assert len(W) == E[0].shape[0]
    rng = np.random.default_rng(order)
    for _ in range(3):
        modes = rng.normal(size=(3, L))
        vals = {d: [indep.st_value(modes[a], order, p) for p in nodes]
                for a, d in enumerate('fgh')}
        ref = E[0] @ modes[0] + E[1] @ modes[1] + E[2] @ modes[2]
        got = np.array([sum(float(c) * vals[d][j - 1] for (d, j), c in lin.items())
                        for lin in W])
        assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max()), (got, ref)


def _face_poly(order, rng):
    fm = indep.face_modes(order)
    return fm, rng.normal(size=len(fm))


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_average_weights_exact(order):
    # the face-time average of the normal flux: only the modes constant in
    # both transverse coordinates have a nonzero mean, tau^d has 1/(d+1)
    rng = np.random.default_rng(10 + order)
    nodes = [tuple(float(c) for c in p) for p in GEN.face_nodes(order)]
    for _ in range(3):
        fm, c = _face_poly(order, rng)
        ref = sum(ck / (d + 1) for ck, (a, b, d) in zip(c, fm) if a == 0 and b == 0)
        got = sum(float(w) * indep.face_value(c, order, nodes[j - 1])
                  for j, w in GEN.face_average_weights(order).items())
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("sign", [-1, 1])
def test_edge_average_weights_exact(order, which, sign):
    # eq. (57): the average along the edge t_which = sign/2, over the other
    # transverse coordinate and tau
    rng = np.random.default_rng(20 + order)
    nodes = [tuple(float(c) for c in p) for p in GEN.face_nodes(order)]
    for _ in range(3):
        fm, c = _face_poly(order, rng)
        ref = 0.0
        for ck, (a, b, d) in zip(c, fm):
            on, off = (a, b) if which == 0 else (b, a)
            if off == 0:
                ref += ck * float(indep.P(on, 0.5 * sign)) / (d + 1)
        got = sum(float(w) * indep.face_value(c, order, nodes[j - 1])
                  for j, w in GEN.edge_average_weights(order, which, sign).items())
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)), (got, ref)


def _generated_predictor(order, form, w, c):
    """The steps the generated predictor takes (the fluxes at the tau = 0
    nodes once, then order - 1 iterations over the later nodes, every node's
    fluxes weighted into the evolutionary modes), here for the linear flux
    F = c u in reference units, states evaluated with the independent basis."""
    nodes = [tuple(float(x) for x in p) for p in GEN.pred_nodes(order, form)]
    W = GEN.evolution_weights(order, form)
    ne = len(indep.st_modes(order)) - len(w)

    def flux_sum(e, js):
        vals = {j: indep.st_value(np.concatenate([w, e]), order, nodes[j - 1]) for j in js}
        acc = np.zeros(ne)
        for k, lin in enumerate(W):
            for (d, j), cf in lin.items():
                if j in vals:
                    acc[k] += float(cf) * c['fgh'.index(d)] * vals[j]
        return acc

    first = [j for j in range(1, len(nodes) + 1) if nodes[j - 1][3] == 0]
    later = [j for j in range(1, len(nodes) + 1) if nodes[j - 1][3] != 0]
    e = np.zeros(ne)
    a0 = flux_sum(e, first)
    if not later:
        return a0
    for _ in range(order - 1):
        e = a0 + flux_sum(e, later)
    return e


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("form", ["modal", "nodal"])
def test_generated_predictor_exact_for_linear_advection(order, form):
    # linear flux on data of degree <= M - 1: the space-time polynomial of
    # the generated steps must be w(x - c tau) after the M - 1 iterations,
    # in both the modal (Sec. IV) and the nodal (App. A-C) form
    rng = np.random.default_rng(30 + order)
    ls = len([m for m in indep.st_modes(order) if m[3] == 0])
    w = rng.normal(size=ls)
    c = np.array([0.7, -1.3, 0.4]) * 0.05 / np.array([0.1, 0.2, 0.125])
    e = _generated_predictor(order, form, w, c)
    coef = np.concatenate([w, e])
    for p in rng.uniform(-0.5, 0.5, size=(10, 4)):
        tau = p[3] + 0.5
        got = indep.st_value(coef, order, (p[0], p[1], p[2], tau))
        shifted = p[:3] - c * tau
        ref = indep.st_value(np.concatenate([w, np.zeros(len(e))]), order,
                             (shifted[0], shifted[1], shifted[2], 0.0))
        assert abs(got - ref) < 1e-13 * max(1.0, abs(ref)), (order, form, got, ref)
