"""Pins of the oracle's reconstruction (Sec. II.1, III) and Riemann fluxes
(Sec. II.3, V)."""

import numpy as np
import pytest

from oracle import basis, physics, riemann, weno
from tests import indep


def _cell_avg_of_monomial(p, lo, hi):
    return (hi ** (p + 1) - lo ** (p + 1)) / ((p + 1) * (hi - lo))


@pytest.mark.parametrize("order", [3, 4])
def test_candidates_reproduce_polynomials(order):
    # each stencil's candidate is the unique degree M-1 polynomial matching
    # the cell averages: it must return the exact Hermite moments
    rng = np.random.default_rng(order)
    mats = weno.candidate_matrices(order)
    for _ in range(3):
        m_true = rng.normal(size=order)
        # cell averages of sum m_a P_a over zone offsets via exact integration
        def avg(o):
            xs, ws = indep.gauss(4, o - 0.5, o + 0.5)
            return sum(np.dot(ws, indep.P(a, xs)) * m_true[a] for a in range(order))
        for s, st in enumerate(weno.stencils(order)):
            data = np.array([avg(o) for o in st])
            assert np.allclose(mats[s] @ data, m_true, rtol=0, atol=1e-12)


def test_smoothness_indicator_matches_paper_forms():
    # eq. (24) and (29) print IS for quadratic and cubic candidates
    rng = np.random.default_rng(1)
    S3, S4 = weno.smoothness_matrix(3), weno.smoothness_matrix(4)
    for _ in range(5):
        m = rng.normal(size=4)
        is3 = m[:3] @ S3 @ m[:3]
        assert abs(is3 - (m[1] ** 2 + 13 * m[2] ** 2 / 3)) < 1e-13
        is4 = m @ S4 @ m
        ref = (m[1] + 0.1 * m[3]) ** 2 + 13 * m[2] ** 2 / 3 + 781 * m[3] ** 2 / 20
        assert abs(is4 - ref) < 1e-12


def test_eq22_candidate_interpolates_face_values():
    # eq. (22): the face-B candidate of stencil S1 matches the face values at
    # xi = -3/2, -1/2, +1/2 (a cross-check of the Hermite basis in eq. (21))
    rng = np.random.default_rng(2)
    bm3, bm1, bp1 = rng.normal(size=3)
    b0 = (8 * bm1 - bm3 + 5 * bp1) / 12
    bx = bp1 - bm1
    bxx = (bp1 + bm3 - 2 * bm1) / 2
    p = lambda x: b0 + bx * indep.P(1, x) + bxx * indep.P(2, x)  # noqa: E731
    assert np.allclose([p(-1.5), p(-0.5), p(0.5)], [bm3, bm1, bp1], atol=1e-14)


@pytest.mark.parametrize("order", [3, 4])
def test_reconstruction_exact_for_global_polynomials(order):
    # every candidate is full order, so any convex combination reproduces a
    # global polynomial of total degree <= M-1: moments come out exactly
    rng = np.random.default_rng(10 + order)
    n = 12
    exps = [(a, b, c) for a in range(order) for b in range(order) for c in range(order)
            if a + b + c <= order - 1]
    coef = {e: rng.normal() for e in exps}
    # zone (i,j,k) centred at (i,j,k) in units of the zone size
    idx = np.arange(n, dtype=float)
    U = np.zeros((1, n, n, n))
    for (a, b, c), v in coef.items():
        ax = np.array([_cell_avg_of_monomial(a, i - 0.5, i + 0.5) for i in idx])
        by = np.array([_cell_avg_of_monomial(b, i - 0.5, i + 0.5) for i in idx])
        cz = np.array([_cell_avg_of_monomial(c, i - 0.5, i + 0.5) for i in idx])
        U[0] += v * cz[:, None, None] * by[None, :, None] * ax[None, None, :]
    what = weno.reconstruct(U, order)
    # exact modes of the global polynomial in the local frame of zone (k,j,i):
    # project onto P_a P_b P_c by Gauss quadrature
    xs, ws = indep.gauss(5, -0.5, 0.5)
    r = order - 1
    for (k, j, i) in [(r + 1, r + 2, r + 3), (6, 5, 7)]:
        for m, (a, b, c) in enumerate(basis.SPATIAL_MODES[:basis.N_SPATIAL[order]]):
            num = 0.0
            for X, wx in zip(xs, ws):
                for Y, wy in zip(xs, ws):
                    for Z, wz in zip(xs, ws):
                        val = sum(v * (i + X) ** e[0] * (j + Y) ** e[1] * (k + Z) ** e[2]
                                  for e, v in coef.items())
                        num += wx * wy * wz * val * indep.P(a, X) * indep.P(b, Y) * indep.P(c, Z)
            den = (np.dot(ws, indep.P(a, xs) ** 2) * np.dot(ws, indep.P(b, xs) ** 2)
                   * np.dot(ws, indep.P(c, xs) ** 2))
            assert abs(what[m, 0, k, j, i] - num / den) < 1e-9 * (1 + abs(num / den))


def test_minmod_slopes():
    U = np.zeros((1, 1, 1, 6))
    U[0, 0, 0] = [0.0, 1.0, 3.0, 2.0, 2.0, 5.0]
    what = weno.reconstruct(U, 2)
    # slopes along x: minmod(forward, backward); periodic wrap at the ends
    assert np.allclose(what[1, 0, 0, 0], [0.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    assert np.all(what[2] == 0) and np.all(what[3] == 0)


def _euler_state(rng, n=4):
    rho = rng.uniform(0.5, 2.0, size=n)
    v = rng.normal(size=(3, n))
    P = rng.uniform(0.5, 2.0, size=n)
    return physics.conserved(rho, v, P, None, 1.4)


def _packet(u, axis):
    return {'ub': u, 'u': u, 'f': physics.flux(u, axis, 1.4)}


@pytest.mark.parametrize("solver", ["hll", "linearized"])
def test_riemann_consistency(solver):
    rng = np.random.default_rng(3)
    u = _euler_state(rng)
    fn = riemann.hll if solver == 'hll' else riemann.linearized_euler
    for axis in range(3):
        F = fn(_packet(u, axis), _packet(u, axis), axis, 1.4)
        assert np.allclose(F, physics.flux(u, axis, 1.4), rtol=1e-14, atol=1e-14)


def test_hll_supersonic_is_upwind():
    rng = np.random.default_rng(4)
    ul = physics.conserved(np.array([1.0]), np.array([[5.0], [0.1], [0.0]]), np.array([1.0]), None, 1.4)
    ur = physics.conserved(np.array([1.2]), np.array([[5.5], [0.0], [0.2]]), np.array([0.8]), None, 1.4)
    F = riemann.hll(_packet(ul, 0), _packet(ur, 0), 0, 1.4)
    assert np.allclose(F, physics.flux(ul, 0, 1.4), rtol=1e-15)
    del rng


def _jacobian(u, axis, gamma, h=1e-6):
    n = u.shape[0]
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = h * max(1.0, abs(u[k]))
        J[:, k] = (physics.flux(u + e, axis, gamma) - physics.flux(u - e, axis, gamma)) / (2 * e[k])
    return J


def test_linearized_dissipation_is_abs_jacobian():
    # R |Lambda| L du equals |A| du with A the (finite-difference) flux
    # Jacobian at the frozen state, diagonalised by numpy
    rng = np.random.default_rng(6)
    for axis in range(3):
        u = _euler_state(rng, 1)[:, 0]
        A = _jacobian(u, axis, 1.4)
        lam, R = np.linalg.eig(A)
        absA = (R @ np.diag(np.abs(lam.real)) @ np.linalg.inv(R)).real
        du = rng.normal(size=5)
        got = riemann.euler_eigen_dissipation(u[:, None], u[:, None], du[:, None], axis, 1.4)[:, 0]
        assert np.allclose(got, absA @ du, rtol=1e-6, atol=1e-6)


def test_gaussian_units_beta():
    # the MHD blast ambient state (P = 0.1, B = 20/sqrt(3) in each component)
    # has plasma beta 0.00628 only in Gaussian units, beta = 8 pi P / B^2
    B = np.full(3, 20.0 / np.sqrt(3.0))
    beta = 8 * np.pi * 0.1 / (B @ B)
    assert abs(beta - 0.00628) < 5e-6
    u = physics.conserved(np.array([1.0]), np.zeros((3, 1)), np.array([0.1]), B[:, None], 5.0 / 3.0)
    assert abs(u[4, 0] - (0.1 / (2.0 / 3.0) + (B @ B) / (8 * np.pi))) < 1e-12
