"""Pins of the oracle's basis, nodal-to-modal flux rules, evolution equations
and predictor (Sec. II.1-II.2, Sec. IV, App. A) against facts the paper and
the mathematics fix."""

import os

import numpy as np
import pytest
import sympy as sp

from oracle import basis
from oracle import predictor as pr
from tests import indep


@pytest.mark.parametrize("a", [0, 1, 2, 3])
def test_basis_is_monic_legendre(a):
    # eq. (9): P_a is the Legendre polynomial rescaled to [-1/2, 1/2], monic
    x = np.linspace(-0.5, 0.5, 17)
    assert np.allclose(basis.P(a, x), indep.P(a, x), rtol=0, atol=1e-15)


def test_basis_orthogonal_zero_mean():
    x, w = indep.gauss(8, -0.5, 0.5)
    G = np.array([[np.dot(w, basis.P(a, x) * basis.P(b, x)) for b in range(4)] for a in range(4)])
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-16)
    assert np.allclose(np.diag(G), [1.0, 1.0 / 12, 1.0 / 180, 1.0 / 2800], rtol=1e-14)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_mode_order_matches_paper(order):
    # eq. (10)-(16)
    assert basis.spacetime_modes(order) == indep.st_modes(order)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_node_sets_are_mirror_symmetric(order):
    nodes = {tuple(float(c) for c in n) for n in pr.NODES_MODAL[order]}
    assert len(nodes) == {2: 7, 3: 20, 4: 42}[order]
    for axis in range(3):
        for n in nodes:
            m = list(n)
            m[axis] = -m[axis]
            assert tuple(m) in nodes


def _rule_exactness(order, seed):
    """Apply the oracle's rule to nodal values of random polynomials in the
    space-time span; every mode it returns must come out exactly."""
    rng = np.random.default_rng(seed)
    L = basis.N_SPACETIME[order]
    cf, cg, ch = rng.normal(size=(3, L))
    nodes = pr.NODES_MODAL[order]
    fv = [None] + [indep.st_value(cf, order, n) for n in nodes]
    gv = [None] + [indep.st_value(cg, order, n) for n in nodes]
    hv = [None] + [indep.st_value(ch, order, n) for n in nodes]
    modes = pr.FLUX_MODES[order](fv, gv, hv)
    ref = {'f': cf, 'g': cg, 'h': ch}
    for key, val in modes.items():
        k = int(key[1:])
        assert abs(val - ref[key[0]][k - 1]) < 1e-12, (order, key, val, ref[key[0]][k - 1])
    return modes


@pytest.mark.parametrize("order", [2, 3, 4])
def test_flux_rules_exact_on_span(order):
    # eq. (33), (40)-(42), (49)-(51)
    for seed in range(3):
        _rule_exactness(order, seed)


def _galerkin_matrices(order):
    """Exact Galerkin operators of the space-time predictor.

    For every evolutionary test function phi_k:
      int phi_k (d_tau u + d_xi f + d_eta g + d_zeta h) = 0
    over [-1/2,1/2]^3 x [0,1], with u, f, g, h in the full space-time span.
    Returns (E, Kf, Kg, Kh) with u_evol = E_f f + E_g g + E_h h (rationals).
    """
    x, t = sp.symbols('x t')
    Pp = [sp.Integer(1), x, x ** 2 - sp.Rational(1, 12), x ** 3 - sp.Rational(3, 20) * x]

    def i_pp(a, b):
        return sp.integrate(Pp[a] * Pp[b], (x, -sp.Rational(1, 2), sp.Rational(1, 2)))

    def i_pdp(a, b):
        return sp.integrate(Pp[a] * sp.diff(Pp[b], x), (x, -sp.Rational(1, 2), sp.Rational(1, 2)))

    def i_tt(d, e):
        return sp.integrate(t ** d * t ** e, (t, 0, 1))

    def i_tdt(d, e):
        return sp.integrate(t ** d * sp.diff(t ** e, t), (t, 0, 1))

    modes = indep.st_modes(order)
    ls = basis.N_SPATIAL[order]
    evol = list(range(ls, len(modes)))
    L = len(modes)
    Mt = sp.zeros(len(evol), len(evol))
    K = [sp.zeros(len(evol), L) for _ in range(3)]
    for r, k in enumerate(evol):
        ak = modes[k]
        for c, m in enumerate(evol):
            am = modes[m]
            Mt[r, c] = (i_pp(ak[0], am[0]) * i_pp(ak[1], am[1]) * i_pp(ak[2], am[2])
                        * i_tdt(ak[3], am[3]))
        for m in range(L):
            am = modes[m]
            for axis in range(3):
                f = [i_pp(ak[i], am[i]) for i in range(3)]
                f[axis] = i_pdp(ak[axis], am[axis])
                K[axis][r, m] = f[0] * f[1] * f[2] * i_tt(ak[3], am[3])
    Minv = Mt.inv()
    return [-(Minv * Kd) for Kd in K]


@pytest.mark.parametrize("order", [2, 3, 4])
def test_evolution_equations_match_galerkin(order):
    # eq. (30), (36), (45) against the Galerkin weak form derived here
    E = [np.array(e.tolist(), dtype=np.float64) for e in _galerkin_matrices(order)]
    rng = np.random.default_rng(7)
    L = basis.N_SPACETIME[order]
    for _ in range(3):
        fv, gv, hv = rng.normal(size=(3, L))
        ref = E[0] @ fv + E[1] @ gv + E[2] @ hv
        r = {}
        for name, vec in (('f', fv), ('g', gv), ('h', hv)):
            for k in range(1, L + 1):
                r['%s%d' % (name, k)] = vec[k - 1]
        got = np.array(pr.EVOLVE[order](r))
        assert np.allclose(got, ref, rtol=0, atol=1e-13), (got, ref)


def test_nodal_A4_reading():
    # (A.4) derived from the nodal basis (A.2): the z-difference uses node 4
    x, y, z, t = sp.symbols('x y z t')
    Pn = [1 - 2 * x - 2 * y - 2 * z - t, 2 * x, 2 * y, 2 * z, t]
    nodes = [(0, 0, 0, 0), (sp.Rational(1, 2), 0, 0, 0), (0, sp.Rational(1, 2), 0, 0),
             (0, 0, sp.Rational(1, 2), 0), (0, 0, 0, 1)]
    for i, p in enumerate(Pn):
        for j, n in enumerate(nodes):
            assert p.subs({x: n[0], y: n[1], z: n[2], t: n[3]}) == (1 if i == j else 0)
    ub = sp.symbols('u1:6')
    hb = sp.symbols('h1:6')
    u = sum(ub[i] * Pn[i] for i in range(5))
    hz = sum(hb[i] * Pn[i] for i in range(5))
    box = [(x, -sp.Rational(1, 2), sp.Rational(1, 2)), (y, -sp.Rational(1, 2), sp.Rational(1, 2)),
           (z, -sp.Rational(1, 2), sp.Rational(1, 2)), (t, 0, 1)]
    eq = sp.integrate(Pn[4] * (sp.diff(u, t) + sp.diff(hz, z)), *box)
    sol = sp.solve(eq, ub[4])[0]
    assert sp.simplify(sol - (ub[0] - 2 * (hb[3] - hb[0]))) == 0


def test_nodal_B2_B3_from_galerkin():
    # (B.2) and (B.3) at their fixed point are the continuous-Galerkin
    # equations written with the nodal basis of the fifteen nodes (B.1):
    # interpolate u and the scaled fluxes f, g, h on that basis, require the
    # residual u_t + f_x + g_y + h_z to be orthogonal to the basis functions
    # of the five later nodes, and solve for their nodal values.  This pins
    # every printed flux coefficient of (B.2)-(B.3) (sources are zero here).
    x, y, z, t = sp.symbols('x y z t')
    h = sp.Rational(1, 2)
    nodes = [(0, 0, 0, 0), (h, 0, 0, 0), (-h, 0, 0, 0), (0, h, 0, 0), (0, -h, 0, 0),
             (0, 0, h, 0), (0, 0, -h, 0), (0, h, h, 0), (h, 0, h, 0), (h, h, 0, 0),
             (0, 0, 0, h), (h, 0, 0, h), (0, h, 0, h), (0, 0, h, h), (0, 0, 0, 1)]
    assert [tuple(float(c) for c in n) for n in nodes] == pr.NODES_NODAL_3
    p2 = lambda s: s ** 2 - sp.Rational(1, 12)  # noqa: E731
    modes = [sp.Integer(1), x, y, z, p2(x), p2(y), p2(z), x * y, y * z, x * z,
             t, t ** 2, x * t, y * t, z * t]
    V = sp.Matrix([[m.subs({x: n[0], y: n[1], z: n[2], t: n[3]}) for m in modes] for n in nodes])
    Vi = V.inv()
    Pn = [sp.expand(sum(modes[m] * Vi[m, i] for m in range(15))) for i in range(15)]
    u, f, g, hh = (sp.symbols(s + '1:16') for s in ('u', 'f', 'g', 'h'))
    interp = lambda c: sum(c[i] * Pn[i] for i in range(15))  # noqa: E731
    R = sp.diff(interp(u), t) + sp.diff(interp(f), x) + sp.diff(interp(g), y) + sp.diff(interp(hh), z)
    box = [(x, -h, h), (y, -h, h), (z, -h, h), (t, 0, 1)]
    eqs = [sp.integrate(sp.expand(w * R), *box) for w in Pn[10:]]
    sol = sp.solve(eqs, u[10:], dict=True)[0]
    # the oracle's (B.2) then (B.3), every nodal value and flux an
    # independent random number (later-node fluxes at their fixed point)
    rng = np.random.default_rng(3)
    vals = {s: rng.normal() for s in list(u[:10]) + list(f) + list(g) + list(hh)}
    one = lambda c, n: [None] + [vals[c[k]] for k in range(n)]  # noqa: E731
    F, G, H = one(f, 15), one(g, 15), one(hh, 15)
    got = pr.nodal3_b3(pr.nodal3_b2(one(u, 10), F, G, H), F, G, H)
    for k in range(11, 16):
        ref = float(sol[u[k - 1]].subs(vals))
        assert abs(got[k] - ref) < 1e-12, (k, got[k], ref)


def test_nodal_B5_recovers_the_modes():
    # (B.5) inverts the nodal values of (B.1) back to modes 11-15: a random
    # space-time polynomial, evaluated at the nodes by the tests' own
    # evaluator, must give back its own evolutionary modes
    rng = np.random.default_rng(8)
    uhat = rng.normal(size=15)
    val = [None] + [indep.st_value(uhat, 3, p) for p in pr.NODES_NODAL_3]
    later = {k: val[k] for k in range(11, 16)}
    got = pr.nodal3_b5(val, later)
    assert np.allclose(got, uhat[10:], rtol=0, atol=1e-13)


def _golden(name):
    with open(os.path.join(os.path.dirname(__file__), 'golden', name)) as fh:
        return [line.split() for line in fh if line.strip() and not line.startswith('#')]


def _read_app_c():
    rows = []
    for name, d, den, *pairs in _golden('app_c_nodal4.txt'):
        coef = {int(k): int(v) for k, v in (p.split(':') for p in pairs)}
        rows.append((name, d, int(den), coef))
    return rows


def test_nodal_C2_C3_printed_coefficients():
    # every coefficient the paper prints in (C.2) (temporaries q21 .. q35)
    # and (C.3) (evolutionary equations u21 .. u35) -- f, g, h, s and the
    # starting nodal value, unprinted ones being zero -- equals the exact
    # rational Galerkin map over the nodes (C.1)
    from fractions import Fraction
    ex = pr.nodal_maps_exact(4)
    A = {'f': ex['Af'], 'g': ex['Ag'], 'h': ex['Ah'], 's': ex['As']}
    t0, lt = ex['t0'], ex['lt']
    rows = _read_app_c()
    assert len(rows) == 135
    covered = set()
    for name, d, den, coef in rows:
        k = int(name[1:]) - 21          # later node 21 + k
        assert set(coef) <= {j + 1 for j in (t0 if name[0] == 'q' else lt)}, name
        if d == 'u':
            for jj, j in enumerate(t0):
                assert ex['Au'][k][jj] == Fraction(coef.get(j + 1, 0), den), (name, j + 1)
            covered.add((name, d))
            continue
        for j in (t0 if name[0] == 'q' else lt):
            assert A[d][k][j] == Fraction(coef.get(j + 1, 0), den), (name, d, j + 1)
        covered.add((name, d))
    # every row of every map is printed: q (tau = 0 columns) and u (later
    # columns) for each direction and the source, and the u start of each q
    for k in range(21, 36):
        for d in 'fghs':
            assert ('q%d' % k, d) in covered and ('u%d' % k, d) in covered
        assert ('q%d' % k, 'u') in covered


def test_nodal_C5_printed_modes_from_nodes():
    # (C.5), the modes 21-35 from the nodal values, against the exact
    # inverse of the nodal evaluation; the only difference is the misprint
    # in the u35 line (u_24 printed for u_26)
    from fractions import Fraction
    C = pr.nodal_maps_exact(4)['C']
    diffs = []
    for name, fac, *pairs in _golden('app_c_c5.txt'):
        m = int(name[1:]) - 1
        coef = {int(k): int(v) for k, v in (p.split(':') for p in pairs)}
        for j in range(35):
            want = Fraction(fac) * coef.get(j + 1, 0)
            if C[m][j] != want:
                diffs.append((m + 1, j + 1, C[m][j], want))
    assert diffs == [(35, 24, 0, -12), (35, 26, -12, 0)], diffs


def test_nodal_C4_printed_nodes_from_modes():
    # (C.4), the twenty tau = 0 nodal values from the spatial modes through
    # the temporaries q1-q3 as printed, equals direct evaluation of the
    # spatial polynomial (eq. 9, 12) at the nodes (C.1), for every mode
    from fractions import Fraction as F
    h = F(1, 2)

    def c4(w):
        w = [None] + w
        q1 = F(1, 4) * w[2] - F(1, 8) * (w[8] + w[10]) \
            + (-21 * w[11] + 40 * w[16] + 40 * w[18] + 60 * w[20]) / 960
        q2 = F(1, 4) * w[3] - F(1, 8) * (w[8] + w[9]) \
            + (-21 * w[12] + 40 * w[14] + 40 * w[19] + 60 * w[20]) / 960
        q3 = F(1, 4) * w[4] - F(1, 8) * (w[9] + w[10]) \
            + (-21 * w[13] + 40 * w[15] + 40 * w[17] + 60 * w[20]) / 960
        u = {1: w[1] - (w[5] + w[6] + w[7]) / 12}
        u[3] = u[1] + h * w[2] + F(1, 4) * w[5] + F(1, 20) * w[11] - (w[16] + w[18]) / 24
        u[4] = 2 * u[1] - u[3] + h * w[5]
        u[5] = u[1] + h * w[3] + F(1, 4) * w[6] + F(1, 20) * w[12] - (w[14] + w[19]) / 24
        u[6] = 2 * u[1] - u[5] + h * w[6]
        u[7] = u[1] + h * w[4] + F(1, 4) * w[7] + F(1, 20) * w[13] - (w[15] + w[17]) / 24
        u[8] = 2 * u[1] - u[7] + h * w[7]
        u[9] = u[5] + u[7] - u[1] + F(1, 4) * w[9] + F(1, 8) * (w[17] + w[19])
        u[11] = u[3] + u[7] - u[1] + F(1, 4) * w[10] + F(1, 8) * (w[15] + w[18])
        u[13] = u[3] + u[5] - u[1] + F(1, 4) * w[8] + F(1, 8) * (w[14] + w[16])
        u[10] = 2 * u[7] - u[11] + h * w[5] + F(1, 4) * w[15]
        u[12] = 2 * u[3] - u[13] + h * w[6] + F(1, 4) * w[16]
        u[14] = 2 * u[5] - u[9] + h * w[7] + F(1, 4) * w[19]
        u[2] = u[11] + u[9] - u[7] + F(1, 4) * w[8] + F(1, 8) * (w[14] + w[16] + w[20])
        u[15] = 2 * u[8] - u[14] - q1 + F(1, 16) * w[5] + h * w[6] \
            - F(1, 32) * (w[14] + w[15]) - F(1, 4) * w[17]
        u[17] = 2 * u[4] - u[10] - q2 + F(1, 16) * w[6] + h * w[7] \
            - F(1, 32) * (w[16] + w[17]) - F(1, 4) * w[18]
        u[19] = 2 * u[6] - u[12] - q3 + h * w[5] + F(1, 16) * w[7] - F(1, 4) * w[14] \
            - F(1, 32) * (w[18] + w[19])
        u[16], u[18], u[20] = u[15] + 2 * q1, u[17] + 2 * q2, u[19] + 2 * q3
        return u

    def p1(a, x):      # eq. (9) in exact arithmetic
        return [F(1), x, x * x - F(1, 12), x ** 3 - F(3, 20) * x][a]

    nodes = [tuple(F(c).limit_denominator(12) for c in x) for x in pr.NODES_NODAL_4[:20]]
    for unit in range(20):
        w = [F(0)] * 20
        w[unit] = F(1)
        u = c4(w)
        a, b, c = basis.SPATIAL_MODES[unit]
        for j, x in enumerate(nodes):
            assert u[j + 1] == p1(a, x[0]) * p1(b, x[1]) * p1(c, x[2]), (unit + 1, j + 1)


def test_nodal_C6_printed_source_average():
    # (C.6): dt S-bar = (15 s1 - 2 (s3 .. s8) - 27 s21 + 6 (s22 .. s27)
    # + 9 s31 + 3 s35) / 24, the integrals of the nodal basis functions
    from fractions import Fraction
    w = pr.nodal_maps_exact(4)['wbar']
    printed = {1: 15, 3: -2, 4: -2, 5: -2, 6: -2, 7: -2, 8: -2, 21: -27, 22: 6, 23: 6, 24: 6,
               25: 6, 26: 6, 27: 6, 31: 9, 35: 3}
    assert w == [Fraction(printed.get(j, 0), 24) for j in range(1, 36)]


def test_nodal_map_at_third_order_is_B2_B3():
    # the same Galerkin construction over the nodes (B.1) gives the
    # explicit (B.2)-(B.3) of the third-order oracle
    nodes, t0, lt, Au, Af, Ag, Ah, C = pr.nodal_update_map(3)
    rng = np.random.default_rng(5)
    u = [None] + list(rng.normal(size=10))
    F, G, H = ([None] + list(rng.normal(size=15)) for _ in range(3))
    got = pr.nodal3_b3(pr.nodal3_b2(u, F, G, H), F, G, H)
    ref = Au @ np.array(u[1:]) + Af @ np.array(F[1:]) + Ag @ np.array(G[1:]) + Ah @ np.array(H[1:])
    for k in range(11, 16):
        assert abs(got[k] - ref[k - 11]) < 1e-12


def test_nodal_source_terms_from_galerkin():
    # the source part of the same Galerkin construction reproduces the
    # printed source terms of (A.4), (B.2)-(B.3) and the averages (A.7),
    # (B.6): the explicit third-order source functions of the oracle against
    # the map, every source an independent random number
    As2, w2 = pr.nodal_source_map(2)
    assert np.allclose(As2[0], [1.0 / 3.0, 0, 0, 0, 2.0 / 3.0], atol=1e-14)
    assert np.allclose(w2, [0.5, 0, 0, 0, 0.5], atol=1e-14)
    As3, w3 = pr.nodal_source_map(3)
    rng = np.random.default_rng(21)
    s = [None] + list(rng.normal(size=15))
    q = pr.nodal3_b2_source(s)
    later = pr.nodal3_b3_source(s)
    ref = As3 @ np.array(s[1:])
    for k in range(11, 16):
        assert abs(q[k] + later[k] - ref[k - 11]) < 1e-13, k
    assert abs(pr.nodal3_b6(s) - w3 @ np.array(s[1:])) < 1e-13


def _linear_flux(adv):
    return lambda u, axis: adv[axis] * u


def _spatial_value(what, order, point):
    ls = basis.N_SPATIAL[order]
    c = np.zeros(basis.N_SPACETIME[order])
    c[:ls] = what
    return indep.st_value(c, order, (point[0], point[1], point[2], 0.0))


@pytest.mark.parametrize("order,form", [(2, 'modal'), (2, 'nodal'), (3, 'modal'), (3, 'nodal'),
                                        (4, 'modal'), (4, 'nodal')])
def test_predictor_exact_for_linear_advection(order, form):
    # constant-coefficient linear flux on data of degree <= M-1: the
    # space-time polynomial must be w(x - c tau) after M-1 iterations
    rng = np.random.default_rng(11 + order)
    ls = basis.N_SPATIAL[order]
    what = rng.normal(size=(ls, 1))
    adv = np.array([0.7, -1.3, 0.4])
    dt, dx = 0.05, (0.1, 0.2, 0.125)
    c = adv * dt / np.array(dx)
    if form == 'nodal':
        nodal = {2: pr.predict_nodal_2, 3: pr.predict_nodal_3, 4: pr.predict_nodal_4}[order]
        uhat = nodal(what, dt, dx, 1.4, flux_fn=_linear_flux(adv))
    else:
        uhat = pr.predict_modal(what, order, dt, dx, 1.4, flux_fn=_linear_flux(adv))
    for p in rng.uniform(-0.5, 0.5, size=(10, 4)):
        tau = p[3] + 0.5
        got = indep.st_value(uhat[:, 0], order, (p[0], p[1], p[2], tau))
        ref = _spatial_value(what[:, 0], order, p[:3] - c * tau)
        assert abs(got - ref) < 1e-13
