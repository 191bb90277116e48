"""Positivity of the zone polynomials: the check of the paper's scheme and
an optional safeguard (the paper describes no positivity treatment).

Two modes, chosen by ``OracleConfig.positivity``:

* ``'check'`` (the default, the paper's scheme): nothing is changed; the
  polynomials are evaluated at the check sets below and ``NonPhysical`` is
  raised if any point has rho <= 0 or P <= 0, since the fluxes and wave
  speeds there have no meaning.  The step is the paper's step wherever it
  does not raise.
* ``'limit'`` (an opt-in added here): the Zhang-Shu scaling described next.

Component-wise WENO of the conserved variables (Sec. II.1, VII) can put
negative density or pressure at the predictor and facial nodes next to strong
blasts (the Sedov-type overpressure workload does so within two steps), which
makes the fluxes and wave speeds meaningless.  The safeguard is the scaling
limiter of Zhang & Shu (J. Comput. Phys. 229, 2010): every non-constant mode
of a zone is multiplied by one factor theta in [0, 1], the largest for which
density and pressure stay above eps times their zone-average values at every
point of the zone's check set.  The zone average is untouched, so the scheme
stays conservative, and theta = 1 (no change at all) wherever the polynomial
is already positive there, so smooth solutions and every other pin are
unaffected.

For MHD the pressure includes B^2 / 8 pi, the facial check set holds every
facial node (the edge averages use them all) and the pressure bound is
located by bisection.

Check sets.  Before the predictor the spatial modes are checked at the
spatial positions of every predictor node (eq. 31/37/46, or A.1) and of every
facial node that enters a face average; after the predictor all modes are
checked at those facial nodes of the six sides and at the six face
barycentres (eq. 54), the points where the step evaluates the space-time
polynomial.  The facial nodes entering the face average of (D.5)/(D.10)/(D.15)
composed with (D.4)/(D.9)/(D.14) are nodes 1-4 of (D.1), nodes 1 and 6-10 of
(D.6) and nodes 1, 2, 5, 6, 9, 14-19 and 24 of (D.11); the others carry zero
weight.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .basis import N_SPATIAL, evaluate
from .faces import FACE_NODES, zone_point
from .predictor import NODES_MODAL, NODES_NODAL

EPS_REL = 1.0e-8

MODES = ('check', 'limit')


class NonPhysical(ArithmeticError):
    """A check point of some zone has rho <= 0 or P <= 0 (check mode)."""


# 1-based facial nodes with a nonzero weight in the face average
FACE_AVERAGE_NODES = {2: [1, 2, 3, 4], 3: [1, 6, 7, 8, 9, 10],
                      4: [1, 2, 5, 6, 9, 14, 15, 16, 17, 18, 19, 24]}


def facial_check_points(order, all_nodes=False):
    """Space-time points of the facial check set, six sides, fixed order
    (every facial node when the edge averages of MHD use them all)."""
    pts = []
    nodes = range(1, len(FACE_NODES[order]) + 1) if all_nodes else FACE_AVERAGE_NODES[order]
    for d in range(3):
        for s in (-1, 1):
            for j in nodes:
                t1, t2, tau = FACE_NODES[order][j - 1]
                pts.append(zone_point(d, s, t1, t2, tau))
            pts.append(zone_point(d, s, 0.0, 0.0, 0.5))
    return [tuple(float(c) for c in p) for p in pts]


def spatial_check_points(order, form, all_nodes=False):
    """Distinct spatial positions of the predictor nodes and of the facial
    check points (tau set to 0)."""
    pts = list(NODES_NODAL[order] if form == 'nodal' else NODES_MODAL[order])
    pts += facial_check_points(order, all_nodes)
    return sorted(set((float(p[0]), float(p[1]), float(p[2]), 0.0) for p in pts))


def _pressure_like(u, gamma):
    """(gamma-1)(E - m^2 / 2 rho [- B^2 / 8 pi]) of an Euler or MHD state."""
    m2 = u[1] ** 2 + u[2] ** 2 + u[3] ** 2
    mag = 0.0
    if u.shape[0] == 8:
        mag = (u[5] ** 2 + u[6] ** 2 + u[7] ** 2) / (8.0 * np.pi)
    return (gamma - 1.0) * (u[4] - 0.5 * m2 / u[0] - mag)


def _pressure_root_bisect(ubar, du, eps_p, gamma, iters=60):
    """MHD: the pressure along ubar + t du is concave where rho > 0 (a cubic
    after clearing rho); the largest t in [0, 1] with pressure >= eps_p and
    rho > 0 up to it is found by bisection (lower end kept)."""
    lo = np.zeros_like(ubar[0])
    hi = np.ones_like(ubar[0])
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        v = ubar + mid * du
        ok = (v[0] > 0.0) & (_pressure_like(v, gamma) >= eps_p)
        lo = np.where(ok, mid, lo)
        hi = np.where(ok, hi, mid)
    return lo


def _pressure_root(ubar, du, eps_p, gamma):
    """Smallest t in (0, 1] with pressure(ubar + t du) = eps_p.

    rho(t) (E(t) - e) - |m(t)|^2 / 2 is the quadratic a t^2 + b t + c with
    e = eps_p / (gamma - 1); c > 0 at t = 0 and the value at t = 1 is < 0.
    """
    e = eps_p / (gamma - 1.0)
    r0, m0, E0 = ubar[0], ubar[1:4], ubar[4]
    dr, dm, dE = du[0], du[1:4], du[4]
    a = dr * dE - 0.5 * (dm * dm).sum(axis=0)
    b = r0 * dE + dr * (E0 - e) - (m0 * dm).sum(axis=0)
    c = r0 * (E0 - e) - 0.5 * (m0 * m0).sum(axis=0)
    with np.errstate(all='ignore'):
        disc = np.sqrt(np.maximum(b * b - 4.0 * a * c, 0.0))
        qq = -0.5 * (b + np.where(b >= 0.0, disc, -disc))
        t1 = qq / a
        t2 = c / qq
        lin = -c / b
    big = 2.0
    t1 = np.where(np.isfinite(t1) & (t1 >= 0.0), t1, big)
    t2 = np.where(np.isfinite(t2) & (t2 >= 0.0), t2, big)
    t = np.minimum(t1, t2)
    t = np.where(a == 0.0, lin, t)
    return np.clip(t, 0.0, 1.0)


def scale_factor(ubar, values, gamma):
    """theta in [0, 1] of one zone polynomial given its point values."""
    rho_eps = EPS_REL * ubar[0]
    p_bar = _pressure_like(ubar, gamma)
    p_eps = EPS_REL * p_bar
    theta = np.ones_like(ubar[0])
    for u in values:
        with np.errstate(divide='ignore', invalid='ignore'):
            t = np.where(u[0] < rho_eps, (ubar[0] - rho_eps) / (ubar[0] - u[0]), 1.0)
        theta = np.minimum(theta, t)
    theta_rho = theta
    root = _pressure_root if ubar.shape[0] == 5 else _pressure_root_bisect
    for u in values:
        v = ubar + theta_rho * (u - ubar)
        p = _pressure_like(v, gamma)
        t = np.where(p < p_eps, theta_rho * root(ubar, v - ubar, p_eps, gamma), theta_rho)
        theta = np.minimum(theta, t)
    return theta


def limit_spatial(what, order, form, gamma):
    """Scale w_2..w_{L_S} so the spatial polynomial is positive at the
    spatial positions of the check set."""
    pts = spatial_check_points(order, form, all_nodes=what.shape[1] == 8)
    vals = [evaluate(_as_spacetime(what, order), order, p) for p in pts]
    theta = scale_factor(what[0], vals, gamma)
    out = what.copy()
    out[1:] = out[1:] * theta
    return out


def _as_spacetime(what, order):
    from .basis import N_SPACETIME
    uh = np.zeros((N_SPACETIME[order],) + what.shape[1:])
    uh[:N_SPATIAL[order]] = what
    return uh


def limit_spacetime(uhat, order, form, gamma):
    """Scale every mode but the zone average so the space-time polynomial is
    positive at the facial check points."""
    vals = [evaluate(uhat, order, p) for p in facial_check_points(order, uhat.shape[1] == 8)]
    theta = scale_factor(uhat[0], vals, gamma)
    out = uhat.copy()
    out[1:] = out[1:] * theta
    return out


def _check(values, gamma, where, mask=None):
    """Raise NonPhysical if any of the point states has rho <= 0 or P <= 0
    (or a non-finite value), in the zones where ``mask`` is set (all zones
    without one)."""
    bad = None
    for u in values:
        with np.errstate(divide='ignore', invalid='ignore'):
            ok = (u[0] > 0.0) & (_pressure_like(u, gamma) > 0.0)
        b = ~ok
        bad = b if bad is None else bad | b
    if bad is not None and mask is not None:
        bad = bad & mask
    if bad is not None and bad.any():
        raise NonPhysical('%s: %d zone(s) with rho <= 0 or P <= 0 at a check point'
                          % (where, int(bad.sum())))


def check_spatial(what, order, form, gamma, mask=None):
    """The check mode's test of the spatial polynomial at the spatial check
    set (before the predictor)."""
    pts = spatial_check_points(order, form, all_nodes=what.shape[1] == 8)
    _check([evaluate(_as_spacetime(what, order), order, p) for p in pts], gamma, 'spatial', mask)


def check_spacetime(uhat, order, form, gamma, mask=None):
    """The check mode's test of the space-time polynomial at the facial
    check set (after the predictor)."""
    pts = facial_check_points(order, uhat.shape[1] == 8)
    _check([evaluate(uhat, order, p) for p in pts], gamma, 'space-time', mask)


def safeguard_spatial(what, order, form, gamma, mode, mask=None):
    """The spatial polynomial after the positivity handling of ``mode``
    (the check restricted to the zones of ``mask`` if given)."""
    if mode == 'limit':
        return limit_spatial(what, order, form, gamma)
    if mode != 'check':
        raise ValueError('positivity mode %r' % (mode,))
    check_spatial(what, order, form, gamma, mask)
    return what


def safeguard_spacetime(uhat, order, form, gamma, mode, mask=None):
    """The space-time polynomial after the positivity handling of ``mode``
    (the check restricted to the zones of ``mask`` if given)."""
    if mode == 'limit':
        return limit_spacetime(uhat, order, form, gamma)
    if mode != 'check':
        raise ValueError('positivity mode %r' % (mode,))
    check_spacetime(uhat, order, form, gamma, mask)
    return uhat


def limited_zones(what, uhat, order, form, gamma):
    """Number of zones the limit mode scales (theta < 1) before and after the
    predictor, for reporting."""
    pts = spatial_check_points(order, form, all_nodes=what.shape[1] == 8)
    th_s = scale_factor(what[0], [evaluate(_as_spacetime(what, order), order, p) for p in pts],
                        gamma)
    vals = [evaluate(uhat, order, p) for p in facial_check_points(order, uhat.shape[1] == 8)]
    th_t = scale_factor(uhat[0], vals, gamma)
    return int((th_s < 1.0).sum()), int((th_t < 1.0).sum())
