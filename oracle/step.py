"""One ADER-CG time step on a periodic Cartesian mesh (Sec. II).

step = reconstruction (Sec. II.1) -> space-time predictor (Sec. II.2, IV,
App. A) -> face-side quantities and Riemann fluxes (Sec. II.3, V, App. D) ->
one-step finite-volume update (eq. 6).

Time step (the paper gives only the CFL numbers, 0.3 in 3D): the reading
here is dt = C / max_zones sum_d (|v_d| + c_f,d) / dx_d with the zone-average
state.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from dataclasses import dataclass

import numpy as np

from .bweno import zone_b_mean, zone_b_modes
from .faces import face_side_packet, transverse_axes
from .physics import primitives, fast_speed
from .positivity import safeguard_spatial, safeguard_spacetime
from .predictor import (predict_modal, predict_modal_source, predict_nodal_2, predict_nodal_3,
                        predict_nodal_4, predict_nodal_source, source_average)
from .riemann import (hll, hll_combine, hll_speeds, linearized_euler, linearized_mhd_combine,
                      mhd_abs_jacobian)
from .weno import reconstruct


@dataclass
class OracleConfig:
    order: int = 3                 # 2, 3 or 4
    form: str = 'modal'            # 'modal' (Sec. IV) or 'nodal' (App. A, B, C)
    riemann: str = 'hll'           # 'hll' or 'linearized'
    gamma: float = 1.4
    lengths: tuple = (1.0, 1.0, 1.0)   # domain (lx, ly, lz)
    zone_size: tuple = None            # (dx, dy, dz); overrides ``lengths``
    source: object = None              # S(u), a non-stiff source (Euler)
    # 'check': the paper's scheme, NonPhysical raised where rho <= 0 or
    # P <= 0 at a check point; 'limit': the Zhang-Shu scaling (opt-in)
    positivity: str = 'check'
    # zones (bool, (nz, ny, nx)) the check mode tests; None: all
    check_mask: object = None

    def spacing(self, shape):
        if self.zone_size is not None:
            return tuple(self.zone_size)
        nz, ny, nx = shape
        return (self.lengths[0] / nx, self.lengths[1] / ny, self.lengths[2] / nz)

    def ghost(self, mhd=False):
        """Zones of neighbourhood one zone's update depends on, per side."""
        if mhd:
            return 2 * self.order + 1
        return {2: 2, 3: 3, 4: 4}[self.order]


def _nb(arr, axis, o):
    return np.roll(arr, -o, axis=arr.ndim - 1 - axis)


def compute_dt(U, cfg, cfl, B=None):
    """dt = cfl / max_zones sum_d (|v_d| + c_d) / dx_d (for MHD c_d is the
    fast speed with the zone field taken as the mean of its face values)."""
    dx = cfg.spacing(U.shape[1:])
    if B is not None:
        U = np.concatenate([U, zone_b_mean(B)])
    rho, v, P, _ = primitives(U, cfg.gamma)
    rate = np.zeros_like(rho)
    for d in range(3):
        rate = rate + (np.abs(v[d]) + fast_speed(U, d, cfg.gamma)) / dx[d]
    return cfl / rate.max()


def predictor(U, dt, cfg, B=None):
    """Spatial reconstruction (for MHD the hydro variables plus the zone
    field of Sec. III) followed by the space-time predictor, each followed by
    the positivity handling of ``cfg.positivity`` (the check, or the
    scaling)."""
    dx = cfg.spacing(U.shape[1:])
    what = reconstruct(U, cfg.order)
    if B is not None:
        what = np.concatenate([what, zone_b_modes(B, cfg.order)], axis=1)
    what = safeguard_spatial(what, cfg.order, cfg.form, cfg.gamma, cfg.positivity, cfg.check_mask)
    if cfg.form == 'nodal':
        if cfg.order == 2:
            uhat = predict_nodal_2(what, dt, dx, cfg.gamma)
        elif cfg.order == 3:
            uhat = predict_nodal_3(what, dt, dx, cfg.gamma)
        else:
            uhat = predict_nodal_4(what, dt, dx, cfg.gamma)
    else:
        uhat = predict_modal(what, cfg.order, dt, dx, cfg.gamma)
    return safeguard_spacetime(uhat, cfg.order, cfg.form, cfg.gamma, cfg.positivity,
                               cfg.check_mask)


def face_fluxes(uhat, cfg):
    """Numerical flux at the lower face of every zone along each axis."""
    riemann = {'hll': hll, 'linearized': linearized_euler}[cfg.riemann]
    out = []
    for d in range(3):
        plus = face_side_packet(uhat, cfg.order, d, +1, cfg.gamma)
        minus = face_side_packet(uhat, cfg.order, d, -1, cfg.gamma)
        left = {k: _nb(v, d, -1) for k, v in plus.items()}   # zone i-1, top side
        out.append(riemann(left, minus, d, cfg.gamma))
    return out


def _roll_packet(pk, d):
    """The packet of the zone below along axis d."""
    out = {}
    for k, v in pk.items():
        out[k] = {kk: _nb(vv, d, -1) for kk, vv in v.items()} if isinstance(v, dict) else _nb(v, d, -1)
    return out


def _levi(d, a, c):
    return {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1,
            (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}[(d, a, c)]


def step_mhd(U, B, dt, cfg):
    """Ideal MHD step: eq. (6) for the five hydro variables and the
    constrained-transport update of eq. (8) for the face fields.

    Edge electric fields (Sec. II.3, Sec. V): every face's Riemann problem,
    with its own barycentre speeds (HLL) or frozen eigen-system (linearized),
    is applied to the edge averages of eq. (57) on each of its four edges;
    eq. (7) maps the induction flux of the component along the edge's
    transverse axis to the edge field, E_c = -eps_{dac} Flux_d(B_a), and each
    edge field is the mean of its four face values (the reading of "averages
    of appropriate components").
    """
    dx = cfg.spacing(U.shape[1:])
    uhat = predictor(U, dt, cfg, B)
    flows, E = mhd_fluxes(uhat, cfg)
    Un = U.copy()
    for d in range(3):
        Un = Un - dt / dx[d] * (_nb(flows[d], d, 1) - flows[d])
    return Un, B - dt * curl_e(E, dx)


def mhd_fluxes(uhat, cfg):
    """Face fluxes of the five hydro variables at the lower face of every
    zone along each axis, and the edge fields E_c at the lower c-edges, from
    the space-time modes of the eight MHD variables."""
    lin = cfg.riemann == 'linearized'
    flows = []
    E = [np.zeros_like(uhat[0, 0]) for _ in range(3)]
    for d in range(3):
        plus = face_side_packet(uhat, cfg.order, d, +1, cfg.gamma, edges=True)
        minus = face_side_packet(uhat, cfg.order, d, -1, cfg.gamma, edges=True)
        left = _roll_packet(plus, d)
        if lin:
            absA = mhd_abs_jacobian(left['ub'], minus['ub'], d, cfg.gamma)

            def combine(fl, fr, ul, ur):
                return linearized_mhd_combine(fl, fr, ul, ur, absA, d)
        else:
            lam_l, lam_r = hll_speeds(left['ub'], minus['ub'], d, cfg.gamma)

            def combine(fl, fr, ul, ur):
                return hll_combine(fl, fr, ul, ur, lam_l, lam_r)
        flows.append(combine(left['f'], minus['f'], left['u'], minus['u'])[:5])
        tr = transverse_axes(d)
        for which in (0, 1):
            a = tr[which]
            c = 3 - d - a
            sgn = -_levi(d, a, c)
            fe = {}
            for sign in (-1, 1):
                # the whole edge-averaged state enters (the linearized
                # dissipation couples the components); its field row 5 + a
                # is the induction flux
                fe[sign] = combine(left['f_edge'][(which, sign)],
                                   minus['f_edge'][(which, sign)],
                                   left['u_edge'][(which, sign)],
                                   minus['u_edge'][(which, sign)])[5 + a]
            # edge at x_a = lower edge of this zone's face: own face (side -)
            # and the face of the zone below along a (side +)
            E[c] = E[c] + sgn * (fe[-1] + _nb(fe[1], a, -1))
    return flows, [0.25 * e for e in E]


def curl_e(E, dx):
    """Eq. (8) per unit time: the face-field rate is minus this (B_d at the
    lower d-face, E_c at the lower c-edge of the zone)."""
    Ex, Ey, Ez = E
    out = np.empty((3,) + Ex.shape)
    out[0] = (_nb(Ez, 1, 1) - Ez) / dx[1] - (_nb(Ey, 2, 1) - Ey) / dx[2]
    out[1] = (_nb(Ex, 2, 1) - Ex) / dx[2] - (_nb(Ez, 0, 1) - Ez) / dx[0]
    out[2] = (_nb(Ey, 0, 1) - Ey) / dx[0] - (_nb(Ex, 1, 1) - Ex) / dx[1]
    return out


def step(U, dt, cfg, B=None):
    """Eq. (6): U^{n+1} = U^n - sum_d dt/dx_d (F_{i+1/2} - F_{i-1/2}).
    With face fields B (MHD) returns (U^{n+1}, B^{n+1}), see step_mhd."""
    if B is not None:
        if cfg.source is not None:
            raise NotImplementedError('source terms are built for the Euler equations')
        return step_mhd(U, B, dt, cfg)
    dx = cfg.spacing(U.shape[1:])
    if cfg.source is None:
        uhat = predictor(U, dt, cfg)
    else:
        uhat, dts = predictor_source(U, dt, cfg)
    flows = face_fluxes(uhat, cfg)
    Un = U.copy()
    for d in range(3):
        Un = Un - dt / dx[d] * (_nb(flows[d], d, 1) - flows[d])
    if cfg.source is not None:
        Un = Un + dts     # eq. (6): + dt S-bar
    return Un


def predictor_source(U, dt, cfg):
    """The predictor with a source term (Euler): the space-time polynomial
    after the positivity handling, and dt times the space-time average of
    the source (eq. 35, 44, 53; A.7, B.6 in the nodal form), from the
    sources at the nodes of the final polynomial -- in the limit mode the
    scaled one, so the source average and the fluxes see the same
    polynomial."""
    dx = cfg.spacing(U.shape[1:])
    what = safeguard_spatial(reconstruct(U, cfg.order), cfg.order, cfg.form, cfg.gamma,
                             cfg.positivity, cfg.check_mask)
    if cfg.form == 'nodal':
        uhat, dts = predict_nodal_source(what, cfg.order, dt, dx, cfg.gamma, cfg.source)
    else:
        uhat, dts = predict_modal_source(what, cfg.order, dt, dx, cfg.gamma, cfg.source)
    out = safeguard_spacetime(uhat, cfg.order, cfg.form, cfg.gamma, cfg.positivity,
                              cfg.check_mask)
    if cfg.positivity == 'limit':
        dts = source_average(out, cfg.order, cfg.form, dt, cfg.source)
    return out, dts


def step_block(U, dt, cfg, origin, shape, B=None):
    """The updated state of the sub-box ``origin`` (z, y, x) of ``shape`` of a
    periodic mesh, computed from a periodically wrapped block with ghost
    zones, so the oracle can check single zones of a large mesh.  With face
    fields B returns (U, B) of the sub-box."""
    g = cfg.ghost(mhd=B is not None)
    nz, ny, nx = U.shape[1:]
    iz = (np.arange(origin[0] - g, origin[0] + shape[0] + g)) % nz
    iy = (np.arange(origin[1] - g, origin[1] + shape[1] + g)) % ny
    ix = (np.arange(origin[2] - g, origin[2] + shape[2] + g)) % nx
    blk = U[:, iz][:, :, iy][:, :, :, ix]
    # the block keeps the zone size of the full mesh
    sub = OracleConfig(order=cfg.order, form=cfg.form, riemann=cfg.riemann,
                       gamma=cfg.gamma, zone_size=cfg.spacing(U.shape[1:]),
                       source=cfg.source, positivity=cfg.positivity)
    cut = (slice(None), slice(g, g + shape[0]), slice(g, g + shape[1]), slice(g, g + shape[2]))
    with np.errstate(all='ignore'):
        if B is None:
            return step(blk, dt, sub)[cut]
        bblk = B[:, iz][:, :, iy][:, :, :, ix]
        Un, Bn = step(blk, dt, sub, bblk)
    return Un[cut], Bn[cut]
