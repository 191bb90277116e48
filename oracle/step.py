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

from .faces import face_side_packet
from .physics import primitives, fast_speed
from .positivity import limit_spatial, limit_spacetime
from .predictor import predict_modal, predict_nodal_2
from .riemann import hll, linearized_euler
from .weno import reconstruct


@dataclass
class OracleConfig:
    order: int = 3                 # 2, 3 or 4
    form: str = 'modal'            # 'modal' (Sec. IV) or 'nodal' (App. A, order 2)
    riemann: str = 'hll'           # 'hll' or 'linearized'
    gamma: float = 1.4
    lengths: tuple = (1.0, 1.0, 1.0)   # domain (lx, ly, lz)
    zone_size: tuple = None            # (dx, dy, dz); overrides ``lengths``

    def spacing(self, shape):
        if self.zone_size is not None:
            return tuple(self.zone_size)
        nz, ny, nx = shape
        return (self.lengths[0] / nx, self.lengths[1] / ny, self.lengths[2] / nz)

    def ghost(self):
        """Zones of neighbourhood one zone's update depends on, per side."""
        return {2: 2, 3: 3, 4: 4}[self.order]


def _nb(arr, axis, o):
    return np.roll(arr, -o, axis=arr.ndim - 1 - axis)


def compute_dt(U, cfg, cfl, B=None):
    """dt = cfl / max_zones sum_d (|v_d| + c_d) / dx_d."""
    dx = cfg.spacing(U.shape[1:])
    rho, v, P, _ = primitives(U, cfg.gamma)
    rate = np.zeros_like(rho)
    for d in range(3):
        rate = rate + (np.abs(v[d]) + fast_speed(U, d, cfg.gamma)) / dx[d]
    return cfl / rate.max()


def predictor(U, dt, cfg):
    """Spatial reconstruction followed by the space-time predictor, each
    followed by the positivity safeguard."""
    dx = cfg.spacing(U.shape[1:])
    what = limit_spatial(reconstruct(U, cfg.order), cfg.order, cfg.form, cfg.gamma)
    if cfg.form == 'nodal':
        if cfg.order != 2:
            raise NotImplementedError('nodal formulation is built at order 2 only')
        uhat = predict_nodal_2(what, dt, dx, cfg.gamma)
    else:
        uhat = predict_modal(what, cfg.order, dt, dx, cfg.gamma)
    return limit_spacetime(uhat, cfg.order, cfg.form, cfg.gamma)


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


def step(U, dt, cfg, B=None):
    """Eq. (6): U^{n+1} = U^n - sum_d dt/dx_d (F_{i+1/2} - F_{i-1/2})."""
    if B is not None:
        raise NotImplementedError('MHD step is not part of this oracle module')
    dx = cfg.spacing(U.shape[1:])
    uhat = predictor(U, dt, cfg)
    flows = face_fluxes(uhat, cfg)
    Un = U.copy()
    for d in range(3):
        Un = Un - dt / dx[d] * (_nb(flows[d], d, 1) - flows[d])
    return Un


def step_block(U, dt, cfg, origin, shape, B=None):
    """The updated state of the sub-box ``origin`` (z, y, x) of ``shape`` of a
    periodic mesh, computed from a periodically wrapped block with ghost
    zones, so the oracle can check single zones of a large mesh."""
    g = cfg.ghost()
    nz, ny, nx = U.shape[1:]
    iz = (np.arange(origin[0] - g, origin[0] + shape[0] + g)) % nz
    iy = (np.arange(origin[1] - g, origin[1] + shape[1] + g)) % ny
    ix = (np.arange(origin[2] - g, origin[2] + shape[2] + g)) % nx
    blk = U[:, iz][:, :, iy][:, :, :, ix]
    # the block keeps the zone size of the full mesh
    sub = OracleConfig(order=cfg.order, form=cfg.form, riemann=cfg.riemann,
                       gamma=cfg.gamma, zone_size=cfg.spacing(U.shape[1:]))
    with np.errstate(all='ignore'):
        out = step(blk, dt, sub)
    return out[:, g:g + shape[0], g:g + shape[1], g:g + shape[2]]
