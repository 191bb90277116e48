"""Linear advection u_t + a . grad u = 0 of five independent components,
stepped by the same ADER-CG scheme (Sec. II): reconstruction (Sec. II.1),
the space-time predictor (Sec. IV, App. A-C) with the linear flux
F_d(u) = a_d u, the face-side averages (Sec. V, App. D), the HLL flux of
eq. (56) with the exact signal speeds min(a_d, 0) and max(a_d, 0) -- which
is the upwind face flux -- and the update of eq. (6).  It is the system on
which the scheme's exact-translation property holds: at |a_x| dt = dx with
a along x every zone average moves by exactly one zone, for any data.  No
positivity handling applies (the components are not densities).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .faces import face_side_packet
from .predictor import predict_modal, predict_nodal_2, predict_nodal_3, predict_nodal_4
from .weno import reconstruct


def _nb(arr, axis, o):
    return np.roll(arr, -o, axis=arr.ndim - 1 - axis)


def advection_flux(a):
    """F_d(u) = a_d u, for every component."""
    def fn(u, axis):
        return a[axis] * u
    return fn


def compute_dt(U, cfg, cfl, a):
    """dt = cfl / sum_d |a_d| / dx_d (the CFL rule of the Euler path with
    the signal speeds |a_d|)."""
    dx = cfg.spacing(U.shape[1:])
    return cfl / sum(abs(a[d]) / dx[d] for d in range(3))


def upwind(fl, fr, a_d):
    """Eq. (56) with lambda_L = min(a_d, 0), lambda_R = max(a_d, 0): the
    left side's flux for a_d > 0, the right side's for a_d < 0, and zero
    (the flux a_d u itself) for a_d = 0."""
    if a_d > 0:
        return fl
    if a_d < 0:
        return fr
    return np.zeros_like(fl)


def step(U, dt, cfg, a):
    """One ADER-CG step of linear advection with velocity a = (ax, ay, az)."""
    dx = cfg.spacing(U.shape[1:])
    fn = advection_flux(a)
    what = reconstruct(U, cfg.order)
    if cfg.form == 'nodal':
        pred = {2: predict_nodal_2, 3: predict_nodal_3, 4: predict_nodal_4}[cfg.order]
        uhat = pred(what, dt, dx, None, flux_fn=fn)
    else:
        uhat = predict_modal(what, cfg.order, dt, dx, None, flux_fn=fn)
    Un = U.copy()
    for d in range(3):
        plus = face_side_packet(uhat, cfg.order, d, +1, None, flux_fn=fn)
        minus = face_side_packet(uhat, cfg.order, d, -1, None, flux_fn=fn)
        F = upwind(_nb(plus['f'], d, -1), minus['f'], a[d])   # at the lower face
        Un = Un - dt / dx[d] * (_nb(F, d, 1) - F)
    return Un
