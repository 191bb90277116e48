"""SSP Runge-Kutta time stepping (Sec. II.d, eq. 18-20) with the spatial
operator of the ADER step.

The space-time predictor of Sec. II.2 is bypassed: each stage reconstructs
the stage state (Sec. II.1, with the positivity handling of
``cfg.positivity`` on the spatial polynomial), takes the face-side packets of Sec. V / App. D from the spatial
polynomial held constant over the stage (so the App. D face averages become
face averages at the stage time), solves the Riemann problems (Sec. II.3)
and forms L(U) = -sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d, the right-hand side
of eq. (4) written as dU/dt = L(U).  The stage combinations are those of
eq. (18) (SSP-RK2), (19) (SSP-RK3) and (20) (the optimal five-stage,
fourth-order scheme), matched to the spatial order 2, 3, 4 as in Sec. VII.
For ideal MHD the face fields advance with the same weights, their rate
being minus the curl of the stage's edge fields (eq. 8 per unit time), and
the zone field of Sec. III is rebuilt from the stage's face fields.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .basis import N_SPACETIME, N_SPATIAL
from .positivity import safeguard_spatial
from .bweno import zone_b_modes
from .step import _nb, curl_e, face_fluxes, mhd_fluxes
from .weno import reconstruct

SCHEME_OF_ORDER = {2: 'ssprk2', 3: 'ssprk3', 4: 'ssprk54'}


def spatial_operator(U, cfg):
    """L(U) for the five Euler variables on the periodic mesh."""
    dx = cfg.spacing(U.shape[1:])
    what = reconstruct(U, cfg.order)
    what = safeguard_spatial(what, cfg.order, 'modal', cfg.gamma, cfg.positivity)
    uhat = np.zeros((N_SPACETIME[cfg.order],) + what.shape[1:])
    uhat[:N_SPATIAL[cfg.order]] = what
    flows = face_fluxes(uhat, cfg)
    out = np.zeros_like(U)
    for d in range(3):
        out = out - (_nb(flows[d], d, 1) - flows[d]) / dx[d]
    return out


def mhd_operator(state, cfg):
    """(L_U, L_B) for ideal MHD: the hydro flux divergence and minus the curl
    of the edge fields, from the face-side packets of the spatial polynomial
    of the eight variables (hydro from U, field from B by Sec. III)."""
    U, B = state
    dx = cfg.spacing(U.shape[1:])
    what = np.concatenate([reconstruct(U, cfg.order), zone_b_modes(B, cfg.order)], axis=1)
    what = safeguard_spatial(what, cfg.order, 'modal', cfg.gamma, cfg.positivity)
    uhat = np.zeros((N_SPACETIME[cfg.order],) + what.shape[1:])
    uhat[:N_SPATIAL[cfg.order]] = what
    flows, E = mhd_fluxes(uhat, cfg)
    LU = np.zeros_like(U)
    for d in range(3):
        LU = LU - (_nb(flows[d], d, 1) - flows[d]) / dx[d]
    return _Pair(LU, -curl_e(E, dx))


class _Pair:
    """(U, B) with the linear operations the stage combinations use."""

    def __init__(self, a, b):
        self.a, self.b = a, b

    def __add__(self, o):
        return _Pair(self.a + o.a, self.b + o.b)

    def __mul__(self, s):
        return _Pair(self.a * s, self.b * s)

    __rmul__ = __mul__

    def __truediv__(self, s):
        return _Pair(self.a / s, self.b / s)

    def __iter__(self):
        return iter((self.a, self.b))


def ssp_step(U, dt, L, scheme):
    """One step of eq. (18), (19) or (20) for dU/dt = L(U)."""
    if scheme == 'ssprk2':
        U1 = U + dt * L(U)
        return 0.5 * U + 0.5 * U1 + 0.5 * dt * L(U1)
    if scheme == 'ssprk3':
        U1 = U + dt * L(U)
        U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * L(U1)
        return U / 3.0 + 2.0 / 3.0 * U2 + 2.0 / 3.0 * dt * L(U2)
    if scheme == 'ssprk54':
        U1 = U + 0.39175222700392 * dt * L(U)
        U2 = 0.44437049406734 * U + 0.55562950593266 * U1 + 0.36841059262959 * dt * L(U1)
        L2 = L(U2)
        U3 = 0.62010185138540 * U + 0.37989814861460 * U2 + 0.25189177424738 * dt * L2
        L3 = L(U3)
        U4 = 0.17807995410773 * U + 0.82192004589227 * U3 + 0.54497475021237 * dt * L3
        L4 = L(U4)
        return (0.00683325884039 * U + 0.51723167208978 * U2 + 0.12759831133288 * U3
                + 0.34833675773694 * U4 + 0.08460416338212 * dt * L3
                + 0.22600748319395 * dt * L4)
    raise ValueError(scheme)


def step_rk(U, dt, cfg):
    """One SSP-RK step of the order-matched scheme (Euler)."""
    return ssp_step(U, dt, lambda V: spatial_operator(V, cfg), SCHEME_OF_ORDER[cfg.order])


def step_rk_mhd(U, B, dt, cfg):
    """One SSP-RK step of ideal MHD: returns (U, B)."""
    out = ssp_step(_Pair(U, B), dt, lambda S: mhd_operator(S, cfg), SCHEME_OF_ORDER[cfg.order])
    return out.a, out.b
