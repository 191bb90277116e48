"""Conserved variables and fluxes of eq. (3) (Gaussian units).

U = (rho, rho vx, rho vy, rho vz, eps[, Bx, By, Bz]) with
eps = rho v^2/2 + P/(gamma-1) + B^2/(8 pi).  The Euler system is eq. (3) with
B = 0 and only the first five components.  ``axis`` 0/1/2 selects F/G/H.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

FOUR_PI = 4.0 * np.pi
EIGHT_PI = 8.0 * np.pi


def primitives(u, gamma):
    """(rho, v[3], P, B[3] or None) from conserved u of shape (nv, ...)."""
    rho = u[0]
    v = u[1:4] / rho
    if u.shape[0] == 8:
        B = u[5:8]
        b2 = (B * B).sum(axis=0)
    else:
        B = None
        b2 = 0.0
    P = (gamma - 1.0) * (u[4] - 0.5 * rho * (v * v).sum(axis=0) - b2 / EIGHT_PI)
    return rho, v, P, B


def conserved(rho, v, P, B, gamma):
    """Inverse of ``primitives``."""
    nv = 5 if B is None else 8
    u = np.zeros((nv,) + np.shape(rho))
    u[0] = rho
    u[1:4] = rho * v
    b2 = 0.0 if B is None else (B * B).sum(axis=0)
    u[4] = 0.5 * rho * (v * v).sum(axis=0) + P / (gamma - 1.0) + b2 / EIGHT_PI
    if B is not None:
        u[5:8] = B
    return u


def flux(u, axis, gamma):
    """Physical flux F (axis 0), G (axis 1) or H (axis 2) of eq. (3)."""
    rho, v, P, B = primitives(u, gamma)
    vn = v[axis]
    f = np.zeros_like(u)
    f[0] = rho * vn
    if B is None:
        f[1:4] = u[1:4] * vn
        f[1 + axis] += P
        f[4] = (u[4] + P) * vn
        return f
    Bn = B[axis]
    b2 = (B * B).sum(axis=0)
    vB = (v * B).sum(axis=0)
    ptot = P + b2 / EIGHT_PI
    f[1:4] = u[1:4] * vn - B * Bn / FOUR_PI
    f[1 + axis] += ptot
    f[4] = (u[4] + ptot) * vn - Bn * vB / FOUR_PI
    # induction part: d/dx_axis of (v_axis B - B_axis v); zero on the normal
    f[5:8] = vn * B - Bn * v
    f[5 + axis] = 0.0
    return f


def fast_speed(u, axis, gamma):
    """Sound speed (Euler) or fast magnetosonic speed (MHD) along ``axis``."""
    rho, v, P, B = primitives(u, gamma)
    a2 = gamma * P / rho
    if B is None:
        return np.sqrt(a2)
    b2 = (B * B).sum(axis=0) / (FOUR_PI * rho)
    bn2 = B[axis] ** 2 / (FOUR_PI * rho)
    s = a2 + b2
    return np.sqrt(0.5 * (s + np.sqrt(np.maximum(s * s - 4.0 * a2 * bn2, 0.0))))
