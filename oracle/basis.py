"""Basis functions and mode orderings of the ADER-CG scheme.

Sec. II.1 eq. (9): spatial Hermite polynomials P0..P3 on [-1/2, 1/2].
Sec. II.2 eq. (13): temporal monomials Q0..Q3 on [0, 1].
Eq. (10)-(12): order of the L_S spatial modes; eq. (14)-(16): order of the L
space-time modes (the first L_S are the spatial modes with Q0 = 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np


def P(a, x):
    """Eq. (9): P0 = 1, P1 = x, P2 = x^2 - 1/12, P3 = x^3 - 3x/20."""
    x = np.asarray(x, dtype=np.float64)
    if a == 0:
        return np.ones_like(x)
    if a == 1:
        return x
    if a == 2:
        return x * x - 1.0 / 12.0
    if a == 3:
        return x * x * x - 3.0 * x / 20.0
    raise ValueError(a)


def dP(a, x):
    """Derivative of P_a."""
    x = np.asarray(x, dtype=np.float64)
    if a == 0:
        return np.zeros_like(x)
    if a == 1:
        return np.ones_like(x)
    if a == 2:
        return 2.0 * x
    if a == 3:
        return 3.0 * x * x - 3.0 / 20.0
    raise ValueError(a)


def Q(d, t):
    """Eq. (13): Q_d(tau) = tau^d."""
    t = np.asarray(t, dtype=np.float64)
    return t ** d


# Eq. (10)-(12): spatial modes as exponent triples (a, b, c) of
# P_a(xi) P_b(eta) P_c(zeta), in the paper's numbering w_1 .. w_20.
SPATIAL_MODES = [
    (0, 0, 0),
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2),
    (1, 1, 0), (0, 1, 1), (1, 0, 1),
    (3, 0, 0), (0, 3, 0), (0, 0, 3),
    (2, 1, 0), (2, 0, 1),
    (1, 2, 0), (0, 2, 1),
    (1, 0, 2), (0, 1, 2),
    (1, 1, 1),
]

# Eq. (14)-(16): the evolutionary space-time modes u_{L_S+1} .. u_L as
# (a, b, c, d) = P_a(xi) P_b(eta) P_c(zeta) Q_d(tau).
EVOLUTIONARY_MODES = {
    2: [(0, 0, 0, 1)],
    3: [(0, 0, 0, 1), (0, 0, 0, 2),
        (1, 0, 0, 1), (0, 1, 0, 1), (0, 0, 1, 1)],
    4: [(0, 0, 0, 1), (0, 0, 0, 2), (0, 0, 0, 3),
        (1, 0, 0, 1), (0, 1, 0, 1), (0, 0, 1, 1),
        (1, 0, 0, 2), (0, 1, 0, 2), (0, 0, 1, 2),
        (2, 0, 0, 1), (0, 2, 0, 1), (0, 0, 2, 1),
        (1, 1, 0, 1), (0, 1, 1, 1), (1, 0, 1, 1)],
}

N_SPATIAL = {2: 4, 3: 10, 4: 20}      # L_S, Sec. II.1
N_SPACETIME = {2: 5, 3: 15, 4: 35}    # L, Sec. II.2


def spacetime_modes(order):
    """All L space-time modes of eq. (14)/(15)/(16) as (a, b, c, d)."""
    ls = N_SPATIAL[order]
    return [m + (0,) for m in SPATIAL_MODES[:ls]] + EVOLUTIONARY_MODES[order]


def phi(mode, xi, eta, zeta, tau):
    """Value of one space-time basis function at a point."""
    a, b, c, d = mode
    return P(a, xi) * P(b, eta) * P(c, zeta) * Q(d, tau)


def evaluate(uhat, order, point):
    """u(xi, eta, zeta, tau) = sum_m uhat_m phi_m(point), eq. (14)-(16).

    ``uhat`` has shape (L, ...) with the paper's mode order on axis 0; the
    result has shape ``uhat.shape[1:]``.  Direct evaluation: the plain
    definition of the modal-to-nodal transcription of eq. (32), (38)-(39) and
    (47)-(48).
    """
    xi, eta, zeta, tau = point
    out = np.zeros(uhat.shape[1:])
    for m, mode in enumerate(spacetime_modes(order)):
        out = out + float(phi(mode, xi, eta, zeta, tau)) * uhat[m]
    return out
