"""Face-side space-time quantities (Sec. V and Appendix D).

For every zone and each of its six face sides (normal axis d, side s = +1 for
the top face "x+", -1 for the bottom face "x-") the oracle builds

* u_b: the space-time barycentre state u(s/2, 0, 0, 1/2), eq. (54);
* <u>: the face space-time average of u, eq. (55), by exact integration of
  the modal polynomial (each P_a with a >= 1 integrates to zero, Q_d to
  1/(d+1));
* <F>: the face space-time average of the physical normal flux: the state is
  evaluated at the facial nodes (D.1)/(D.6)/(D.11), the normal flux is taken
  there, the face flux modes follow from (D.4)/(D.9)/(D.14), and the average
  is the exact integral of the face flux polynomial (D.2)/(D.7)/(D.12);
* edge averages of u and F along the four edges of the face, eq. (57), used
  by the MHD electric fields.

Transverse coordinates: for the x-face (t1, t2) = (eta, zeta), for the y-face
(xi, zeta), for the z-face (xi, eta).  The facial node sets and rules are
symmetric under t1 <-> t2, so this choice does not change any face average.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .basis import P, Q, spacetime_modes, evaluate
from .physics import flux

H = 0.5
T3 = 1.0 / 3.0
T23 = 2.0 / 3.0
Q4 = 0.25

# Facial nodes as (t1, t2, tau).
FACE_NODES = {
    2: [(H, 0, H), (-H, 0, H), (0, H, H), (0, -H, H), (0, 0, 1)],           # (D.1)
    3: [(0, 0, 0), (H, H, 0), (-H, H, 0), (H, -H, 0), (-H, -H, 0),         # (D.6)
        (H, 0, H), (-H, 0, H), (0, H, H), (0, -H, H), (0, 0, 1)],
    4: [(0, 0, 0), (H, 0, 0), (Q4, 0, 0), (-Q4, 0, 0), (-H, 0, 0),         # (D.11)
        (0, H, 0), (0, Q4, 0), (0, -Q4, 0), (0, -H, 0),
        (H, H, 0), (-H, H, 0), (H, -H, 0), (-H, -H, 0),
        (0, 0, T3), (H, H, T3), (-H, H, T3), (H, -H, T3), (-H, -H, T3),
        (0, 0, T23), (H, 0, T23), (-H, 0, T23), (0, H, T23), (0, -H, T23),
        (0, 0, 1)],
}

# Face flux modes as exponents (a1, a2, d) of P_a1(t1) P_a2(t2) Q_d(tau).
FACE_MODES = {
    2: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],                         # (D.2)
    3: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 0), (0, 2, 0), (1, 1, 0),    # (D.7)
        (0, 0, 1), (0, 0, 2), (1, 0, 1), (0, 1, 1)],
    4: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 0), (0, 2, 0), (1, 1, 0),    # (D.12)
        (3, 0, 0), (0, 3, 0), (2, 1, 0), (1, 2, 0),
        (0, 0, 1), (0, 0, 2), (0, 0, 3),
        (1, 0, 1), (0, 1, 1), (1, 0, 2), (0, 1, 2),
        (2, 0, 1), (0, 2, 1), (1, 1, 1)],
}


def face_rule_2(f):
    """Eq. (D.4); ``f`` is 1-based over the nodes of (D.1)."""
    m = [None] * 5
    m[2] = f[1] - f[2]
    m[3] = f[3] - f[4]
    m[4] = 2.0 * f[5] - 0.5 * (f[1] + f[2] + f[3] + f[4])
    m[1] = f[5] - m[4]
    return m


def face_rule_3(f):
    """Eq. (D.9); ``f`` is 1-based over the nodes of (D.6)."""
    m = [None] * 11
    q2 = 0.5 * (f[2] + f[4] - 4.0 * f[1] + f[3] + f[5])
    q3 = f[6] + f[7] - f[8] - f[9]
    m[1] = 2.0 * (f[1] + 0.125 * (f[2] + f[3] + f[4] + f[5])) / 3.0
    m[2] = 0.5 * (f[2] + f[4] - f[3] - f[5])
    m[3] = 0.5 * (f[2] + f[3] - f[4] - f[5])
    m[4] = q2 + q3
    m[5] = q2 - q3
    m[6] = f[2] - f[3] - f[4] + f[5]
    m[8] = 2.0 * (f[1] + f[10]) - (f[6] + f[7] + f[8] + f[9]) + q2
    m[7] = f[10] - f[1] - m[8]
    m[9] = 2.0 * (f[6] - f[7] - m[2])
    m[10] = 2.0 * (f[8] - f[9] - m[3])
    return m


def face_rule_4(f):
    """Eq. (D.14); ``f`` is 1-based over the nodes of (D.11)."""
    m = [None] * 21
    q1 = 3.0 * (f[20] - f[21]) - 1.5 * (f[15] - f[16] + f[17] - f[18])
    q2 = 1.5 * (f[20] - f[21] - f[2] + f[5])
    q3 = 3.0 * (f[22] - f[23]) - 1.5 * (f[15] + f[16] - f[17] - f[18])
    q4 = 1.5 * (f[22] - f[23] - f[6] + f[9])
    m[1] = (2.0 * f[1] + f[2] + f[5] + f[6] + f[9]) / 6.0
    m[4] = 2.0 * (f[2] - 2.0 * f[1] + f[5])
    m[5] = 2.0 * (f[6] - 2.0 * f[1] + f[9])
    m[6] = f[10] - f[11] - f[12] + f[13]
    m[7] = 16.0 * (f[2] - 2.0 * f[3] + 2.0 * f[4] - f[5]) / 3.0
    m[8] = 16.0 * (f[6] - 2.0 * f[7] + 2.0 * f[8] - f[9]) / 3.0
    m[9] = 2.0 * (f[10] - 2.0 * f[6] + f[11] - f[12] + 2.0 * f[9] - f[13])
    m[10] = 2.0 * (f[10] - 2.0 * f[2] + f[12] - f[11] + 2.0 * f[5] - f[13])
    m[2] = f[2] - f[5] + m[10] / 12.0 - 0.1 * m[7]
    m[3] = f[6] - f[9] + m[9] / 12.0 - 0.1 * m[8]
    m[13] = 4.5 * (f[24] - f[1]) - 13.5 * (f[19] - f[14])
    m[12] = 2.25 * (f[24] - f[19] - f[14] + f[1] - 2.0 * m[13] / 3.0)
    m[11] = (1.5 * f[24] - 2.5 * f[14] + 0.25 * (f[15] + f[16] + f[17] + f[18])
             - 0.25 * m[4] - 0.25 * m[5] - 4.0 * m[12] / 3.0 - 13.0 * m[13] / 9.0)
    m[14] = 3.0 * q2 - 2.0 * q1 - 1.5 * m[10]
    m[16] = 3.0 * (q1 - q2) + 2.25 * m[10]
    m[15] = 3.0 * q4 - 2.0 * q3 - 1.5 * m[9]
    m[17] = 3.0 * (q3 - q4) + 2.25 * m[9]
    m[18] = 3.0 * (f[20] - 2.0 * f[19] + f[21]) - 1.5 * m[4]
    m[19] = 3.0 * (f[22] - 2.0 * f[19] + f[23]) - 1.5 * m[5]
    m[20] = 3.0 * (f[15] - f[16] - f[17] + f[18]) - 3.0 * m[6]
    return m


FACE_RULE = {2: face_rule_2, 3: face_rule_3, 4: face_rule_4}


def transverse_axes(d):
    return {0: (1, 2), 1: (0, 2), 2: (0, 1)}[d]


def zone_point(d, s, t1, t2, tau):
    """Reference-element point on side s of the face with normal axis d."""
    p = [0.0, 0.0, 0.0]
    p[d] = 0.5 * s
    a1, a2 = transverse_axes(d)
    p[a1] = t1
    p[a2] = t2
    return (p[0], p[1], p[2], tau)


def face_average_of_modes(modes, order):
    """Exact space-time face average of the face polynomial (D.2/7/12)."""
    out = 0.0
    for k, (a1, a2, d) in enumerate(FACE_MODES[order]):
        if a1 == 0 and a2 == 0:
            out = out + modes[k + 1] / (d + 1.0)
    return out


def edge_average_of_modes(modes, order, which, sign):
    """Exact average along the edge t_which = sign/2 of the face polynomial
    over the other transverse coordinate and tau (eq. 57)."""
    out = 0.0
    for k, (a1, a2, d) in enumerate(FACE_MODES[order]):
        a_on, a_off = (a1, a2) if which == 0 else (a2, a1)
        if a_off == 0:
            out = out + modes[k + 1] * float(P(a_on, 0.5 * sign)) / (d + 1.0)
    return out


def barycentre_state(uhat, order, d, s):
    """Eq. (54)."""
    return evaluate(uhat, order, zone_point(d, s, 0.0, 0.0, 0.5))


def face_average_u(uhat, order, d, s):
    """Eq. (55) by exact integration of the modal polynomial."""
    out = np.zeros(uhat.shape[1:])
    for m, (a, b, c, dd) in enumerate(spacetime_modes(order)):
        e = (a, b, c)
        if all(e[ax] == 0 for ax in transverse_axes(d)):
            out = out + uhat[m] * float(P(e[d], 0.5 * s)) / (dd + 1.0)
    return out


def edge_average_u(uhat, order, d, s, e_axis, e_sign):
    """Eq. (57): average over the remaining axis and tau of u on the edge
    {x_d = s/2, x_{e_axis} = e_sign/2}."""
    out = np.zeros(uhat.shape[1:])
    free = [ax for ax in range(3) if ax not in (d, e_axis)][0]
    for m, (a, b, c, dd) in enumerate(spacetime_modes(order)):
        e = (a, b, c)
        if e[free] == 0:
            w = float(P(e[d], 0.5 * s)) * float(P(e[e_axis], 0.5 * e_sign)) / (dd + 1.0)
            out = out + uhat[m] * w
    return out


def facial_flux_modes(uhat, order, d, s, gamma, flux_fn=None):
    """Face flux modes of the physical normal flux from the facial nodes."""
    fvals = [None]
    for (t1, t2, tau) in FACE_NODES[order]:
        u = evaluate(uhat, order, zone_point(d, s, t1, t2, tau))
        fvals.append(flux(u, d, gamma) if flux_fn is None else flux_fn(u, d))
    return FACE_RULE[order](fvals)


def face_side_packet(uhat, order, d, s, gamma, flux_fn=None, edges=False):
    """All face-side quantities of one side of every zone.

    Returns a dict with 'ub', 'u', 'f' (each (nv, ...)) and, when ``edges``
    is set, 'u_edge' / 'f_edge' keyed by (transverse index 0/1, sign +-1).
    """
    modes = facial_flux_modes(uhat, order, d, s, gamma, flux_fn)
    out = {
        'ub': barycentre_state(uhat, order, d, s),
        'u': face_average_u(uhat, order, d, s),
        'f': face_average_of_modes(modes, order),
    }
    if edges:
        tr = transverse_axes(d)
        out['u_edge'] = {}
        out['f_edge'] = {}
        for which in (0, 1):
            for sign in (-1, 1):
                out['u_edge'][(which, sign)] = edge_average_u(uhat, order, d, s, tr[which], sign)
                out['f_edge'][(which, sign)] = edge_average_of_modes(modes, order, which, sign)
    return out
