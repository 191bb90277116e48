"""ADER-CG space-time predictor (Sec. IV modal; Appendices A, B nodal).

Starting from the spatial modes w_1..w_{L_S} of a zone, the evolutionary modes
u_{L_S+1}..u_L of eq. (14)-(16) are found by M-1 Picard iterations (Sec. IV.2):
each iteration evaluates the current space-time polynomial at the predictor
nodes, evaluates the scaled fluxes f = dt F/dx, g = dt G/dy, h = dt H/dz at
those nodes (eq. 5), forms the flux modes the evolution equations need with the
paper's nodal-to-modal rules, and applies the evolution equations.  The initial
guess has all evolutionary modes zero (eq. 10-12 taken as eq. 14-16 at tau=0).

The oracle evaluates the polynomial at every node by direct summation over the
basis (the plain definition of eq. 32, 38-39, 47-48), recomputes every node on
every iteration (the paper reuses the tau=0 ones, which are identical), and
drops the source terms (S = 0 for every system handled here).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from fractions import Fraction as F

import numpy as np

from .basis import N_SPATIAL, N_SPACETIME, P, Q, dP, evaluate, phi, spacetime_modes
from .physics import flux

H = 0.5
T3 = 1.0 / 3.0
T23 = 2.0 / 3.0

# Eq. (31): the seven second-order nodes (xi, eta, zeta, tau).
NODES_MODAL_2 = [(H, 0, 0, 0), (-H, 0, 0, 0), (0, H, 0, 0), (0, -H, 0, 0),
                 (0, 0, H, 0), (0, 0, -H, 0), (0, 0, 0, 1)]

# Eq. (37): the twenty third-order nodes.
NODES_MODAL_3 = [(0, 0, 0, 0),
                 (H, H, 0, 0), (H, -H, 0, 0), (H, 0, H, 0), (H, 0, -H, 0),
                 (-H, H, 0, 0), (-H, -H, 0, 0), (-H, 0, H, 0), (-H, 0, -H, 0),
                 (0, H, H, 0), (0, -H, H, 0), (0, H, -H, 0), (0, -H, -H, 0),
                 (H, 0, 0, H), (-H, 0, 0, H), (0, H, 0, H), (0, -H, 0, H),
                 (0, 0, H, H), (0, 0, -H, H), (0, 0, 0, 1)]

# Eq. (46): the forty-two fourth-order nodes.
Q4 = 0.25
NODES_MODAL_4 = [(0, 0, 0, 0), (H, 0, 0, 0), (Q4, 0, 0, 0), (-Q4, 0, 0, 0), (-H, 0, 0, 0),
                 (0, H, 0, 0), (0, Q4, 0, 0), (0, -Q4, 0, 0), (0, -H, 0, 0),
                 (0, 0, H, 0), (0, 0, Q4, 0), (0, 0, -Q4, 0), (0, 0, -H, 0),
                 (H, H, H, 0), (H, -H, H, 0), (H, H, -H, 0), (H, -H, -H, 0),
                 (-H, H, H, 0), (-H, -H, H, 0), (-H, H, -H, 0), (-H, -H, -H, 0),
                 (0, 0, 0, T3), (H, H, 0, T3), (H, -H, 0, T3), (H, 0, H, T3), (H, 0, -H, T3),
                 (-H, H, 0, T3), (-H, -H, 0, T3), (-H, 0, H, T3), (-H, 0, -H, T3),
                 (0, H, H, T3), (0, -H, H, T3), (0, H, -H, T3), (0, -H, -H, T3),
                 (0, 0, 0, T23), (H, 0, 0, T23), (-H, 0, 0, T23), (0, H, 0, T23),
                 (0, -H, 0, T23), (0, 0, H, T23), (0, 0, -H, T23), (0, 0, 0, 1)]

# Eq. (A.1): the five nodes of the second-order nodal formulation.
NODES_NODAL_2 = [(0, 0, 0, 0), (H, 0, 0, 0), (0, H, 0, 0), (0, 0, H, 0), (0, 0, 0, 1)]

# Eq. (B.1): the fifteen nodes of the third-order nodal formulation.
NODES_NODAL_3 = [(0, 0, 0, 0), (H, 0, 0, 0), (-H, 0, 0, 0), (0, H, 0, 0), (0, -H, 0, 0),
                 (0, 0, H, 0), (0, 0, -H, 0), (0, H, H, 0), (H, 0, H, 0), (H, H, 0, 0),
                 (0, 0, 0, H), (H, 0, 0, H), (0, H, 0, H), (0, 0, H, H), (0, 0, 0, 1)]

# Eq. (C.1): the thirty-five nodes of the fourth-order nodal formulation.
NODES_NODAL_4 = [(0, 0, 0, 0), (H, H, H, 0), (H, 0, 0, 0), (-H, 0, 0, 0), (0, H, 0, 0),
                 (0, -H, 0, 0), (0, 0, H, 0), (0, 0, -H, 0), (0, H, H, 0), (-H, 0, H, 0),
                 (H, 0, H, 0), (H, -H, 0, 0), (H, H, 0, 0), (0, H, -H, 0),
                 (-Q4, -H, -H, 0), (Q4, -H, -H, 0), (-H, -Q4, -H, 0), (-H, Q4, -H, 0),
                 (-H, -H, -Q4, 0), (-H, -H, Q4, 0),
                 (0, 0, 0, T3), (H, 0, 0, T3), (-H, 0, 0, T3), (0, H, 0, T3), (0, -H, 0, T3),
                 (0, 0, H, T3), (0, 0, -H, T3), (0, H, H, T3), (H, 0, H, T3), (H, H, 0, T3),
                 (0, 0, 0, T23), (H, 0, 0, T23), (0, H, 0, T23), (0, 0, H, T23), (0, 0, 0, 1)]

NODES_NODAL = {2: NODES_NODAL_2, 3: NODES_NODAL_3, 4: NODES_NODAL_4}

NODES_MODAL = {2: NODES_MODAL_2, 3: NODES_MODAL_3, 4: NODES_MODAL_4}


def _one_based(values):
    """Index nodal values 1..N as the paper does."""
    return [None] + list(values)


# ---------------------------------------------------------------------------
# Nodal-to-modal flux rules (the modes each evolution equation needs)
# ---------------------------------------------------------------------------

def flux_modes_2(f, g, h):
    """Eq. (33)."""
    return {'f2': f[1] - f[2], 'g3': g[3] - g[4], 'h4': h[5] - h[6]}


def flux_modes_3(f, g, h):
    """Eq. (40) (x-flux), (41) (y-flux), (42) (z-flux)."""
    r = {}
    q1 = f[2] + f[3] + f[4] + f[5]
    q2 = f[6] + f[7] + f[8] + f[9]
    q3 = f[10] + f[11] + f[12] + f[13]
    r['f2'] = 0.25 * (q1 - q2)
    r['f5'] = 0.5 * (q1 + q2 - q3) - 2.0 * f[1]
    r['f8'] = f[2] - f[3] - f[6] + f[7]
    r['f10'] = f[4] - f[5] - f[8] + f[9]
    r['f13'] = 2.0 * (f[14] - f[15] - r['f2'])

    q4 = g[2] + g[6] + g[10] + g[12]
    q5 = g[3] + g[7] + g[11] + g[13]
    q6 = g[4] + g[5] + g[8] + g[9]
    r['g3'] = 0.25 * (q4 - q5)
    r['g6'] = 0.5 * (q4 + q5 - q6) - 2.0 * g[1]
    r['g8'] = g[2] - g[3] - g[6] + g[7]
    r['g9'] = g[10] - g[11] - g[12] + g[13]
    r['g14'] = 2.0 * (g[16] - g[17] - r['g3'])

    q7 = h[4] + h[8] + h[10] + h[11]
    q8 = h[5] + h[9] + h[12] + h[13]
    q9 = h[2] + h[3] + h[6] + h[7]
    r['h4'] = 0.25 * (q7 - q8)
    r['h7'] = 0.5 * (q7 + q8 - q9) - 2.0 * h[1]
    r['h9'] = h[10] - h[11] - h[12] + h[13]
    r['h10'] = h[4] - h[5] - h[8] + h[9]
    r['h15'] = 2.0 * (h[18] - h[19] - r['h4'])
    return r


def _corner_sums(f):
    """The temporaries q1..q9 shared by eq. (49), (50) and (51)."""
    q = {}
    q[1] = f[14] + f[15] + f[16] + f[17]
    q[2] = f[18] + f[19] + f[20] + f[21]
    q[3] = f[14] + f[16] + f[18] + f[20]
    q[4] = f[15] + f[17] + f[19] + f[21]
    q[5] = f[14] + f[15] + f[18] + f[19]
    q[6] = f[16] + f[17] + f[20] + f[21]
    q[7] = f[23] + f[24] - f[25] - f[26] - f[27] - f[28] + f[29] + f[30]
    q[8] = f[23] + f[27] - f[24] - f[28] - f[31] - f[33] + f[32] + f[34]
    q[9] = f[25] + f[29] - f[26] - f[30] - f[31] - f[32] + f[33] + f[34]
    return q


def _mixed_modes(f, q):
    """Modes 14..20 in eq. (49)-(51): the same formulas for f, g and h."""
    r = {}
    r[20] = f[14] - f[15] - f[16] + f[17] - f[18] + f[19] + f[20] - f[21]
    r[14] = q[8] + 0.5 * (q[3] - q[4]) - 2.0 * (f[6] - f[9])
    r[15] = q[9] + 0.5 * (q[5] - q[6]) - 2.0 * (f[10] - f[13])
    r[16] = q[7] + 0.5 * (q[1] - q[2]) - 2.0 * (f[2] - f[5])
    r[17] = -2.0 * q[9] + r[15]
    r[18] = -2.0 * q[7] + r[16]
    r[19] = -2.0 * q[8] + r[14]
    return r


def flux_modes_4(f, g, h):
    """Eq. (49) (x-flux), (50) (y-flux), (51) (z-flux)."""
    r = {}
    # ---- x-flux, eq. (49)
    q = _corner_sums(f)
    q10 = f[23] + f[24] + f[25] + f[26] - f[27] - f[28] - f[29] - f[30]
    r['f5'] = 2.0 * (f[2] - 2.0 * f[1] + f[5])
    r['f8'] = 0.5 * (f[14] - f[15] + f[16] - f[17] - f[18] + f[19] - f[20] + f[21])
    r['f10'] = 0.5 * (f[14] + f[15] - f[16] - f[17] - f[18] - f[19] + f[20] + f[21])
    r['f11'] = 16.0 * (f[2] - 2.0 * f[3] + 2.0 * f[4] - f[5]) / 3.0
    r['f2'] = 2.0 * (f[2] - f[5]) / 3.0 - 0.1 * r['f11'] + (q[1] - q[2]) / 12.0
    mx = _mixed_modes(f, q)
    for k in (14, 15, 16, 18, 20):
        r['f%d' % k] = mx[k]
    r['f27'] = 1.125 * (q[1] - q[2]) + 4.5 * (f[36] - f[37]) - 2.25 * q10
    r['f24'] = (3.0 * (f[36] - f[37]) - 0.75 * q10 + 0.375 * (mx[16] + mx[18])
                - r['f27'])
    r['f30'] = 3.0 * (f[36] - 2.0 * f[35] + f[37]) - 1.5 * r['f5']
    r['f33'] = 3.0 * (f[23] - f[27] - f[24] + f[28]) - 3.0 * r['f8']
    r['f35'] = 3.0 * (f[25] - f[29] - f[26] + f[30]) - 3.0 * r['f10']

    # ---- y-flux, eq. (50)
    q = _corner_sums(g)
    q11 = g[23] - g[24] + g[27] - g[28] + g[31] - g[32] + g[33] - g[34]
    r['g6'] = 2.0 * (g[6] - 2.0 * g[1] + g[9])
    r['g8'] = 0.5 * (g[14] - g[15] + g[16] - g[17] - g[18] + g[19] - g[20] + g[21])
    r['g9'] = 0.5 * (g[14] - g[15] - g[16] + g[17] + g[18] - g[19] - g[20] + g[21])
    r['g12'] = 16.0 * (g[6] - 2.0 * g[7] + 2.0 * g[8] - g[9]) / 3.0
    r['g3'] = 2.0 * (g[6] - g[9]) / 3.0 - 0.1 * r['g12'] + (q[3] - q[4]) / 12.0
    my = _mixed_modes(g, q)
    for k in (14, 16, 17, 19, 20):
        r['g%d' % k] = my[k]
    r['g28'] = 1.125 * (q[3] - q[4]) + 4.5 * (g[38] - g[39]) - 2.25 * q11
    r['g25'] = (3.0 * (g[38] - g[39]) - 0.75 * q11 + 0.375 * (my[14] + my[19])
                - r['g28'])
    r['g31'] = 3.0 * (g[38] - 2.0 * g[35] + g[39]) - 1.5 * r['g6']
    r['g33'] = 3.0 * (g[23] - g[27] - g[24] + g[28]) - 3.0 * r['g8']
    r['g34'] = 3.0 * (g[31] - g[32] - g[33] + g[34]) - 3.0 * r['g9']

    # ---- z-flux, eq. (51)
    q = _corner_sums(h)
    q12 = h[25] - h[26] + h[29] - h[30] + h[31] + h[32] - h[33] - h[34]
    r['h7'] = 2.0 * (h[10] - 2.0 * h[1] + h[13])
    r['h9'] = 0.5 * (h[14] - h[15] - h[16] + h[17] + h[18] - h[19] - h[20] + h[21])
    r['h10'] = 0.5 * (h[14] + h[15] - h[16] - h[17] - h[18] - h[19] + h[20] + h[21])
    r['h13'] = 16.0 * (h[10] - 2.0 * h[11] + 2.0 * h[12] - h[13]) / 3.0
    r['h4'] = 2.0 * (h[10] - h[13]) / 3.0 - 0.1 * r['h13'] + (q[5] - q[6]) / 12.0
    mz = _mixed_modes(h, q)
    for k in (15, 17, 18, 19, 20):
        r['h%d' % k] = mz[k]
    r['h29'] = 1.125 * (q[5] - q[6]) + 4.5 * (h[40] - h[41]) - 2.25 * q12
    r['h26'] = (3.0 * (h[40] - h[41]) - 0.75 * q12 + 0.375 * (mz[15] + mz[17])
                - r['h29'])
    r['h32'] = 3.0 * (h[40] - 2.0 * h[35] + h[41]) - 1.5 * r['h7']
    r['h34'] = 3.0 * (h[31] - h[32] - h[33] + h[34]) - 3.0 * r['h9']
    r['h35'] = 3.0 * (h[25] - h[26] - h[29] + h[30]) - 3.0 * r['h10']
    return r


# ---------------------------------------------------------------------------
# Evolution equations (source terms dropped: S = 0)
# ---------------------------------------------------------------------------

def evolve_2(r):
    """Eq. (30): returns [u_5]."""
    return [-r['f2'] - r['g3'] - r['h4']]


def evolve_3(r):
    """Eq. (36): returns [u_11 .. u_15]."""
    return [
        -r['f2'] - r['g3'] - r['h4'],
        -0.5 * r['f13'] - 0.5 * r['g14'] - 0.5 * r['h15'],
        -2.0 * r['f5'] - r['g8'] - r['h10'],
        -r['f8'] - 2.0 * r['g6'] - r['h9'],
        -r['f10'] - r['g9'] - 2.0 * r['h7'],
    ]


def evolve_4(r):
    """Eq. (45): returns [u_21 .. u_35]."""
    return [
        -r['f11'] / 10.0 - r['f2'] - r['g12'] / 10.0 - r['g3'] - r['h13'] / 10.0 - r['h4'],
        -r['f24'] / 2.0 - r['g25'] / 2.0 - r['h26'] / 2.0,
        -r['f27'] / 3.0 - r['g28'] / 3.0 - r['h29'] / 3.0,
        -2.0 * r['f5'] - r['g8'] - r['h10'],
        -r['f8'] - 2.0 * r['g6'] - r['h9'],
        -r['f10'] - r['g9'] - 2.0 * r['h7'],
        -r['f30'] - r['g33'] / 2.0 - r['h35'] / 2.0,
        -r['f33'] / 2.0 - r['g31'] - r['h34'] / 2.0,
        -r['f35'] / 2.0 - r['g34'] / 2.0 - r['h32'],
        -3.0 * r['f11'] - r['g14'] - r['h15'],
        -r['f16'] - 3.0 * r['g12'] - r['h17'],
        -r['f18'] - r['g19'] - 3.0 * r['h13'],
        -2.0 * r['f14'] - 2.0 * r['g16'] - r['h20'],
        -r['f20'] - 2.0 * r['g17'] - 2.0 * r['h19'],
        -2.0 * r['f15'] - r['g20'] - 2.0 * r['h18'],
    ]


FLUX_MODES = {2: flux_modes_2, 3: flux_modes_3, 4: flux_modes_4}
EVOLVE = {2: evolve_2, 3: evolve_3, 4: evolve_4}


def _scaled_fluxes(ubar, dt, dx, gamma):
    fbar = _one_based([dt / dx[0] * flux(u, 0, gamma) for u in ubar[1:]])
    gbar = _one_based([dt / dx[1] * flux(u, 1, gamma) for u in ubar[1:]])
    hbar = _one_based([dt / dx[2] * flux(u, 2, gamma) for u in ubar[1:]])
    return fbar, gbar, hbar


# ----------------------------------------------------------- source terms --
# The scaled nodal sources are s = dt S(u) at the nodes of eq. (31), (37),
# (46).  Their modes follow the flux rules with f, g, h -> s where the paper
# says so, and eq. (34), (43), (52) for the rest; they enter the evolution
# equations (30), (36), (45), and dt times the space-time average of the
# source, eq. (35), (44), (53), enters the update eq. (6).

def source_modes_2(s):
    """Eq. (34)."""
    m = {1: (s[1] + s[2] + s[3] + s[4] + s[5] + s[6]) / 6.0}
    m[5] = s[7] - m[1]
    return m


def source_modes_3(s):
    """Eq. (40)-(42) with f, g, h -> s, then eq. (43)."""
    r = flux_modes_3(s, s, s)
    m = {2: r['f2'], 3: r['g3'], 4: r['h4'], 5: r['f5'], 6: r['g6'], 7: r['h7'],
         13: r['f13'], 14: r['g14'], 15: r['h15']}
    m[1] = s[1] + (m[5] + m[6] + m[7]) / 12.0
    m[11] = 2.0 * (s[14] + s[15] + s[16] + s[17] + s[18] + s[19] - 6.0 * m[1]) / 3.0 - s[20] + s[1]
    m[12] = s[20] - s[1] - m[11]
    return m


def source_modes_4(s):
    """Eq. (49)-(51) with f, g, h -> s, then eq. (52)."""
    r = flux_modes_4(s, s, s)
    m = {2: r['f2'], 3: r['g3'], 4: r['h4'], 5: r['f5'], 6: r['g6'], 7: r['h7'], 8: r['f8'],
         9: r['g9'], 10: r['f10'], 24: r['f24'], 25: r['g25'], 26: r['h26'], 27: r['f27'],
         28: r['g28'], 29: r['h29'], 30: r['f30'], 31: r['g31'], 32: r['h32'], 33: r['f33'],
         34: r['g34'], 35: r['f35']}
    m[1] = 0.125 * (s[14] + s[15] + s[16] + s[17] + s[18] + s[19] + s[20] + s[21]) \
        - (m[5] + m[6] + m[7]) / 6.0
    m[23] = 4.5 * (s[42] - s[1]) - 13.5 * (s[35] - s[22])
    m[22] = 2.25 * (s[1] - s[22] - s[35] + s[42]) - 1.5 * m[23]
    m[21] = s[42] - s[1] - m[22] - m[23] + (m[30] + m[31] + m[32]) / 12.0
    return m


def evolve_source_2(m):
    """The source terms of eq. (30)."""
    return [m[1] + 2.0 / 3.0 * m[5]]


def evolve_source_3(m):
    """The source terms of eq. (36), for u_11 .. u_15."""
    return [m[1] - 0.3 * m[12], 0.5 * m[11] + 0.6 * m[12], m[2] + 2.0 / 3.0 * m[13],
            m[3] + 2.0 / 3.0 * m[14], m[4] + 2.0 / 3.0 * m[15]]


def evolve_source_4(m):
    """The source terms of eq. (45), for u_21 .. u_35."""
    return [m[1] + 8.0 / 70.0 * m[23], 0.5 * m[21] - 3.0 / 7.0 * m[23],
            m[22] / 3.0 + 4.0 / 7.0 * m[23],
            m[2] - 0.3 * m[27], m[3] - 0.3 * m[28], m[4] - 0.3 * m[29],
            0.5 * m[24] + 0.6 * m[27], 0.5 * m[25] + 0.6 * m[28], 0.5 * m[26] + 0.6 * m[29],
            m[5] + 2.0 / 3.0 * m[30], m[6] + 2.0 / 3.0 * m[31], m[7] + 2.0 / 3.0 * m[32],
            m[8] + 2.0 / 3.0 * m[33], m[9] + 2.0 / 3.0 * m[34], m[10] + 2.0 / 3.0 * m[35]]


def source_integral(m, order):
    """dt times the space-time average of the source: eq. (35), (44), (53)."""
    if order == 2:
        return m[1] + 0.5 * m[5]
    if order == 3:
        return m[1] + 0.5 * m[11] + m[12] / 3.0
    return m[1] + 0.5 * m[21] + m[22] / 3.0 + 0.25 * m[23]


SOURCE_MODES = {2: source_modes_2, 3: source_modes_3, 4: source_modes_4}
EVOLVE_SOURCE = {2: evolve_source_2, 3: evolve_source_3, 4: evolve_source_4}


def predict_modal_source(what, order, dt, dx, gamma, source_fn, flux_fn=None):
    """Modal ADER-CG with a non-stiff source S(u) (Sec. IV with the source
    terms): returns (uhat, dt * S-bar).  Each iteration evaluates the fluxes
    and the scaled sources dt S at the nodes of the current polynomial; dt
    S-bar comes from the source modes of the final polynomial (the sources
    evaluated once more at its nodes, as the flux modes may be rebuilt once
    the evolutionary modes are final), which keeps it of the design order
    (with the modes of the last iterate a single iteration at second order
    would reduce to forward Euler for a pure source)."""
    ls, L = N_SPATIAL[order], N_SPACETIME[order]
    uhat = np.zeros((L,) + what.shape[1:])
    uhat[:ls] = what
    nodes = NODES_MODAL[order]
    for _ in range(order - 1):
        ubar = _one_based([evaluate(uhat, order, x) for x in nodes])
        if flux_fn is None:
            fbar, gbar, hbar = _scaled_fluxes(ubar, dt, dx, gamma)
        else:
            fbar = _one_based([dt / dx[0] * flux_fn(u, 0) for u in ubar[1:]])
            gbar = _one_based([dt / dx[1] * flux_fn(u, 1) for u in ubar[1:]])
            hbar = _one_based([dt / dx[2] * flux_fn(u, 2) for u in ubar[1:]])
        sb = _one_based([dt * source_fn(u) for u in ubar[1:]])
        modes = FLUX_MODES[order](fbar, gbar, hbar)
        sm = SOURCE_MODES[order](sb)
        evo = EVOLVE[order](modes)
        src = EVOLVE_SOURCE[order](sm)
        uhat[ls:] = np.stack([a + b for a, b in zip(evo, src)])
    ubar = _one_based([evaluate(uhat, order, x) for x in nodes])
    sm = SOURCE_MODES[order](_one_based([dt * source_fn(u) for u in ubar[1:]]))
    return uhat, source_integral(sm, order)


def source_average(uhat, order, form, dt, source_fn):
    """dt times the space-time average of the source over a zone whose
    space-time polynomial is ``uhat``: the sources at the nodes of eq. (31),
    (37), (46) and the rule eq. (35), (44), (53) in the modal form; in the
    nodal form the sources at the nodes of (A.1), (B.1), (C.1) and the
    averages (A.7), (B.6) or the integrals of the nodal basis."""
    if form == 'modal':
        ubar = _one_based([evaluate(uhat, order, x) for x in NODES_MODAL[order]])
        sm = SOURCE_MODES[order](_one_based([dt * source_fn(u) for u in ubar[1:]]))
        return source_integral(sm, order)
    s = [dt * source_fn(evaluate(uhat, order, x)) for x in NODES_NODAL[order]]
    if order == 2:
        return 0.5 * (s[0] + s[4])
    if order == 3:
        return nodal3_b6([None] + s)
    _, wbar = nodal_source_map(4)
    return _apply(wbar[None, :], np.stack(s))[0]


def gravity_source(g):
    """S(u) of a uniform gravitational acceleration g = (gx, gy, gz) on the
    Euler variables: (0, rho g, m . g)."""
    g = np.asarray(g, dtype=np.float64)

    def source(u):
        out = np.zeros_like(u)
        out[1:4] = u[0][None] * g.reshape((3,) + (1,) * (u.ndim - 1))
        out[4] = u[1] * g[0] + u[2] * g[1] + u[3] * g[2]
        return out
    return source


def predict_modal(what, order, dt, dx, gamma, flux_fn=None):
    """Modal ADER-CG of Sec. IV.1-IV.3: spatial modes -> all L modes.

    ``what``: (L_S, nv, ...).  ``dx`` = (dx, dy, dz).  ``flux_fn(u, axis)``
    overrides the physical flux (used by the pins with linear fluxes).
    Returns uhat of shape (L, nv, ...).
    """
    ls, L = N_SPATIAL[order], N_SPACETIME[order]
    uhat = np.zeros((L,) + what.shape[1:])
    uhat[:ls] = what
    nodes = NODES_MODAL[order]
    for _ in range(order - 1):
        ubar = _one_based([evaluate(uhat, order, x) for x in nodes])
        if flux_fn is None:
            fbar, gbar, hbar = _scaled_fluxes(ubar, dt, dx, gamma)
        else:
            fbar = _one_based([dt / dx[0] * flux_fn(u, 0) for u in ubar[1:]])
            gbar = _one_based([dt / dx[1] * flux_fn(u, 1) for u in ubar[1:]])
            hbar = _one_based([dt / dx[2] * flux_fn(u, 2) for u in ubar[1:]])
        modes = FLUX_MODES[order](fbar, gbar, hbar)
        uhat[ls:] = np.stack(EVOLVE[order](modes))
    return uhat


def predict_nodal_2(what, dt, dx, gamma, flux_fn=None):
    """Nodal ADER-CG at second order, Appendix A.

    Nodal values at the first four nodes of (A.1) by (A.5); one iteration of
    the evolution equation (A.4) gives the fifth nodal value; (A.6) returns
    the fifth mode.  (A.4) as printed subtracts h_3; the Galerkin derivation
    with the nodal basis (A.2) gives h_4 (the z-node), which is used here.
    """
    ubar = _one_based([
        what[0],
        what[0] + 0.5 * what[1],
        what[0] + 0.5 * what[2],
        what[0] + 0.5 * what[3],
    ])
    if flux_fn is None:
        fn = lambda u, a: flux(u, a, gamma)  # noqa: E731
    else:
        fn = flux_fn
    f1, f2 = dt / dx[0] * fn(ubar[1], 0), dt / dx[0] * fn(ubar[2], 0)
    g1, g3 = dt / dx[1] * fn(ubar[1], 1), dt / dx[1] * fn(ubar[3], 1)
    h1, h4 = dt / dx[2] * fn(ubar[1], 2), dt / dx[2] * fn(ubar[4], 2)
    u5 = ubar[1] - 2.0 * (f2 - f1) - 2.0 * (g3 - g1) - 2.0 * (h4 - h1)
    uhat = np.zeros((5,) + what.shape[1:])
    uhat[:4] = what
    uhat[4] = u5 - ubar[1]
    return uhat


def nodal3_b2_source(s):
    """The source terms of (B.2), from the scaled sources s_1 .. s_7."""
    return {
        11: (-9 * s[1] + 2 * (s[2] + s[3] + s[4] + s[5] + s[6] + s[7])) / 24.0,
        12: (7 * s[1] - 8 * s[2] - 4 * s[3] + 2 * (s[4] + s[5] + s[6] + s[7])) / 24.0,
        13: (7 * s[1] + 2 * (s[2] + s[3]) - 8 * s[4] - 4 * s[5] + 2 * (s[6] + s[7])) / 24.0,
        14: (7 * s[1] + 2 * (s[2] + s[3] + s[4] + s[5]) - 8 * s[6] - 4 * s[7]) / 24.0,
        15: (-27 * s[1] + 5 * (s[2] + s[3] + s[4] + s[5] + s[6] + s[7])) / 30.0,
    }


def nodal3_b3_source(s):
    """The source terms of (B.3) at the later nodes, from s_11 .. s_15."""
    q1 = 0.0
    q2 = (-4 * s[11] - 3 * s[15]) / 24.0
    return {11: 0.125 * (4 * s[11] - s[15]) + q1, 12: q2 + 2 * s[12] / 3.0,
            13: q2 + 2 * s[13] / 3.0, 14: q2 + 2 * s[14] / 3.0,
            15: 4 * q1 + 0.1 * (8 * s[11] + s[15])}


def nodal3_b6(s):
    """(B.6): dt times the space-time average of the source."""
    return (-5 * s[1] + s[2] + s[3] + s[4] + s[5] + s[6] + s[7] + 4 * s[11] + s[15]) / 6.0


def nodal3_b2(u, f, g, h):
    """(B.2) without source terms: the temporaries q_11 .. q_15 from the
    nodal values u_1 .. u_10 at the tau = 0 nodes and their scaled fluxes
    (sequences indexed by the paper's 1-based node numbers)."""
    return {
        11: u[1] + 0.5 * (f[3] - f[1]) + 0.5 * (g[5] - g[1]) + 0.5 * (h[7] - h[1]),
        12: u[2] + (36 * f[1] - 24 * f[2] - 12 * f[3]
                    - 36 * g[1] + 24 * g[2] + 24 * g[4] + 12 * g[5] - 24 * g[10]
                    - 36 * h[1] + 24 * h[2] + 24 * h[6] + 12 * h[7] - 24 * h[9]) / 24.0,
        13: u[4] + (-36 * f[1] + 24 * f[2] + 12 * f[3] + 24 * f[4] - 24 * f[10]
                    + 36 * g[1] - 24 * g[4] - 12 * g[5]
                    - 36 * h[1] + 24 * h[4] + 24 * h[6] + 12 * h[7] - 24 * h[8]) / 24.0,
        14: u[6] + (-36 * f[1] + 24 * f[2] + 12 * f[3] + 24 * f[6] - 24 * f[9]
                    - 36 * g[1] + 24 * g[4] + 12 * g[5] + 24 * g[6] - 24 * g[8]
                    + 36 * h[1] - 24 * h[6] - 12 * h[7]) / 24.0,
        15: u[1] + (-60 * f[1] + 30 * f[2] + 30 * f[3] - 60 * g[1] + 30 * g[4] + 30 * g[5]
                    - 60 * h[1] + 30 * h[6] + 30 * h[7]) / 30.0,
    }


def nodal3_b3(q, f, g, h):
    """(B.3) without source terms: the nodal values at the later nodes 11 ..
    15 from the temporaries q of (B.2) and the scaled fluxes at nodes 11-14
    (indexed by node number)."""
    q1 = 0.5 * (f[11] - f[12]) + 0.5 * (g[11] - g[13]) + 0.5 * (h[11] - h[14])
    q2 = q1
    return {11: q[11] + q1, 12: q[12] + q2, 13: q[13] + q2, 14: q[14] + q2, 15: q[15] + 4.0 * q1}


def predict_nodal_3(what, dt, dx, gamma, flux_fn=None):
    """Nodal ADER-CG at third order, Appendix B (no source terms).

    The nodal values at the ten tau = 0 nodes of (B.1) are the spatial
    polynomial there (what (B.4) evaluates); their scaled fluxes build the
    temporaries of (B.2) once.  The five later nodal values start from the
    spatial polynomial at their positions (no time dependence, as in the
    modal iteration) and take two iterations of (B.3), each with the fluxes
    of the previous iterate; (B.5) returns modes 11-15.
    """
    if flux_fn is None:
        fn = lambda u, a: flux(u, a, gamma)  # noqa: E731
    else:
        fn = flux_fn
    uhat = np.zeros((15,) + what.shape[1:])
    uhat[:10] = what
    u = _one_based([evaluate(uhat, 3, x) for x in NODES_NODAL_3[:10]])
    f = [None] + [dt / dx[0] * fn(u[k], 0) for k in range(1, 11)]
    g = [None] + [dt / dx[1] * fn(u[k], 1) for k in range(1, 11)]
    h = [None] + [dt / dx[2] * fn(u[k], 2) for k in range(1, 11)]
    q = nodal3_b2(u, f, g, h)
    # later nodes 11..15 start from the tau = 0 values at the same positions
    later = {11: u[1], 12: u[2], 13: u[4], 14: u[6], 15: u[1]}
    for _ in range(2):
        fl = {k: dt / dx[0] * fn(later[k], 0) for k in (11, 12)}
        gl = {k: dt / dx[1] * fn(later[k], 1) for k in (11, 13)}
        hl = {k: dt / dx[2] * fn(later[k], 2) for k in (11, 14)}
        later = nodal3_b3(q, fl, gl, hl)
    uhat[10:] = np.stack(nodal3_b5(u, later))
    return uhat


def nodal3_b5(u, later):
    """(B.5): modes 11 (tau), 12 (tau^2), 13 (xi tau), 14 (eta tau) and 15
    (zeta tau) from the nodal values at nodes 1, 2, 4, 6 (u, 1-based) and at
    the later nodes 11-15."""
    m12 = 2.0 * (later[15] - 2.0 * later[11] + u[1])
    m11 = 2.0 * (later[11] - u[1] - 0.25 * m12)
    m13 = 4.0 * (later[12] - later[11] - u[2] + u[1])
    m14 = 4.0 * (later[13] - later[11] - u[4] + u[1])
    m15 = 4.0 * (later[14] - later[11] - u[6] + u[1])
    return [m11, m12, m13, m14, m15]


_EXACT_MAPS = {}


# --- exact rational arithmetic on the basis of eq. (9) and (13) -------------
# A 1D polynomial is a list of Fraction coefficients (constant term first).

_P1D = {0: [F(1)], 1: [F(0), F(1)], 2: [F(-1, 12), F(0), F(1)],
        3: [F(0), F(-3, 20), F(0), F(1)]}       # eq. (9)


def _q1d(d):
    """Eq. (13): tau^d."""
    return [F(0)] * d + [F(1)]


def _val(p, x):
    out = F(0)
    for c in reversed(p):
        out = out * x + c
    return out


def _der(p):
    return [k * c for k, c in enumerate(p)][1:] or [F(0)]


def _mul(p, q):
    out = [F(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _int_space(p):
    """Integral over [-1/2, 1/2]."""
    return sum(c * (F(1, 2) ** (k + 1) - F(-1, 2) ** (k + 1)) / (k + 1) for k, c in enumerate(p))


def _int_time(p):
    """Integral over [0, 1]."""
    return sum(c / (k + 1) for k, c in enumerate(p))


def _inverse(A):
    """Exact inverse of a square matrix of Fractions (Gauss-Jordan)."""
    n = len(A)
    M = [list(row) + [F(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


def _matmul(A, B):
    Bt = list(zip(*B))
    return [[sum((a * b for a, b in zip(row, col) if a and b), F(0)) for col in Bt] for row in A]


def _transpose(A):
    return [list(r) for r in zip(*A)]


def nodal_maps_exact(order):
    """The nodal ADER-CG of App. A (order 2), B (3), C (4) in exact rational
    arithmetic: the solution and the scaled fluxes and sources are
    interpolated on the Lagrange basis psi_j of the nodes (A.1)/(B.1)/(C.1)
    (psi_j = sum_m C[m][j] phi_m, C the inverse of the matrix of basis
    values at the nodes, eq. 9 and 13), and the residual u_tau + f_xi +
    g_eta + h_zeta - s is orthogonal to the psi of the later (tau > 0)
    nodes over the space-time element.  That gives the later nodal values

        u_later = Au u_0 + Af f + Ag g + Ah h + As s

    (u_0 the tau = 0 nodal values, f, g, h, s at every node); the tau = 0
    columns are the temporaries q of (B.2)/(C.2) and the later columns the
    evolutionary equations (B.3)/(C.3).  wbar_j, the integral of psi_j over
    the element, weights dt times the space-time average of the source
    (eq. A.7, B.6, C.6).  Returns a dict of lists of Fractions: nodes, t0,
    lt, C, Au, Af, Ag, Ah, As, wbar."""
    if order in _EXACT_MAPS:
        return _EXACT_MAPS[order]
    nodes = [tuple(F(c).limit_denominator(12) for c in x) for x in NODES_NODAL[order]]
    modes = spacetime_modes(order)
    L = len(modes)
    basis = [([_P1D[a], _P1D[b], _P1D[c]], _q1d(d)) for (a, b, c, d) in modes]
    V = [[_val(sp[0], x[0]) * _val(sp[1], x[1]) * _val(sp[2], x[2]) * _val(tq, x[3])
          for (sp, tq) in basis] for x in nodes]
    C = _inverse(V)                          # mode m = sum_j C[m][j] u_j

    def gram(deriv):
        """G[m][n] = integral of phi_m times the `deriv` derivative of phi_n
        (deriv 0..2 a space axis, 3 time, None none)."""
        G = [[F(0)] * L for _ in range(L)]
        for m, (sm, tm) in enumerate(basis):
            for n, (sn, tn) in enumerate(basis):
                v = F(1)
                for ax in range(3):
                    q = _der(sn[ax]) if deriv == ax else sn[ax]
                    v *= _int_space(_mul(sm[ax], q))
                    if v == 0:
                        break
                if v != 0:
                    v *= _int_time(_mul(tm, _der(tn) if deriv == 3 else tn))
                G[m][n] = v
        return G

    Ct = _transpose(C)
    # in the nodal basis: N[i][j] = integral psi_i (d) psi_j
    nodal = {k: _matmul(_matmul(Ct, gram(k)), C) for k in (0, 1, 2, 3, None)}
    t0 = [i for i, x in enumerate(nodes) if x[3] == 0]
    lt = [i for i, x in enumerate(nodes) if x[3] != 0]
    E = [nodal[3][i] for i in lt]
    Einv = _inverse([[row[j] for j in lt] for row in E])
    neg = [[-v for v in row] for row in Einv]
    Au = _matmul(neg, [[row[j] for j in t0] for row in E])
    Af, Ag, Ah = (_matmul(neg, [nodal[a][i] for i in lt]) for a in range(3))
    As = _matmul(Einv, [nodal[None][i] for i in lt])
    mean = [_int_space(sp[0]) * _int_space(sp[1]) * _int_space(sp[2]) * _int_time(tq)
            for (sp, tq) in basis]
    wbar = [sum((C[m][j] * mean[m] for m in range(L)), F(0)) for j in range(L)]
    out = dict(nodes=nodes, t0=t0, lt=lt, C=C, Au=Au, Af=Af, Ag=Ag, Ah=Ah, As=As, wbar=wbar)
    _EXACT_MAPS[order] = out
    return out


def _floats(A):
    return np.array([[float(v) for v in row] for row in A])


def nodal_update_map(order):
    """The nodal update equations of App. B and C in matrix form, rounded
    once from the exact rational maps of nodal_maps_exact:
        u_later = Au @ u_0 + Af @ f + Ag @ g + Ah @ h.
    Returns the node list, the index arrays of the tau = 0 and later nodes,
    Au, Af, Ag, Ah and the inverse Vandermonde matrix C (mode m = sum_j
    C[m, j] u_j)."""
    ex = nodal_maps_exact(order)
    return (NODES_NODAL[order], np.array(ex['t0']), np.array(ex['lt']), _floats(ex['Au']),
            _floats(ex['Af']), _floats(ex['Ag']), _floats(ex['Ah']), _floats(ex['C']))


def _apply(A, x):
    """sum_j A[i, j] x[j] over the leading axis of x, summed in j order with
    elementwise operations, so that every zone gets the same rounding (a
    library matrix product may order its sums differently per element)."""
    out = np.zeros((A.shape[0],) + x.shape[1:])
    for i in range(A.shape[0]):
        acc = np.zeros(x.shape[1:])
        for j in range(A.shape[1]):
            if A[i, j] != 0.0:
                acc = acc + A[i, j] * x[j]
        out[i] = acc
    return out


def predict_nodal_4(what, dt, dx, gamma, flux_fn=None):
    """Nodal ADER-CG at fourth order, Appendix C (no source terms).

    The nodal values at the twenty tau = 0 nodes of (C.1) are the spatial
    polynomial there; their scaled fluxes build the fifteen temporaries of
    (C.2) once.  The fifteen later nodal values start from the spatial
    polynomial at their positions (as in the modal iteration) and take
    three iterations of (C.3), each with the fluxes of the previous iterate;
    the modes 21-35 follow from the 35 nodal values (the inverse of the
    nodal evaluation).  The coefficients of (C.2)-(C.3) come from
    nodal_update_map (the printed ones are its values).
    """
    if flux_fn is None:
        fn = lambda u, a: flux(u, a, gamma)  # noqa: E731
    else:
        fn = flux_fn
    nodes, t0, lt, Au, Af, Ag, Ah, C = nodal_update_map(4)
    L = len(nodes)
    ls = N_SPATIAL[4]
    uhat = np.zeros((L,) + what.shape[1:])
    uhat[:ls] = what

    def scaled(u_nodes):
        return (np.stack([dt / dx[0] * fn(u, 0) for u in u_nodes]),
                np.stack([dt / dx[1] * fn(u, 1) for u in u_nodes]),
                np.stack([dt / dx[2] * fn(u, 2) for u in u_nodes]))

    u0 = np.stack([evaluate(uhat, 4, nodes[i]) for i in t0])
    f0, g0, h0 = scaled(u0)
    q = _apply(Au, u0) + _apply(Af[:, t0], f0) + _apply(Ag[:, t0], g0) + _apply(Ah[:, t0], h0)
    later = np.stack([evaluate(uhat, 4, tuple(nodes[i][:3]) + (0.0,)) for i in lt])
    for _ in range(3):
        fl, gl, hl = scaled(later)
        later = q + _apply(Af[:, lt], fl) + _apply(Ag[:, lt], gl) + _apply(Ah[:, lt], hl)
    allv = np.empty((L,) + what.shape[1:])
    allv[t0] = u0
    allv[lt] = later
    uhat[ls:] = _apply(C, allv)[ls:]
    return uhat


def nodal_source_map(order):
    """The source part of the nodal update of App. A-C (nodal_maps_exact),
    rounded once: As adds As @ s to the later nodal values (s at every
    node), and dt times the space-time average of the source is wbar @ s
    (eq. A.7, B.6, C.6)."""
    ex = nodal_maps_exact(order)
    return _floats(ex['As']), np.array([float(v) for v in ex['wbar']])


def predict_nodal_source(what, order, dt, dx, gamma, source_fn):
    """The nodal ADER-CG of App. A (order 2), B (3) or C (4) with a source
    S(u): returns (uhat, dt * S-bar).  Orders 2 and 3 take the printed source
    terms of (A.4) and (B.2)-(B.3); order 4 the source part of the Galerkin
    map (nodal_source_map).  dt S-bar is (A.7), (B.6) or wbar @ s with the
    sources of the final nodal values."""
    fn = lambda u, a: flux(u, a, gamma)  # noqa: E731
    nodes = NODES_NODAL[order]
    L = len(nodes)
    ls = N_SPATIAL[order]
    uhat = np.zeros((L,) + what.shape[1:])
    uhat[:ls] = what
    t0 = [i for i, x in enumerate(nodes) if x[3] == 0]
    lt = [i for i, x in enumerate(nodes) if x[3] != 0]
    u = [None] * L
    for i in t0:
        u[i] = evaluate(uhat, order, nodes[i])
    for i in lt:   # start: the spatial polynomial at the later nodes' positions
        u[i] = evaluate(uhat, order, tuple(nodes[i][:3]) + (0.0,))

    def sc(i, a):
        return dt / dx[a] * fn(u[i], a)

    def src(i):
        return dt * source_fn(u[i])

    if order == 2:
        f1, f2 = sc(0, 0), sc(1, 0)
        g1, g3 = sc(0, 1), sc(2, 1)
        h1, h4 = sc(0, 2), sc(3, 2)
        s1, s5 = src(0), src(4)
        u[4] = u[0] - 2.0 * (f2 - f1) - 2.0 * (g3 - g1) - 2.0 * (h4 - h1) + s1 / 3.0 + 2.0 * s5 / 3.0
        uhat[4] = u[4] - u[0]
        return uhat, 0.5 * (src(0) + src(4))
    if order == 3:
        one = lambda vals: [None] + list(vals)  # noqa: E731
        f = one([sc(i, 0) for i in t0])
        g = one([sc(i, 1) for i in t0])
        h = one([sc(i, 2) for i in t0])
        s0 = one([src(i) for i in t0])
        q = nodal3_b2(one([u[i] for i in t0]), f, g, h)
        qs = nodal3_b2_source(s0)
        q = {k: q[k] + qs[k] for k in q}
        for _ in range(2):
            fl = {k: sc(k - 1, 0) for k in (11, 12)}
            gl = {k: sc(k - 1, 1) for k in (11, 13)}
            hl = {k: sc(k - 1, 2) for k in (11, 14)}
            sl = {k: src(k - 1) for k in (11, 12, 13, 14, 15)}
            later = nodal3_b3(q, fl, gl, hl)
            ls_ = nodal3_b3_source(sl)
            for k in later:
                u[k - 1] = later[k] + ls_[k]
        uhat[10:] = np.stack(nodal3_b5(one([u[i] for i in t0]), {k: u[k - 1] for k in range(11, 16)}))
        s_all = one([src(i) for i in range(L)])
        return uhat, nodal3_b6(s_all)
    # order 4: the Galerkin map with its source part
    _, _, _, Au, Af, Ag, Ah, C = nodal_update_map(4)
    As, wbar = nodal_source_map(4)
    u0 = np.stack([u[i] for i in t0])
    fs = [np.stack([sc(i, a) for i in t0]) for a in range(3)]
    s0 = np.stack([src(i) for i in t0])
    q = (_apply(Au, u0) + _apply(Af[:, t0], fs[0]) + _apply(Ag[:, t0], fs[1])
         + _apply(Ah[:, t0], fs[2]) + _apply(As[:, t0], s0))
    for _ in range(3):
        fl = [np.stack([sc(i, a) for i in lt]) for a in range(3)]
        sl = np.stack([src(i) for i in lt])
        later = (q + _apply(Af[:, lt], fl[0]) + _apply(Ag[:, lt], fl[1]) + _apply(Ah[:, lt], fl[2])
                 + _apply(As[:, lt], sl))
        for r, i in enumerate(lt):
            u[i] = later[r]
    allv = np.stack(u)
    uhat[ls:] = _apply(C, allv)[ls:]
    s_all = np.stack([src(i) for i in range(L)])
    return uhat, _apply(wbar[None, :], s_all)[0]
