#!/usr/bin/env python3
"""Generate ``generated/ader_scheme.h``: straight-line device code for the
per-zone pieces of the ADER-CG step at orders 2-4.

Run once after editing this file (``python gen_scheme.py``); the output is
committed and compiled by ``build.py``.  Everything is derived here in exact
rational arithmetic (``fractions.Fraction``) from the paper's definitions:

* basis: Hermite P0..P3 (eq. 9) and tau^d (eq. 13), mode orders eq. (10)-(16);
* predictor nodes: eq. (31), (37), (46) (modal) and (A.1), (B.1) (nodal);
* nodal-to-modal flux rules (33), (40)-(42), (49)-(51) composed with the
  evolution equations (30), (36), (45): every evolutionary mode becomes a
  weighted sum of the scaled nodal fluxes f = dt F/dx, g, h; the nodal
  second-order update (A.4) (z-term read as h4 - h1) and (A.6) likewise, and
  the third-order (B.2), (B.3), (B.5) composed (their nodal values cancel,
  leaving each evolutionary mode a weighted sum of nodal fluxes);
* facial nodes (D.1)/(D.6)/(D.11) with the rules (D.4)/(D.9)/(D.14) composed
  with the face integrals (D.5)/(D.10)/(D.15): the face average of the
  normal flux is a weighted sum of facial nodal fluxes (nodes of zero weight
  are dropped);
* barycentre states (eq. 54) and face averages of u (eq. 55) as weighted sums
  of modes;
* centred WENO candidate matrices and smoothness forms.

A mode value at a point is the sum over modes with nonzero basis value only,
so the emitted code carries no multiplications by zero.
"""

import os
from fractions import Fraction as Fr

HALF = Fr(1, 2)
QTR = Fr(1, 4)
THIRD = Fr(1, 3)

# ---------------------------------------------------------------- basis ----


def P(a, x):
    x = Fr(x)
    return [Fr(1), x, x * x - Fr(1, 12), x ** 3 - Fr(3, 20) * x][a]


def mode_list(order):
    """Space-time modes (a, b, c, d) in the order of eq. (14)-(16)."""
    words = {
        2: "1 x y z t",
        3: "1 x y z xx yy zz xy yz xz t tt xt yt zt",
        4: ("1 x y z xx yy zz xy yz xz xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz "
            "t tt ttt xt yt zt xtt ytt ztt xxt yyt zzt xyt yzt xzt"),
    }[order]
    out = []
    for w in words.split():
        if w == "1":
            out.append((0, 0, 0, 0))
        else:
            out.append((w.count('x'), w.count('y'), w.count('z'), w.count('t')))
    return out


LS = {2: 4, 3: 10, 4: 20}


def phi(mode, pt):
    a, b, c, d = mode
    return P(a, pt[0]) * P(b, pt[1]) * P(c, pt[2]) * Fr(pt[3]) ** d


def point_row(order, pt):
    return [phi(m, pt) for m in mode_list(order)]


# ------------------------------------------------------- predictor nodes ----

def pred_nodes(order, form):
    h, q, t1, t2 = HALF, QTR, THIRD, 2 * THIRD
    if form == 'nodal' and order == 2:
        return [(0, 0, 0, 0), (h, 0, 0, 0), (0, h, 0, 0), (0, 0, h, 0), (0, 0, 0, 1)]
    if form == 'nodal' and order == 3:
        return [(0, 0, 0, 0), (h, 0, 0, 0), (-h, 0, 0, 0), (0, h, 0, 0), (0, -h, 0, 0),
                (0, 0, h, 0), (0, 0, -h, 0), (0, h, h, 0), (h, 0, h, 0), (h, h, 0, 0),
                (0, 0, 0, h), (h, 0, 0, h), (0, h, 0, h), (0, 0, h, h), (0, 0, 0, 1)]
    if form == 'nodal':   # (C.1)
        return [(0, 0, 0, 0), (h, h, h, 0), (h, 0, 0, 0), (-h, 0, 0, 0), (0, h, 0, 0),
                (0, -h, 0, 0), (0, 0, h, 0), (0, 0, -h, 0), (0, h, h, 0), (-h, 0, h, 0),
                (h, 0, h, 0), (h, -h, 0, 0), (h, h, 0, 0), (0, h, -h, 0),
                (-q, -h, -h, 0), (q, -h, -h, 0), (-h, -q, -h, 0), (-h, q, -h, 0),
                (-h, -h, -q, 0), (-h, -h, q, 0),
                (0, 0, 0, t1), (h, 0, 0, t1), (-h, 0, 0, t1), (0, h, 0, t1), (0, -h, 0, t1),
                (0, 0, h, t1), (0, 0, -h, t1), (0, h, h, t1), (h, 0, h, t1), (h, h, 0, t1),
                (0, 0, 0, t2), (h, 0, 0, t2), (0, h, 0, t2), (0, 0, h, t2), (0, 0, 0, 1)]
    if order == 2:
        return [(h, 0, 0, 0), (-h, 0, 0, 0), (0, h, 0, 0), (0, -h, 0, 0),
                (0, 0, h, 0), (0, 0, -h, 0), (0, 0, 0, 1)]
    if order == 3:
        return [(0, 0, 0, 0),
                (h, h, 0, 0), (h, -h, 0, 0), (h, 0, h, 0), (h, 0, -h, 0),
                (-h, h, 0, 0), (-h, -h, 0, 0), (-h, 0, h, 0), (-h, 0, -h, 0),
                (0, h, h, 0), (0, -h, h, 0), (0, h, -h, 0), (0, -h, -h, 0),
                (h, 0, 0, h), (-h, 0, 0, h), (0, h, 0, h), (0, -h, 0, h),
                (0, 0, h, h), (0, 0, -h, h), (0, 0, 0, 1)]
    return [(0, 0, 0, 0), (h, 0, 0, 0), (q, 0, 0, 0), (-q, 0, 0, 0), (-h, 0, 0, 0),
            (0, h, 0, 0), (0, q, 0, 0), (0, -q, 0, 0), (0, -h, 0, 0),
            (0, 0, h, 0), (0, 0, q, 0), (0, 0, -q, 0), (0, 0, -h, 0),
            (h, h, h, 0), (h, -h, h, 0), (h, h, -h, 0), (h, -h, -h, 0),
            (-h, h, h, 0), (-h, -h, h, 0), (-h, h, -h, 0), (-h, -h, -h, 0),
            (0, 0, 0, t1), (h, h, 0, t1), (h, -h, 0, t1), (h, 0, h, t1), (h, 0, -h, t1),
            (-h, h, 0, t1), (-h, -h, 0, t1), (-h, 0, h, t1), (-h, 0, -h, t1),
            (0, h, h, t1), (0, -h, h, t1), (0, h, -h, t1), (0, -h, -h, t1),
            (0, 0, 0, t2), (h, 0, 0, t2), (-h, 0, 0, t2), (0, h, 0, t2),
            (0, -h, 0, t2), (0, 0, h, t2), (0, 0, -h, t2), (0, 0, 0, 1)]


# --------------------------------------------- symbolic linear combinations --

class Lin(dict):
    """A linear combination of named unknowns with rational coefficients."""

    def __add__(self, o):
        r = Lin(self)
        for k, v in o.items():
            r[k] = r.get(k, 0) + v
        return Lin({k: v for k, v in r.items() if v != 0})

    def __neg__(self):
        return Lin({k: -v for k, v in self.items()})

    def __sub__(self, o):
        return self + (-o)

    def __mul__(self, c):
        return Lin({k: v * Fr(c) for k, v in self.items() if v * Fr(c) != 0})

    __rmul__ = __mul__

    def __truediv__(self, c):
        return self * (Fr(1) / Fr(c))


def unknowns(prefix, n):
    return [None] + [Lin({(prefix, j): Fr(1)}) for j in range(1, n + 1)]


def S(*xs):
    out = Lin()
    for x in xs:
        out = out + x
    return out


def rules_o2(f, g, h):
    # eq. (33) and the evolution equation (30)
    return [-(f[1] - f[2]) - (g[3] - g[4]) - (h[5] - h[6])]


def modes_o3(f, g, h):
    """Eq. (40), (41), (42): the modes of the x-, y- and z-fluxes from their
    nodal values, as dicts {mode: combination} (1-based mode numbers)."""
    q1, q2, q3 = S(f[2], f[3], f[4], f[5]), S(f[6], f[7], f[8], f[9]), S(f[10], f[11], f[12], f[13])
    F = {2: (q1 - q2) * QTR}
    F[5] = (q1 + q2 - q3) * HALF - f[1] * 2
    F[8] = f[2] - f[3] - f[6] + f[7]
    F[10] = f[4] - f[5] - f[8] + f[9]
    F[13] = (f[14] - f[15] - F[2]) * 2
    q4, q5, q6 = S(g[2], g[6], g[10], g[12]), S(g[3], g[7], g[11], g[13]), S(g[4], g[5], g[8], g[9])
    G = {3: (q4 - q5) * QTR}
    G[6] = (q4 + q5 - q6) * HALF - g[1] * 2
    G[8] = g[2] - g[3] - g[6] + g[7]
    G[9] = g[10] - g[11] - g[12] + g[13]
    G[14] = (g[16] - g[17] - G[3]) * 2
    q7, q8, q9 = S(h[4], h[8], h[10], h[11]), S(h[5], h[9], h[12], h[13]), S(h[2], h[3], h[6], h[7])
    H = {4: (q7 - q8) * QTR}
    H[7] = (q7 + q8 - q9) * HALF - h[1] * 2
    H[9] = h[10] - h[11] - h[12] + h[13]
    H[10] = h[4] - h[5] - h[8] + h[9]
    H[15] = (h[18] - h[19] - H[4]) * 2
    return F, G, H


def rules_o3(f, g, h):
    # eq. (40)-(42), then the flux part of (36)
    F, G, H = modes_o3(f, g, h)
    return [
        -F[2] - G[3] - H[4],
        -(F[13] + G[14] + H[15]) * HALF,
        -F[5] * 2 - G[8] - H[10],
        -F[8] - G[6] * 2 - H[9],
        -F[10] - G[9] - H[7] * 2,
    ]


def _o4_common(f):
    q = [None] * 10
    q[1] = S(f[14], f[15], f[16], f[17])
    q[2] = S(f[18], f[19], f[20], f[21])
    q[3] = S(f[14], f[16], f[18], f[20])
    q[4] = S(f[15], f[17], f[19], f[21])
    q[5] = S(f[14], f[15], f[18], f[19])
    q[6] = S(f[16], f[17], f[20], f[21])
    q[7] = f[23] + f[24] - f[25] - f[26] - f[27] - f[28] + f[29] + f[30]
    q[8] = f[23] + f[27] - f[24] - f[28] - f[31] - f[33] + f[32] + f[34]
    q[9] = f[25] + f[29] - f[26] - f[30] - f[31] - f[32] + f[33] + f[34]
    m = {}
    m[20] = f[14] - f[15] - f[16] + f[17] - f[18] + f[19] + f[20] - f[21]
    m[14] = q[8] + (q[3] - q[4]) * HALF - (f[6] - f[9]) * 2
    m[15] = q[9] + (q[5] - q[6]) * HALF - (f[10] - f[13]) * 2
    m[16] = q[7] + (q[1] - q[2]) * HALF - (f[2] - f[5]) * 2
    m[17] = m[15] - q[9] * 2
    m[18] = m[16] - q[7] * 2
    m[19] = m[14] - q[8] * 2
    return q, m


def modes_o4(f, g, h):
    """Eq. (49), (50), (51): the modes of the x-, y- and z-fluxes from their
    nodal values, as dicts {mode: combination} (1-based mode numbers)."""
    q, F = _o4_common(f)
    q10 = f[23] + f[24] + f[25] + f[26] - f[27] - f[28] - f[29] - f[30]
    F[5] = (f[2] - f[1] * 2 + f[5]) * 2
    F[8] = (f[14] - f[15] + f[16] - f[17] - f[18] + f[19] - f[20] + f[21]) * HALF
    F[10] = (f[14] + f[15] - f[16] - f[17] - f[18] - f[19] + f[20] + f[21]) * HALF
    F[11] = (f[2] - f[3] * 2 + f[4] * 2 - f[5]) * Fr(16, 3)
    F[2] = (f[2] - f[5]) * Fr(2, 3) - F[11] * Fr(1, 10) + (q[1] - q[2]) / 12
    F[27] = (q[1] - q[2]) * Fr(9, 8) + (f[36] - f[37]) * Fr(9, 2) - q10 * Fr(9, 4)
    F[24] = (f[36] - f[37]) * 3 - q10 * Fr(3, 4) + (F[16] + F[18]) * Fr(3, 8) - F[27]
    F[30] = (f[36] - f[35] * 2 + f[37]) * 3 - F[5] * Fr(3, 2)
    F[33] = (f[23] - f[27] - f[24] + f[28]) * 3 - F[8] * 3
    F[35] = (f[25] - f[29] - f[26] + f[30]) * 3 - F[10] * 3

    q, G = _o4_common(g)
    q11 = g[23] - g[24] + g[27] - g[28] + g[31] - g[32] + g[33] - g[34]
    G[6] = (g[6] - g[1] * 2 + g[9]) * 2
    G[8] = (g[14] - g[15] + g[16] - g[17] - g[18] + g[19] - g[20] + g[21]) * HALF
    G[9] = (g[14] - g[15] - g[16] + g[17] + g[18] - g[19] - g[20] + g[21]) * HALF
    G[12] = (g[6] - g[7] * 2 + g[8] * 2 - g[9]) * Fr(16, 3)
    G[3] = (g[6] - g[9]) * Fr(2, 3) - G[12] * Fr(1, 10) + (q[3] - q[4]) / 12
    G[28] = (q[3] - q[4]) * Fr(9, 8) + (g[38] - g[39]) * Fr(9, 2) - q11 * Fr(9, 4)
    G[25] = (g[38] - g[39]) * 3 - q11 * Fr(3, 4) + (G[14] + G[19]) * Fr(3, 8) - G[28]
    G[31] = (g[38] - g[35] * 2 + g[39]) * 3 - G[6] * Fr(3, 2)
    G[33] = (g[23] - g[27] - g[24] + g[28]) * 3 - G[8] * 3
    G[34] = (g[31] - g[32] - g[33] + g[34]) * 3 - G[9] * 3

    q, H = _o4_common(h)
    q12 = h[25] - h[26] + h[29] - h[30] + h[31] + h[32] - h[33] - h[34]
    H[7] = (h[10] - h[1] * 2 + h[13]) * 2
    H[9] = (h[14] - h[15] - h[16] + h[17] + h[18] - h[19] - h[20] + h[21]) * HALF
    H[10] = (h[14] + h[15] - h[16] - h[17] - h[18] - h[19] + h[20] + h[21]) * HALF
    H[13] = (h[10] - h[11] * 2 + h[12] * 2 - h[13]) * Fr(16, 3)
    H[4] = (h[10] - h[13]) * Fr(2, 3) - H[13] * Fr(1, 10) + (q[5] - q[6]) / 12
    H[29] = (q[5] - q[6]) * Fr(9, 8) + (h[40] - h[41]) * Fr(9, 2) - q12 * Fr(9, 4)
    H[26] = (h[40] - h[41]) * 3 - q12 * Fr(3, 4) + (H[15] + H[17]) * Fr(3, 8) - H[29]
    H[32] = (h[40] - h[35] * 2 + h[41]) * 3 - H[7] * Fr(3, 2)
    H[34] = (h[31] - h[32] - h[33] + h[34]) * 3 - H[9] * 3
    H[35] = (h[25] - h[26] - h[29] + h[30]) * 3 - H[10] * 3
    return F, G, H


def rules_o4(f, g, h):
    # eq. (49)-(51), then the flux part of (45)
    F, G, H = modes_o4(f, g, h)
    t = Fr(1, 10)
    return [
        -F[11] * t - F[2] - G[12] * t - G[3] - H[13] * t - H[4],
        -(F[24] + G[25] + H[26]) * HALF,
        -(F[27] + G[28] + H[29]) * THIRD,
        -F[5] * 2 - G[8] - H[10],
        -F[8] - G[6] * 2 - H[9],
        -F[10] - G[9] - H[7] * 2,
        -F[30] - G[33] * HALF - H[35] * HALF,
        -F[33] * HALF - G[31] - H[34] * HALF,
        -F[35] * HALF - G[34] * HALF - H[32],
        -F[11] * 3 - G[14] - H[15],
        -F[16] - G[12] * 3 - H[17],
        -F[18] - G[19] - H[13] * 3,
        -F[14] * 2 - G[16] * 2 - H[20],
        -F[20] - G[17] * 2 - H[19] * 2,
        -F[15] * 2 - G[20] - H[18] * 2,
    ]


def rules_nodal2(f, g, h):
    # (A.4) with the z-difference taken at node 4, then (A.6): u5 = ubar5 - ubar1
    return [-(f[2] - f[1]) * 2 - (g[3] - g[1]) * 2 - (h[4] - h[1]) * 2]


def rules_nodal3(f, g, h):
    # (B.2): temporaries from the tau = 0 nodes; (B.3) at one iterate; (B.5)
    # to the modes tau, tau^2, xi tau, eta tau, zeta tau.  The nodal values u
    # enter only as differences that (B.5) cancels.
    u = unknowns('u', 15)
    F = Fr(1, 24)
    q11 = u[1] + (f[3] - f[1]) * HALF + (g[5] - g[1]) * HALF + (h[7] - h[1]) * HALF
    q12 = u[2] + (f[1] * 36 - f[2] * 24 - f[3] * 12
                  - g[1] * 36 + g[2] * 24 + g[4] * 24 + g[5] * 12 - g[10] * 24
                  - h[1] * 36 + h[2] * 24 + h[6] * 24 + h[7] * 12 - h[9] * 24) * F
    q13 = u[4] + (-f[1] * 36 + f[2] * 24 + f[3] * 12 + f[4] * 24 - f[10] * 24
                  + g[1] * 36 - g[4] * 24 - g[5] * 12
                  - h[1] * 36 + h[4] * 24 + h[6] * 24 + h[7] * 12 - h[8] * 24) * F
    q14 = u[6] + (-f[1] * 36 + f[2] * 24 + f[3] * 12 + f[6] * 24 - f[9] * 24
                  - g[1] * 36 + g[4] * 24 + g[5] * 12 + g[6] * 24 - g[8] * 24
                  + h[1] * 36 - h[6] * 24 - h[7] * 12) * F
    q15 = u[1] + (-f[1] * 60 + f[2] * 30 + f[3] * 30 - g[1] * 60 + g[4] * 30 + g[5] * 30
                  - h[1] * 60 + h[6] * 30 + h[7] * 30) * Fr(1, 30)
    q1 = (f[11] - f[12]) * HALF + (g[11] - g[13]) * HALF + (h[11] - h[14]) * HALF
    n11, n12, n13, n14, n15 = q11 + q1, q12 + q1, q13 + q1, q14 + q1, q15 + q1 * 4
    m12 = (n15 - n11 * 2 + u[1]) * 2
    m11 = (n11 - u[1] - m12 * QTR) * 2
    m13 = (n12 - n11 - u[2] + u[1]) * 4
    m14 = (n13 - n11 - u[4] + u[1]) * 4
    m15 = (n14 - n11 - u[6] + u[1]) * 4
    out = [m11, m12, m13, m14, m15]
    for m in out:
        assert all(k[0] != 'u' for k in m), m
    return out


# exact polynomial algebra for the fourth-order nodal derivation: a
# polynomial is {(a, b, c, d): coefficient} for xi^a eta^b zeta^c tau^d
P_POW = [{0: Fr(1)}, {1: Fr(1)}, {2: Fr(1), 0: Fr(-1, 12)}, {3: Fr(1), 1: Fr(-3, 20)}]


def _mode_poly(m):
    a, b, c, d = m
    out = {}
    for pa, ca in P_POW[a].items():
        for pb, cb in P_POW[b].items():
            for pc, cc in P_POW[c].items():
                k = (pa, pb, pc, d)
                out[k] = out.get(k, 0) + ca * cb * cc
    return out


def _poly_add(p, q, s=Fr(1)):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, 0) + s * v
    return {k: v for k, v in r.items() if v != 0}


def _poly_mul(p, q):
    out = {}
    for k1, v1 in p.items():
        for k2, v2 in q.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            out[k] = out.get(k, 0) + v1 * v2
    return out


def _poly_diff(p, axis):
    out = {}
    for k, v in p.items():
        if k[axis]:
            kk = list(k)
            kk[axis] -= 1
            out[tuple(kk)] = out.get(tuple(kk), 0) + v * k[axis]
    return out


def _integral(p):
    """Over xi, eta, zeta in [-1/2, 1/2] and tau in [0, 1]."""
    s = Fr(0)
    for (a, b, c, d), v in p.items():
        if a % 2 or b % 2 or c % 2:
            continue
        s += v * Fr(1, 2 ** a * (a + 1)) * Fr(1, 2 ** b * (b + 1)) * Fr(1, 2 ** c * (c + 1)) / (d + 1)
    return s


def _inverse(A):
    n = len(A)
    M = [list(row) + [Fr(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def rules_nodal4(f, g, h):
    # App. C: the nodal update of (C.2)-(C.3) is the continuous-Galerkin
    # system written with the nodal basis of (C.1): u and the fluxes
    # interpolated on it, the residual u_tau + f_xi + g_eta + h_zeta
    # orthogonal to the basis functions of the 15 later nodes.  Solved for the
    # later nodal values and mapped back to modes 21-35, the tau = 0 nodal
    # values cancel and each evolutionary mode is a weighted sum of fluxes.
    nodes = pred_nodes(4, 'nodal')
    modes = mode_list(4)
    n = len(nodes)
    mp = [_mode_poly(m) for m in modes]
    V = [[sum(v * Fr(x[0]) ** k[0] * Fr(x[1]) ** k[1] * Fr(x[2]) ** k[2] * Fr(x[3]) ** k[3]
              for k, v in mp[m].items()) for m in range(n)] for x in nodes]
    Ci = _inverse(V)                      # mode m = sum_j Ci[m][j] u_j
    basis = []
    for j in range(n):
        p = {}
        for m in range(n):
            if Ci[m][j] != 0:
                p = _poly_add(p, mp[m], Ci[m][j])
        basis.append(p)
    t0 = [j for j in range(n) if nodes[j][3] == 0]
    lt = [j for j in range(n) if nodes[j][3] != 0]
    dB = [[_poly_diff(basis[j], ax) for ax in range(4)] for j in range(n)]
    E = [[_integral(_poly_mul(basis[i], dB[j][3])) for j in range(n)] for i in lt]
    D = [[[_integral(_poly_mul(basis[i], dB[j][ax])) for j in range(n)] for i in lt]
         for ax in range(3)]
    Ei = _inverse([[E[r][j] for j in lt] for r in range(len(lt))])
    u = unknowns('u', n)
    flx = (f, g, h)
    later = []
    for r in range(len(lt)):
        v = Lin()
        for s in range(len(lt)):
            c = Ei[r][s]
            if c == 0:
                continue
            for j in t0:
                if E[s][j] != 0:
                    v = v - u[j + 1] * (c * E[s][j])
            for ax in range(3):
                for j in range(n):
                    if D[ax][s][j] != 0:
                        v = v - flx[ax][j + 1] * (c * D[ax][s][j])
        later.append(v)
    value = {j: u[j + 1] for j in t0}
    value.update({j: later[r] for r, j in enumerate(lt)})
    out = []
    for m in range(LS[4], n):
        v = Lin()
        for j in range(n):
            if Ci[m][j] != 0:
                v = v + value[j] * Ci[m][j]
        assert all(k[0] != 'u' for k in v), m
        out.append(v)
    return out


# ------------------------------------------------------------ source terms --
# A non-stiff source S(u) enters the evolutionary modes through the scaled
# nodal sources s = dt S(u) at the predictor nodes.  Modal form: the source
# modes are the flux-mode rules with f, g, h -> s, each mode taken from the
# first of the x-, y-, z-rules that defines it, and eq. (34), (43), (52) for
# the rest; they enter through the source terms of eq. (30), (36), (45).
# Nodal forms: the source is interpolated on the nodal basis like the fluxes
# and enters the Galerkin system of App. A-C (residual u_tau + f_xi + g_eta +
# h_zeta - s orthogonal to the later nodes' basis functions).

def _source_modes_from_rules(F, G, H):
    sm = {}
    for D in (F, G, H):
        for m, v in D.items():
            sm.setdefault(m, v)
    return sm


def source_rules_modal(order):
    """Evolutionary mode k's source part as a combination of the scaled
    nodal sources s_j (unknowns ('s', j))."""
    n = len(pred_nodes(order, 'modal'))
    s = unknowns('s', n)
    if order == 2:
        s1 = S(s[1], s[2], s[3], s[4], s[5], s[6]) / 6                       # eq. (34)
        s5 = s[7] - s1
        return [s1 + s5 * Fr(2, 3)]                                            # eq. (30)
    if order == 3:
        sm = _source_modes_from_rules(*modes_o3(s, s, s))
        sm[1] = s[1] + (sm[5] + sm[6] + sm[7]) / 12                           # eq. (43)
        sm[11] = (S(s[14], s[15], s[16], s[17], s[18], s[19]) - sm[1] * 6) * Fr(2, 3) \
            - s[20] + s[1]
        sm[12] = s[20] - s[1] - sm[11]
        return [sm[1] - sm[12] * Fr(3, 10), sm[11] * HALF + sm[12] * Fr(3, 5),   # eq. (36)
                sm[2] + sm[13] * Fr(2, 3), sm[3] + sm[14] * Fr(2, 3), sm[4] + sm[15] * Fr(2, 3)]
    sm = _source_modes_from_rules(*modes_o4(s, s, s))
    sm[1] = S(*[s[j] for j in range(14, 22)]) * Fr(1, 8) - (sm[5] + sm[6] + sm[7]) / 6   # (52)
    sm[23] = (s[42] - s[1]) * Fr(9, 2) - (s[35] - s[22]) * Fr(27, 2)
    sm[22] = (s[1] - s[22] - s[35] + s[42]) * Fr(9, 4) - sm[23] * Fr(3, 2)
    sm[21] = s[42] - s[1] - sm[22] - sm[23] + (sm[30] + sm[31] + sm[32]) / 12
    two3, three5, three10 = Fr(2, 3), Fr(3, 5), Fr(3, 10)
    return [sm[1] + sm[23] * Fr(8, 70), sm[21] * HALF - sm[23] * Fr(3, 7),      # eq. (45)
            sm[22] * THIRD + sm[23] * Fr(4, 7),
            sm[2] - sm[27] * three10, sm[3] - sm[28] * three10, sm[4] - sm[29] * three10,
            sm[24] * HALF + sm[27] * three5, sm[25] * HALF + sm[28] * three5,
            sm[26] * HALF + sm[29] * three5,
            sm[5] + sm[30] * two3, sm[6] + sm[31] * two3, sm[7] + sm[32] * two3,
            sm[8] + sm[33] * two3, sm[9] + sm[34] * two3, sm[10] + sm[35] * two3]


def source_rules_nodal(order):
    """The source part of the nodal ADER-CG (App. A, B, C) by the Galerkin
    system over the nodes (A.1)/(B.1)/(C.1), mapped back to the evolutionary
    modes."""
    nodes = pred_nodes(order, 'nodal')
    modes = mode_list(order)
    n = len(nodes)
    mp = [_mode_poly(m) for m in modes]
    V = [[sum(v * Fr(x[0]) ** k[0] * Fr(x[1]) ** k[1] * Fr(x[2]) ** k[2] * Fr(x[3]) ** k[3]
              for k, v in mp[m].items()) for m in range(n)] for x in nodes]
    Ci = _inverse(V)
    basis = []
    for j in range(n):
        p = {}
        for m in range(n):
            if Ci[m][j] != 0:
                p = _poly_add(p, mp[m], Ci[m][j])
        basis.append(p)
    lt = [j for j in range(n) if nodes[j][3] != 0]
    E = [[_integral(_poly_mul(basis[i], _poly_diff(basis[j], 3))) for j in range(n)] for i in lt]
    Mm = [[_integral(_poly_mul(basis[i], basis[j])) for j in range(n)] for i in lt]
    Ei = _inverse([[E[r][j] for j in lt] for r in range(len(lt))])
    s = unknowns('s', n)
    later = {}
    for r, j0 in enumerate(lt):
        v = Lin()
        for q in range(len(lt)):
            c = Ei[r][q]
            if c == 0:
                continue
            for j in range(n):
                if Mm[q][j] != 0:
                    v = v + s[j + 1] * (c * Mm[q][j])
        later[j0] = v
    out = []
    for m in range(LS[order], n):
        v = Lin()
        for j0, lv in later.items():
            if Ci[m][j0] != 0:
                v = v + lv * Ci[m][j0]
        out.append(v)
    return out


def source_weights(order, form):
    return source_rules_nodal(order) if form == 'nodal' else source_rules_modal(order)


def mean_weights(order):
    """Space-time mean of u over the element from its modes (only the pure
    time modes have a nonzero mean: tau^d has 1/(d+1))."""
    out = {}
    for m, (a, b, c, d) in enumerate(mode_list(order)):
        if a == 0 and b == 0 and c == 0 and m > 0:
            out[m] = Fr(1, d + 1)
    return out


def evolution_weights(order, form):
    """W[k] = {(dir, node): weight}: evolutionary mode k as a combination of
    the scaled nodal fluxes (dir 'f', 'g', 'h'; nodes 1-based)."""
    n = len(pred_nodes(order, form))
    f, g, h = unknowns('f', n), unknowns('g', n), unknowns('h', n)
    if form == 'nodal':
        return {2: rules_nodal2, 3: rules_nodal3, 4: rules_nodal4}[order](f, g, h)
    return {2: rules_o2, 3: rules_o3, 4: rules_o4}[order](f, g, h)


# ------------------------------------------------------------ facial nodes --

def face_nodes(order):
    h, q, t1, t2 = HALF, QTR, THIRD, 2 * THIRD
    if order == 2:
        return [(h, 0, h), (-h, 0, h), (0, h, h), (0, -h, h), (0, 0, 1)]
    if order == 3:
        return [(0, 0, 0), (h, h, 0), (-h, h, 0), (h, -h, 0), (-h, -h, 0),
                (h, 0, h), (-h, 0, h), (0, h, h), (0, -h, h), (0, 0, 1)]
    return [(0, 0, 0), (h, 0, 0), (q, 0, 0), (-q, 0, 0), (-h, 0, 0),
            (0, h, 0), (0, q, 0), (0, -q, 0), (0, -h, 0),
            (h, h, 0), (-h, h, 0), (h, -h, 0), (-h, -h, 0),
            (0, 0, t1), (h, h, t1), (-h, h, t1), (h, -h, t1), (-h, -h, t1),
            (0, 0, t2), (h, 0, t2), (-h, 0, t2), (0, h, t2), (0, -h, t2), (0, 0, 1)]


FACE_WORDS = {
    2: "1 a b t",                                       # (D.2)
    3: "1 a b aa bb ab t tt at bt",                     # (D.7)
    4: "1 a b aa bb ab aaa bbb aab abb t tt ttt at bt att btt aat bbt abt",  # (D.12)
}


def face_mode_list(order):
    """Face modes as (degree in t1, degree in t2, power of tau)."""
    out = []
    for w in FACE_WORDS[order].split():
        out.append((0, 0, 0) if w == "1" else (w.count('a'), w.count('b'), w.count('t')))
    return out


def face_modes(order):
    """The face flux modes of (D.4), (D.9), (D.14) as combinations of the
    facial nodal fluxes f_1 .. f_n (1-based list of Lin)."""
    n = len(face_nodes(order))
    f = unknowns('f', n)
    m = [None] * (len(face_mode_list(order)) + 1)
    if order == 2:
        m[2] = f[1] - f[2]
        m[3] = f[3] - f[4]
        m[4] = f[5] * 2 - S(f[1], f[2], f[3], f[4]) * HALF
        m[1] = f[5] - m[4]
    elif order == 3:
        q2 = (f[2] + f[4] - f[1] * 4 + f[3] + f[5]) * HALF
        q3 = f[6] + f[7] - f[8] - f[9]
        m[1] = (f[1] + S(f[2], f[3], f[4], f[5]) * Fr(1, 8)) * Fr(2, 3)
        m[2] = (f[2] + f[4] - f[3] - f[5]) * HALF
        m[3] = (f[2] + f[3] - f[4] - f[5]) * HALF
        m[4] = q2 + q3
        m[5] = q2 - q3
        m[6] = f[2] - f[3] - f[4] + f[5]
        m[8] = (f[1] + f[10]) * 2 - S(f[6], f[7], f[8], f[9]) + q2
        m[7] = f[10] - f[1] - m[8]
        m[9] = (f[6] - f[7] - m[2]) * 2
        m[10] = (f[8] - f[9] - m[3]) * 2
    else:
        q1 = (f[20] - f[21]) * 3 - (f[15] - f[16] + f[17] - f[18]) * Fr(3, 2)
        q2 = (f[20] - f[21] - f[2] + f[5]) * Fr(3, 2)
        q3 = (f[22] - f[23]) * 3 - (f[15] + f[16] - f[17] - f[18]) * Fr(3, 2)
        q4 = (f[22] - f[23] - f[6] + f[9]) * Fr(3, 2)
        m[1] = (f[1] * 2 + f[2] + f[5] + f[6] + f[9]) / 6
        m[4] = (f[2] - f[1] * 2 + f[5]) * 2
        m[5] = (f[6] - f[1] * 2 + f[9]) * 2
        m[6] = f[10] - f[11] - f[12] + f[13]
        m[7] = (f[2] - f[3] * 2 + f[4] * 2 - f[5]) * Fr(16, 3)
        m[8] = (f[6] - f[7] * 2 + f[8] * 2 - f[9]) * Fr(16, 3)
        m[9] = (f[10] - f[6] * 2 + f[11] - f[12] + f[9] * 2 - f[13]) * 2
        m[10] = (f[10] - f[2] * 2 + f[12] - f[11] + f[5] * 2 - f[13]) * 2
        m[2] = f[2] - f[5] + m[10] / 12 - m[7] * Fr(1, 10)
        m[3] = f[6] - f[9] + m[9] / 12 - m[8] * Fr(1, 10)
        m[13] = (f[24] - f[1]) * Fr(9, 2) - (f[19] - f[14]) * Fr(27, 2)
        m[12] = (f[24] - f[19] - f[14] + f[1] - m[13] * Fr(2, 3)) * Fr(9, 4)
        m[11] = (f[24] * Fr(3, 2) - f[14] * Fr(5, 2) + S(f[15], f[16], f[17], f[18]) * QTR
                 - m[4] * QTR - m[5] * QTR - m[12] * Fr(4, 3) - m[13] * Fr(13, 9))
        m[14] = q2 * 3 - q1 * 2 - m[10] * Fr(3, 2)
        m[16] = (q1 - q2) * 3 + m[10] * Fr(9, 4)
        m[15] = q4 * 3 - q3 * 2 - m[9] * Fr(3, 2)
        m[17] = (q3 - q4) * 3 + m[9] * Fr(9, 4)
        m[18] = (f[20] - f[19] * 2 + f[21]) * 3 - m[4] * Fr(3, 2)
        m[19] = (f[22] - f[19] * 2 + f[23]) * 3 - m[5] * Fr(3, 2)
        m[20] = (f[15] - f[16] - f[17] + f[18]) * 3 - m[6] * 3
    return m


def _weights_of(lin):
    return {j: c for (name, j), c in lin.items()}


def face_average_weights(order):
    """(D.4)/(D.9)/(D.14) composed with the exact face integral (D.5)/(D.10)/
    (D.15): face average of the normal flux as a weighted sum over facial
    nodes (only nodes of nonzero weight are returned)."""
    m = face_modes(order)
    avg = Lin()
    for k, (a1, a2, d) in enumerate(face_mode_list(order)):
        if a1 == 0 and a2 == 0:
            avg = avg + m[k + 1] * Fr(1, d + 1)
    return _weights_of(avg)


def edge_average_weights(order, which, sign):
    """Average of the face flux polynomial along the edge t_which = sign/2
    (over the other transverse coordinate and tau, eq. 57), as weights over
    facial nodes."""
    m = face_modes(order)
    avg = Lin()
    for k, (a1, a2, d) in enumerate(face_mode_list(order)):
        a_on, a_off = (a1, a2) if which == 0 else (a2, a1)
        if a_off == 0:
            avg = avg + m[k + 1] * (P(a_on, HALF * sign) / (d + 1))
    return _weights_of(avg)


# ------------------------------------------------------------- sides --------

SIDES = [(0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)]


def transverse(d):
    return {0: (1, 2), 1: (0, 2), 2: (0, 1)}[d]


def side_point(d, s, t1, t2, tau):
    p = [Fr(0)] * 3
    p[d] = HALF * s
    a, b = transverse(d)
    p[a] = Fr(t1)
    p[b] = Fr(t2)
    return (p[0], p[1], p[2], Fr(tau))


def face_average_u_row(order, d, s):
    """eq. (55): weights on the modes for the face average of u."""
    row = []
    for (a, b, c, dd) in mode_list(order):
        e = (a, b, c)
        if all(e[x] == 0 for x in transverse(d)):
            row.append(P(e[d], HALF * s) / (dd + 1))
        else:
            row.append(Fr(0))
    return row


# ---------------------------------------------------------------- WENO ------

def weno_tables(order):
    """Candidate matrices (cell averages -> moments 1..M-1) for the M-zone
    stencils covering zone 0, and the smoothness quadratic forms."""
    M = order

    def cell_avg(a, o):
        # average of P_a over [o - 1/2, o + 1/2], exactly from antiderivatives
        lo, hi = Fr(o) - HALF, Fr(o) + HALF
        coeffs = {0: [1], 1: [0, 1], 2: [Fr(-1, 12), 0, 1], 3: [0, Fr(-3, 20), 0, 1]}[a]
        tot = Fr(0)
        for p, c in enumerate(coeffs):
            tot += Fr(c) * (hi ** (p + 1) - lo ** (p + 1)) / (p + 1)
        return tot

    mats = []
    for start in range(-(M - 1), 1):
        st = list(range(start, start + M))
        V = [[cell_avg(a, o) for a in range(M)] for o in st]
        mats.append(_inv(V))
    return mats


def _inv(A):
    n = len(A)
    M = [list(r) + [Fr(int(i == j)) for j in range(n)] for i, r in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [x - fac * y for x, y in zip(M[r], M[c])]
    return [r[n:] for r in M]


# ------------------------------------------------------------ emission ------

# Floating-point operations per zone of the per-zone kernel, counted on the
# emitted code (one per add, multiply, divide, square root; five variables):
#   a point evaluation with t nonzero terms: t - 1 adds and one multiply per
#     coefficient other than 1 (the deviation form drops the add of mode 0);
#   one Euler flux (physics_device.h): 18, or 43 as a deviation flux;
#   one accumulation into a mode: 2 per variable;
#   one positivity check of a point (pressure of the state): 9, plus 5 adds
#     of the zone average in the deviation form.
#   (MHD: eight variables, one MHD flux 50 or 103, one check 16 or 24.)
FLUX_FLOPS = {'euler': 18, 'mhd': 50, 'euler-dev': 43, 'mhd-dev': 103}
CHECK_FLOPS = {'euler': 9, 'mhd': 16, 'euler-dev': 14, 'mhd-dev': 24}
NV_OF = {'euler': 5, 'mhd': 8, 'euler-dev': 5, 'mhd-dev': 8}
SYSTEM = 'euler'    # system whose flops the current emission pass counts
COUNT = {}


def _is_mhd():
    return SYSTEM.startswith('mhd')


def _is_dev():
    return SYSTEM.endswith('-dev')


def _count(key, n):
    """Count under (tag, part) for the system of this pass; parts of the other
    system's code are not counted."""
    tag, part = key
    if part.endswith('-mhd-lin'):
        return
    if part.endswith('-mhd') != _is_mhd() and part != 'predictor':
        return
    k = (tag + ('-mhd' if _is_mhd() else '') + ('-dev' if _is_dev() else ''),
         part.replace('-mhd', ''))
    COUNT[k] = COUNT.get(k, 0) + n


def _eval_flops(row):
    nz = [c for c in row if c != 0]
    adds = len(nz) - 1 - (1 if _is_dev() and row[0] != 0 and len(nz) > 1 else 0)
    return NV_OF[SYSTEM] * (adds + sum(1 for c in nz if c != 1))

def lit(c):
    c = Fr(c)
    if c.denominator == 1:
        return "T(%d.0)" % c.numerator
    return "T(%d.0 / %d.0)" % (c.numerator, c.denominator)


def _terms(row, ls, comp="v"):
    """Source terms of a point evaluation except mode 0."""
    terms = []
    for m, c in enumerate(row):
        if c == 0 or m == 0:
            continue
        src = ("w[%d][%s]" % (m, comp)) if m < ls else ("e[%d][%s]" % (m - ls, comp))
        terms.append(src if c == 1 else "%s * %s" % (lit(c), src))
    return terms


def _value(row, ls, comp="v"):
    """Expression of a point value: with the zone average (mode 0) in the
    point form, without it (the deviation from the average) in the deviation
    form, selected by the constant DEV of the enclosing function."""
    terms = _terms(row, ls, comp)
    if row[0] == 0:
        return " + ".join(terms) if terms else "T(0)"
    assert row[0] == 1
    rest = " + ".join(terms)
    if not terms:
        return "DEV ? T(0) : w[0][%s]" % comp
    return "DEV ? (%s) : (w[0][%s] + %s)" % (rest, comp, rest)


def emit_eval(out, order, pt, dst, indent="    ", count=None):
    """dst[v] = sum over modes with nonzero basis value at pt."""
    row = point_row(order, pt)
    if count:
        _count(count, _eval_flops(row))
    out.append(indent + "for (int v = 0; v < NV; ++v) %s[v] = %s;" % (dst, _value(row, LS[order])))


def emit_spatial_eval(out, order, pt, dst, indent="    ", count=None):
    row = point_row(order, (pt[0], pt[1], pt[2], 0))
    ls = LS[order]
    if count:
        _count(count, _eval_flops(row[:ls]))
    out.append(indent + "for (int v = 0; v < NV; ++v) %s[v] = %s;" % (dst, _value(row[:ls], ls)))


def gen_order(order, form):
    nodes = pred_nodes(order, form)
    W = evolution_weights(order, form)
    ls = LS[order]
    ne = len(mode_list(order)) - ls
    tag = "%s%d" % ('N' if form == 'nodal' else 'M', order)
    out = []
    out.append("// ---- %s order %d ----" % ("nodal" if form == 'nodal' else "modal", order))
    out.append("template <class T, int NV> struct Scheme%s {" % tag)
    out.append("  static constexpr int LS = %d, NE = %d;" % (ls, ne))

    # per node, per direction: list of (k, weight); the scaled sources of
    # an active source functor enter as direction 's'
    node_dirs = {}
    for k, lin in enumerate(W):
        for (dname, j), c in lin.items():
            node_dirs.setdefault(j, {}).setdefault(dname, []).append((k, c))
    Ws = source_weights(order, form)
    for k, lin in enumerate(Ws):
        for (_, j), c in lin.items():
            node_dirs.setdefault(j, {}).setdefault('s', []).append((k, c))
    sigma = [sum(lin.values(), Fr(0)) for lin in Ws]

    def emit_node(j, accname, lines, reps):
        pt = nodes[j - 1]
        key = (tag, 'predictor')
        dirs = node_dirs.get(j, {})
        only_src = not any(d in dirs for d in 'fgh')
        lines.append("    // node %d at (%s)" % (j, ", ".join(str(x) for x in pt)))
        if only_src:
            lines.append("    if constexpr (Src::kActive) {")
        else:
            _count(key, reps * _eval_flops(point_row(order, pt)))
        emit_eval(lines, order, pt, "u")
        for dname, axis in (('f', 0), ('g', 1), ('h', 2)):
            ws = dirs.get(dname)
            if not ws:
                continue
            lines.append("    ph.template flux<%d>(u, fl);" % axis)
            _count(key, reps * (FLUX_FLOPS[SYSTEM] + len(ws) * (1 + 2 * NV_OF[SYSTEM])))
            for k, c in ws:
                lines.append("    for (int v = 0; v < NV; ++v) %s[%d][v] += (%s * s%s) * fl[v];"
                             % (accname, k, lit(c), "xyz"[axis]))
        if 's' in dirs:
            if not only_src:
                lines.append("    if constexpr (Src::kActive) {")
            lines.append("      src(u, fl);")
            for k, c in dirs['s']:
                lines.append("      for (int v = 0; v < NV; ++v) %s[%d][v] += %s * fl[v];"
                             % (accname, k, lit(c)))
            if not only_src:
                lines.append("    }")
        if only_src:
            lines.append("    }")

    # predictor
    out.append("  // Picard iterations of the space-time predictor; fluxes at tau = 0")
    out.append("  // nodes are taken once, the others on each of the %d iterations." % (order - 1))
    out.append("  // ph evaluates the physical flux at a point (point form) or")
    out.append("  // the flux minus that of the zone average (deviation form: w[0] unused).")
    out.append("  // src (if Src::kActive) gives the scaled source dt S at a node state (in")
    out.append("  // the deviation form dt S of the deviation, with src.base[v] = dt S of")
    out.append("  // the zone average, which the constant part of the source modes takes).")
    out.append("  template <class Phys>")
    out.append("  __host__ __device__ static __forceinline__ void predict(const T (&w)[LS][NV], T (&e)[NE][NV],")
    out.append("                                        T sx, T sy, T sz, const Phys& ph) {")
    out.append("    predict(w, e, sx, sy, sz, ph, NoSource{});")
    out.append("  }")
    out.append("  template <class Phys, class Src>")
    out.append("  __host__ __device__ static __forceinline__ void predict(const T (&w)[LS][NV], T (&e)[NE][NV],")
    out.append("                                        T sx, T sy, T sz, const Phys& ph, const Src& src) {")
    out.append("    constexpr bool DEV = Phys::kDeviation;")
    out.append("    T u[NV], fl[NV], a0[NE][NV];")
    out.append("    for (int k = 0; k < NE; ++k) for (int v = 0; v < NV; ++v) { a0[k][v] = T(0); e[k][v] = T(0); }")
    const = [(k, c) for k, c in enumerate(sigma) if c != 0]
    if const:
        out.append("    if constexpr (Src::kActive && DEV) {")
        for k, c in const:
            out.append("      for (int v = 0; v < NV; ++v) a0[%d][v] += %s * src.base[v];" % (k, lit(c)))
        out.append("    }")
    for j in range(1, len(nodes) + 1):
        if nodes[j - 1][3] == 0 and j in node_dirs:
            emit_node(j, "a0", out, 1)
    later = [j for j in range(1, len(nodes) + 1) if nodes[j - 1][3] != 0 and j in node_dirs]
    # modes that receive contributions from tau > 0 nodes change on every
    # iteration; the others are final after the tau = 0 pass
    moving = sorted({k for j in later for ws in node_dirs[j].values() for k, _ in ws})
    if not later:
        for k in range(ne):
            out.append("    for (int v = 0; v < NV; ++v) e[%d][v] = a0[%d][v];" % (k, k))
    else:
        out.append("    for (int it = 0; it < %d; ++it) {" % (order - 1))
        out.append("      T a1[NE][NV];")
        for k in moving:
            out.append("      for (int v = 0; v < NV; ++v) a1[%d][v] = a0[%d][v];" % (k, k))
        body = []
        for j in later:
            emit_node(j, "a1", body, order - 1)
        out.extend("  " + b for b in body)
        # the new iterate; every node of this iteration used the previous one
        for k in range(ne):
            src = "a1" if k in moving else "a0"
            out.append("      for (int v = 0; v < NV; ++v) e[%d][v] = %s[%d][v];" % (k, src, k))
        out.append("    }")
    out.append("  }")
    # the space-time mean of the polynomial minus its zone average (the pure
    # time modes), for dt times the space-time average of an affine source
    mw = mean_weights(order)
    out.append("  // space-time mean of u over the element minus the zone average")
    out.append("  __host__ __device__ static __forceinline__ void mean_dev(const T (&e)[NE][NV], double (&m)[NV]) {")
    terms = " + ".join("%.17g * double(e[%d][v])" % (float(c), k - ls) for k, c in sorted(mw.items()))
    out.append("    for (int v = 0; v < NV; ++v) m[v] = %s;" % terms)
    out.append("  }")

    # spatial check points (positivity, before the predictor)
    fav = face_average_weights(order)
    fnodes = face_nodes(order)
    sp = set()
    for p in nodes:
        sp.add((Fr(p[0]), Fr(p[1]), Fr(p[2])))
    for d, s in SIDES:
        for j in sorted(fav):
            t1, t2, tau = fnodes[j - 1]
            p = side_point(d, s, t1, t2, tau)
            sp.add(p[:3])
        p = side_point(d, s, 0, 0, HALF)
        sp.add(p[:3])
    sp = sorted(sp)
    out.append("  // %d spatial check points of the positivity safeguard" % len(sp))
    out.append("  template <class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void spatial_points(const T (&w)[LS][NV], Acc& acc) {")
    out.append("    constexpr bool DEV = Acc::kDeviation;")
    out.append("    T u[NV];")
    for p in sp:
        emit_spatial_eval(out, order, p, "u", count=(tag, 'positivity'))
        _count((tag, 'positivity'), CHECK_FLOPS[SYSTEM])
        out.append("    acc(u);")
    out.append("  }")

    # tables of the same points for the exact (rare) positivity pass
    fpts = []
    for d, s_ in SIDES:
        for j in sorted(fav):
            t1, t2, tau = fnodes[j - 1]
            fpts.append(side_point(d, s_, t1, t2, tau))
        fpts.append(side_point(d, s_, 0, 0, HALF))
    out.append("  static constexpr int NSPATIAL = %d, NFACIAL = %d;" % (len(sp), len(fpts)))
    out.append("  // basis values of the spatial modes at the spatial check points")
    out.append("  static constexpr double spatial_phi[%d][%d] = {" % (len(sp), ls))
    for p in sp:
        row = point_row(order, (p[0], p[1], p[2], 0))[:ls]
        out.append("    {%s}," % ", ".join("%.17g" % float(c) for c in row))
    out.append("  };")
    L = len(mode_list(order))
    out.append("  // basis values of all modes at the facial check points")
    out.append("  static constexpr double facial_phi[%d][%d] = {" % (len(fpts), L))
    for p in fpts:
        row = point_row(order, p)
        out.append("    {%s}," % ", ".join("%.17g" % float(c) for c in row))
    out.append("  };")

    # facial check points after the predictor
    out.append("  // facial nodes entering the face averages, and barycentres, of all sides")
    out.append("  template <class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void facial_points(const T (&w)[LS][NV], const T (&e)[NE][NV], Acc& acc) {")
    out.append("    constexpr bool DEV = Acc::kDeviation;")
    out.append("    T u[NV];")
    for d, s in SIDES:
        for j in sorted(fav):
            t1, t2, tau = fnodes[j - 1]
            emit_eval(out, order, side_point(d, s, t1, t2, tau), "u")
            out.append("    acc(u);")
        emit_eval(out, order, side_point(d, s, 0, 0, HALF), "u")
        out.append("    acc(u);")
    out.append("  }")

    # face packets
    out.append("  // side packet: barycentre state (eq. 54), face average of u (eq. 55),")
    out.append("  // face average of the physical normal flux (App. D composed); in the")
    out.append("  // deviation form all three are taken minus their zone-average values.")
    out.append("  // acc sees every state the side evaluates (the facial check set of the")
    out.append("  // positivity safeguard: the barycentre and the face-average nodes).")
    out.append("  template <int SIDE, class Phys, class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void side(const T (&w)[LS][NV], const T (&e)[NE][NV], const Phys& ph,")
    out.append("                                     Acc& acc, T (&ub)[NV], T (&ua)[NV], T (&fa)[NV]) {")
    out.append("    constexpr bool DEV = Phys::kDeviation;")
    out.append("    T u[NV], fl[NV];")
    for si, (d, s) in enumerate(SIDES):
        out.append("    %sif constexpr (SIDE == %d) {  // axis %d, side %+d" % ("" if si == 0 else "else ", si, d, s))
        emit_eval(out, order, side_point(d, s, 0, 0, HALF), "ub", indent="      ",
                  count=(tag, 'faces'))
        out.append("      acc(ub);")
        _count((tag, 'positivity'), CHECK_FLOPS[SYSTEM])
        row = face_average_u_row(order, d, s)
        _count((tag, 'faces'), _eval_flops(row))
        out.append("      for (int v = 0; v < NV; ++v) ua[v] = %s;" % _value(row, ls))
        out.append("      for (int v = 0; v < NV; ++v) fa[v] = T(0);")
        for j in sorted(fav):
            t1, t2, tau = fnodes[j - 1]
            emit_eval(out, order, side_point(d, s, t1, t2, tau), "u", indent="      ",
                      count=(tag, 'faces'))
            out.append("      acc(u);")
            _count((tag, 'positivity'), CHECK_FLOPS[SYSTEM])
            _count((tag, 'faces'), FLUX_FLOPS[SYSTEM] + 2 * NV_OF[SYSTEM])
            out.append("      ph.template flux<%d>(u, fl);" % d)
            out.append("      for (int v = 0; v < NV; ++v) fa[v] += %s * fl[v];" % lit(fav[j]))
        out.append("    }")
    out.append("  }")
    if form == 'modal':
        out += gen_rk_side(order, tag, fav, fnodes)
    out += gen_mhd_parts(order, form, tag, nodes, fnodes)
    out.append("};")
    return out


def gen_rk_side(order, tag, fav, fnodes):
    """Side packet of an SSP-RK stage (Sec. II.d): the App. D quadrature
    applied to the spatial polynomial held constant in time.  Facial nodes
    that differ only in tau then carry the same state, so their weights are
    merged and each distinct face point is evaluated once."""
    ls = LS[order]
    merged = {}
    for j in sorted(fav):
        t1, t2, _ = fnodes[j - 1]
        key = (Fr(t1), Fr(t2))
        merged[key] = merged.get(key, 0) + fav[j]
    pts = [(k, c) for k, c in sorted(merged.items()) if c != 0]
    key = (tag + "rk", 'faces')
    out = []
    out.append("  // side packet of an SSP-RK stage (the predictor bypassed): barycentre")
    out.append("  // state, face average of u and of the normal flux of the spatial")
    out.append("  // polynomial at the stage time (App. D with the tau-direction dropped:")
    out.append("  // %d face points per side)." % len(pts))
    out.append("  template <int SIDE, class Phys, class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void side_rk(const T (&w)[LS][NV], const Phys& ph,")
    out.append("                                     Acc& acc, T (&ub)[NV], T (&ua)[NV], T (&fa)[NV]) {")
    out.append("    constexpr bool DEV = Phys::kDeviation;")
    out.append("    T u[NV], fl[NV];")
    for si, (d, s) in enumerate(SIDES):
        out.append("    %sif constexpr (SIDE == %d) {  // axis %d, side %+d" % ("" if si == 0 else "else ", si, d, s))
        emit_spatial_eval(out, order, side_point(d, s, 0, 0, 0), "ub", indent="      ", count=key)
        out.append("      acc(ub);")
        row = face_average_u_row(order, d, s)[:ls]
        _count(key, _eval_flops(row))
        out.append("      for (int v = 0; v < NV; ++v) ua[v] = %s;" % _value(row, ls))
        out.append("      for (int v = 0; v < NV; ++v) fa[v] = T(0);")
        for (t1, t2), c in pts:
            emit_spatial_eval(out, order, side_point(d, s, t1, t2, 0), "u", indent="      ", count=key)
            out.append("      acc(u);")
            _count(key, FLUX_FLOPS[SYSTEM] + 2 * NV_OF[SYSTEM])
            out.append("      ph.template flux<%d>(u, fl);" % d)
            out.append("      for (int v = 0; v < NV; ++v) fa[v] += %s * fl[v];" % lit(c))
        out.append("    }")
    out.append("  }")
    return out


def gen_mhd_parts(order, form, tag, nodes, fnodes):
    """MHD members: check sets over every facial node (the edge averages use
    them all), their tables, and the side packet with the edge averages of
    eq. (57) of the field component along each transverse axis."""
    ls = LS[order]
    L = len(mode_list(order))
    nf = len(fnodes)
    out = []
    sp = set((Fr(p[0]), Fr(p[1]), Fr(p[2])) for p in nodes)
    fpts = []
    for d, s_ in SIDES:
        for j in range(1, nf + 1):
            fpts.append(side_point(d, s_, *fnodes[j - 1]))
        fpts.append(side_point(d, s_, 0, 0, HALF))
    for p in fpts:
        sp.add(p[:3])
    sp = sorted(sp)
    out.append("  // ---- MHD: every facial node checked; side packets with edge averages")
    out.append("  static constexpr int NSPATIAL_ALL = %d, NFACIAL_ALL = %d;" % (len(sp), len(fpts)))
    out.append("  static constexpr double spatial_phi_all[%d][%d] = {" % (len(sp), ls))
    for p in sp:
        row = point_row(order, (p[0], p[1], p[2], 0))[:ls]
        out.append("    {%s}," % ", ".join("%.17g" % float(c) for c in row))
    out.append("  };")
    out.append("  static constexpr double facial_phi_all[%d][%d] = {" % (len(fpts), L))
    for p in fpts:
        out.append("    {%s}," % ", ".join("%.17g" % float(c) for c in point_row(order, p)))
    out.append("  };")
    out.append("  template <class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void spatial_points_all(const T (&w)[LS][NV], Acc& acc) {")
    out.append("    constexpr bool DEV = Acc::kDeviation;")
    out.append("    T u[NV];")
    for p in sp:
        emit_spatial_eval(out, order, p, "u", count=(tag, 'positivity-mhd'))
        _count((tag, 'positivity-mhd'), CHECK_FLOPS[SYSTEM])
        out.append("    acc(u);")
    out.append("  }")
    out.append("  template <class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void facial_points_all(const T (&w)[LS][NV], const T (&e)[NE][NV], Acc& acc) {")
    out.append("    constexpr bool DEV = Acc::kDeviation;")
    out.append("    T u[NV];")
    for p in fpts:
        emit_eval(out, order, p, "u")
        out.append("    acc(u);")
    out.append("  }")
    fav = face_average_weights(order)
    ew = {(which, sg): edge_average_weights(order, which, sg) for which in (0, 1) for sg in (-1, 1)}
    out.append("  // ue[q], fe[q]: edge averages of u and of the normal flux of the field")
    out.append("  // component along transverse axis t_w, edge q = 2 w + (sign > 0);")
    out.append("  // Phys::comp(c) is where variable c sits in this lane's arrays.  acc sees")
    out.append("  // the barycentre and every facial node (the MHD facial check set).")
    out.append("  template <int SIDE, class Phys, class Acc>")
    out.append("  __host__ __device__ static __forceinline__ void side_edges(const T (&w)[LS][NV], const T (&e)[NE][NV], const Phys& ph,")
    out.append("      Acc& acc, T (&ub)[NV], T (&ua)[NV], T (&fa)[NV], T (&ue)[4], T (&fe)[4]) {")
    out.append("    constexpr bool DEV = Phys::kDeviation;")
    out.append("    T u[NV], fl[NV];")
    edge_rows = {}
    for si, (d, s_) in enumerate(SIDES):
        tr = transverse(d)
        out.append("    %sif constexpr (SIDE == %d) {  // axis %d, side %+d" % ("" if si == 0 else "else ", si, d, s_))
        emit_eval(out, order, side_point(d, s_, 0, 0, HALF), "ub", indent="      ",
                  count=(tag, 'faces-mhd'))
        out.append("      acc(ub);")
        _count((tag, 'positivity-mhd'), CHECK_FLOPS[SYSTEM])
        row = face_average_u_row(order, d, s_)
        _count((tag, 'faces-mhd'), _eval_flops(row))
        out.append("      for (int v = 0; v < NV; ++v) ua[v] = %s;" % _value(row, ls))
        # edge averages of u, component of the edge's transverse axis
        for which in (0, 1):
            a = tr[which]
            free = 3 - d - a
            for sg in (-1, 1):
                q = 2 * which + (1 if sg > 0 else 0)
                row = []
                for m, (ea, eb, ec, dd) in enumerate(mode_list(order)):
                    ex = (ea, eb, ec)
                    row.append(0 if ex[free] != 0 else
                               P(ex[d], HALF * s_) * P(ex[a], HALF * sg) / (dd + 1))
                _count((tag, 'faces-mhd'), 2 * (sum(1 for c in row if c != 0) - (1 if _is_dev() else 0)))
                out.append("      ue[%d] = %s;" % (q, _value(row, ls, "Phys::comp(%d)" % (5 + a))))
                edge_rows.setdefault(si, {})[q] = row
        out.append("      for (int v = 0; v < NV; ++v) fa[v] = T(0);")
        out.append("      for (int q = 0; q < 4; ++q) fe[q] = T(0);")
        for j in range(1, nf + 1):
            used_face = j in fav
            used_edge = [(which, sg) for which in (0, 1) for sg in (-1, 1) if j in ew[(which, sg)]]
            emit_eval(out, order, side_point(d, s_, *fnodes[j - 1]), "u", indent="      ",
                      count=(tag, 'faces-mhd'))
            out.append("      acc(u);")
            _count((tag, 'positivity-mhd'), CHECK_FLOPS[SYSTEM])
            if not used_face and not used_edge:
                continue
            out.append("      ph.template flux<%d>(u, fl);" % d)
            _count((tag, 'faces-mhd'), FLUX_FLOPS[SYSTEM])
            if used_face:
                out.append("      for (int v = 0; v < NV; ++v) fa[v] += %s * fl[v];" % lit(fav[j]))
                _count((tag, 'faces-mhd'), 2 * NV_OF[SYSTEM])
            for which, sg in used_edge:
                q = 2 * which + (1 if sg > 0 else 0)
                a = tr[which]
                out.append("      fe[%d] += %s * fl[Phys::comp(%d)];" % (q, lit(ew[(which, sg)][j]), 5 + a))
                _count((tag, 'faces-mhd'), 2)
        out.append("    }")
    out.append("  }")
    # the same side packet split in two: the linear part (barycentre, face and
    # edge averages of u) as code, the nodal part (fluxes at the facial nodes)
    # as tables a loop walks one node at a time
    out.append("  // facial nodes per side; side_node_w[j]: node j's weight in the face")
    out.append("  // average of the flux, then in the edge averages q = 0..3 (as ue/fe)")
    out.append("  static constexpr int NFACE_NODES = %d;" % nf)
    out.append("  static constexpr double side_node_w[%d][5] = {" % nf)
    for j in range(1, nf + 1):
        ws = [fav.get(j, 0)] + [ew[(which, sg)].get(j, 0) for which in (0, 1) for sg in (-1, 1)]
        out.append("    {%s}," % ", ".join("%.17g" % float(c) for c in ws))
    out.append("  };")
    # edge averages of every variable (the linearized solver's edge states)
    # as rows over all modes, per side and edge
    out.append("  static constexpr double edge_rows_all[6][4][%d] = {" % L)
    for si in range(len(SIDES)):
        out.append("    {%s}," % ", ".join(
            "{%s}" % ", ".join("%.17g" % float(c) for c in edge_rows[si][q]) for q in range(4)))
    out.append("  };")
    out.append("  template <int SIDE, class Phys>")
    out.append("  __host__ __device__ static __forceinline__ void side_linear(const T (&w)[LS][NV], const T (&e)[NE][NV],")
    out.append("      T (&ub)[NV], T (&ua)[NV], T (&ue)[4]) {")
    out.append("    constexpr bool DEV = Phys::kDeviation;")
    for si, (d, s_) in enumerate(SIDES):
        tr = transverse(d)
        out.append("    %sif constexpr (SIDE == %d) {" % ("" if si == 0 else "else ", si))
        emit_eval(out, order, side_point(d, s_, 0, 0, HALF), "ub", indent="      ")
        row = face_average_u_row(order, d, s_)
        out.append("      for (int v = 0; v < NV; ++v) ua[v] = %s;" % _value(row, ls))
        for q in range(4):
            a = tr[q // 2]
            out.append("      ue[%d] = %s;" % (q, _value(edge_rows[si][q], ls, "Phys::comp(%d)" % (5 + a))))
        out.append("    }")
    out.append("  }")
    # every component's edge averages (the linearized solver's edge problems)
    out.append("  // ue[q][v]: edge average (eq. 57) of variable v on edge q of side SIDE")
    out.append("  template <int SIDE, bool DEV>")
    out.append("  __host__ __device__ static __forceinline__ void edge_states(const T (&w)[LS][NV], const T (&e)[NE][NV],")
    out.append("                                                         T (&ue)[4][NV]) {")
    for si in range(len(SIDES)):
        out.append("    %sif constexpr (SIDE == %d) {" % ("" if si == 0 else "else ", si))
        for q in range(4):
            row = edge_rows[si][q]
            _count((tag, 'faces-mhd-lin'), NV_OF[SYSTEM] * (2 * sum(1 for c in row if c != 0) - 1))
            out.append("      for (int v = 0; v < NV; ++v) ue[%d][v] = %s;" % (q, _value(row, ls)))
        out.append("    }")
    out.append("  }")
    return out


def gen_weno():
    out = ["// ---- centred WENO tables: candidate moments from the stencil's averages ----"]
    for order in (3, 4):
        mats = weno_tables(order)
        M = order
        out.append("template <class T> struct Weno%d {" % order)
        out.append("  // cand<s>(d, m): moments m[1..%d] of stencil s (zones s-%d .. s) from" % (M - 1, M - 1))
        out.append("  // the averages d[0..%d] at offsets -%d..%d" % (2 * M - 2, M - 1, M - 1))
        for s, mat in enumerate(mats):
            out.append("  __host__ __device__ static __forceinline__ void cand%d(const T* d, T* m) {" % s)
            for a in range(1, M):
                terms = []
                for q in range(M):
                    c = mat[a][q]
                    if c != 0:
                        terms.append("%s * d[%d]" % (lit(c), s + q))
                out.append("    m[%d] = %s;" % (a, " + ".join(terms)))
            out.append("  }")
        out.append("};")
    return out


def face_point_rows(order):
    """Basis values of the space-time modes at the side points the face
    quadrature evaluates (App. D): per side the barycentre and the
    face-average nodes, the six sides in the order of SIDES."""
    fav = face_average_weights(order)
    fn = face_nodes(order)
    rows = []
    for d, s in SIDES:
        rows.append(point_row(order, side_point(d, s, 0, 0, HALF)))
        for j in sorted(fav):
            t1, t2, tau = fn[j - 1]
            rows.append(point_row(order, side_point(d, s, t1, t2, tau)))
    return rows


def _flit(c):
    """FP32 literal of a rational."""
    t = "%.9g" % float(c)
    return t + ("f" if ("." in t or "e" in t) else ".0f")


def gen_face_rows():
    """generated/face_rows.h: the side-point evaluation matrices of orders 3
    and 4 as FP32 tables, the operand of the measurement library's VALU
    against MFMA comparison of that contraction."""
    out = ["// GENERATED by gen_scheme.py -- do not edit by hand.",
           "// Side-point evaluation of the space-time polynomial (App. D): row p holds",
           "// the basis values of the space-time modes at side point p (per side the",
           "// barycentre, then the face-average nodes; sides -x, +x, -y, +y, -z, +z).",
           "#pragma once",
           "namespace ader_gen {"]
    for order in (3, 4):
        rows = face_point_rows(order)
        P, K = len(rows), len(rows[0])
        nnz = sum(1 for r in rows for c in r if c != 0)
        out.append("constexpr int kFaceP%d = %d, kFaceK%d = %d, kFaceNnz%d = %d;"
                   % (order, P, order, K, order, nnz))
        out.append("constexpr float kFaceRows%d[%d][%d] = {" % (order, P, K))
        for r in rows:
            out.append("    {" + ", ".join(_flit(c) for c in r) + "},")
        out.append("};")
    out.append("}  // namespace ader_gen")
    return out


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    lines = [
        "// GENERATED by gen_scheme.py -- do not edit by hand.",
        "// Straight-line per-zone pieces of the ADER-CG step (see gen_scheme.py for",
        "// the derivation from the paper's equations).",
        "#pragma once",
        "namespace ader_gen {",
        "// The inactive source of a step without a source term.",
        "struct NoSource {",
        "  static constexpr bool kActive = false;",
        "  template <class U>",
        "  __host__ __device__ void operator()(const U&, U&) const {}",
        "};",
    ]
    global SYSTEM
    for order, form in ((2, 'modal'), (2, 'nodal'), (3, 'modal'), (3, 'nodal'), (4, 'modal'),
                        (4, 'nodal')):
        SYSTEM = 'euler'
        lines += gen_order(order, form)
        for SYSTEM in ('mhd', 'euler-dev', 'mhd-dev'):   # same code, counted again
            gen_order(order, form)
    SYSTEM = 'euler'
    lines += gen_weno()
    lines.append("}  // namespace ader_gen")
    os.makedirs(os.path.join(here, "generated"), exist_ok=True)
    with open(os.path.join(here, "generated", "ader_scheme.h"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.join(here, "generated", "face_rows.h"), "w") as fh:
        fh.write("\n".join(gen_face_rows()) + "\n")
    counts = {}
    for (tag, part), n in sorted(COUNT.items()):
        counts.setdefault(tag, {})[part] = n
    for tag in counts:
        counts[tag]['total'] = sum(counts[tag].values())
    import json
    with open(os.path.join(here, "generated", "flop_counts.json"), "w") as fh:
        json.dump({"unit": "flops per zone of k_predict (tags without -mhd: Euler, 5 "
                           "variables; -mhd: ideal MHD, 8 variables; -dev: the deviation "
                           "form of the mixed-precision path)",
                   "counts": counts}, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
