"""Zone-centred reconstruction of the conserved variables (Sec. II.1).

The paper delegates the centred WENO formulas to its reference [11] and only
states that the reconstruction is applied component-wise to the conserved
variables (Sec. VII) and that it yields the Hermite moments of eq. (10)-(12).
The reading implemented here (also used by the GPU path, written separately):

* order 2: per axis, the minmod of the two one-sided differences;
* orders 3 and 4: 1D WENO on cell averages.  Candidates are every stencil of
  M consecutive zones that contains the zone (3 stencils at order 3, 4 at
  order 4).  Each candidate is the unique polynomial of degree M-1 in
  P_1..P_{M-1} whose averages over the stencil's zones match the data.
  Smoothness indicator IS = sum_{l>=1} int_{-1/2}^{1/2} (d^l p/dxi^l)^2, the
  form the paper prints for B in eq. (24) and (29).  Nonlinear weights
  omega_s ~ lambda_s / (eps + IS_s)^2 with lambda = 100 for the stencils that
  are centred (order 3) or nearest-centred (order 4) and 1 otherwise,
  eps = 1e-12;
* 3D moments by sweeps x -> y -> z: the x-sweep of the zone averages gives
  m_a; a y-sweep of each field m_a gives m_ab; a z-sweep of each m_ab gives
  m_abc; moments with a + b + c > M - 1 are dropped.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .basis import P, dP, SPATIAL_MODES, N_SPATIAL

WENO_EPS = 1.0e-12
LAMBDA_CENTRAL = 100.0
LAMBDA_SIDE = 1.0

_GL_X, _GL_W = np.polynomial.legendre.leggauss(6)  # exact to degree 11


def _cell_average_of_P(a, offset):
    """Average of P_a over the zone at integer ``offset`` (zone = [o-1/2, o+1/2])."""
    x = offset + 0.5 * _GL_X
    return float(0.5 * np.dot(_GL_W, P(a, x)))


def stencils(order):
    """Offsets of every M-zone stencil that covers offset 0."""
    M = order
    return [list(range(s, s + M)) for s in range(-(M - 1), 1)]


def linear_weights(order):
    n = len(stencils(order))
    lam = np.full(n, LAMBDA_SIDE)
    if order == 3:
        lam[1] = LAMBDA_CENTRAL
    elif order == 4:
        lam[1] = LAMBDA_CENTRAL
        lam[2] = LAMBDA_CENTRAL
    return lam


def candidate_matrices(order):
    """For each stencil, the M x M matrix mapping its cell averages to the
    moments (m_0 .. m_{M-1}) of the interpolating polynomial."""
    mats = []
    for st in stencils(order):
        V = np.array([[_cell_average_of_P(a, o) for a in range(order)] for o in st])
        mats.append(np.linalg.inv(V))
    return mats


def smoothness_matrix(order):
    """S with IS = m^T S m = sum_{l>=1} int (d^l p)^2 over [-1/2, 1/2],
    p = sum_a m_a P_a; built by Gauss-Legendre quadrature of derivatives."""
    xq = 0.5 * _GL_X
    wq = 0.5 * _GL_W
    S = np.zeros((order, order))
    for l in range(1, order):
        D = np.zeros((order, len(xq)))
        for a in range(order):
            D[a] = _deriv(a, l, xq)
        S += (D * wq) @ D.T
    return S


def _deriv(a, l, x):
    """l-th derivative of P_a evaluated at x (P_a is a cubic at most)."""
    if l == 1:
        return dP(a, x)
    # higher derivatives from the monomial coefficients of eq. (9)
    mono = {0: [1, 0, 0, 0], 1: [0, 1, 0, 0], 2: [-1.0 / 12.0, 0, 1, 0],
            3: [0, -3.0 / 20.0, 0, 1]}[a]
    poly = np.polynomial.polynomial.Polynomial(mono)
    return poly.deriv(l)(x)


_TABLES = {}


def _tables(order):
    if order not in _TABLES:
        _TABLES[order] = (candidate_matrices(order), smoothness_matrix(order),
                          linear_weights(order))
    return _TABLES[order]


def weno1d(vals, order):
    """1D WENO on the cell averages ``vals[o + M - 1]`` for o in -(M-1)..(M-1).

    Returns the moments [m_1, .., m_{M-1}] of the zone at offset 0 (m_0 is the
    cell average itself because P_1..P_3 have zero mean).
    """
    r = order - 1
    mats, S, lam = _tables(order)
    cands = []
    alphas = []
    for s, st in enumerate(stencils(order)):
        data = [vals[o + r] for o in st]
        m = [sum(mats[s][a, q] * data[q] for q in range(order)) for a in range(order)]
        IS = 0.0
        for a in range(order):
            for b in range(order):
                if S[a, b] != 0.0:
                    IS = IS + S[a, b] * m[a] * m[b]
        cands.append(m)
        alphas.append(lam[s] / (WENO_EPS + IS) ** 2)
    total = sum(alphas)
    out = []
    for a in range(1, order):
        out.append(sum(alphas[s] * cands[s][a] for s in range(len(cands))) / total)
    return out


def minmod(a, b):
    """minmod(a, b): 0 if the signs differ, else the one of smaller magnitude."""
    return np.where(a * b > 0.0, np.where(np.abs(a) < np.abs(b), a, b), 0.0)


def _nb(arr, axis, o):
    """Periodic neighbour at offset ``o`` along x (0), y (1) or z (2)."""
    return np.roll(arr, -o, axis=arr.ndim - 1 - axis)


def reconstruct(U, order):
    """Spatial modes w_1..w_{L_S} of eq. (10)-(12) for every zone.

    ``U`` has shape (nv, nz, ny, nx); returns shape (L_S, nv, nz, ny, nx).
    """
    ls = N_SPATIAL[order]
    m = {(0, 0, 0): U}
    if order == 2:
        for axis in range(3):
            key = tuple(1 if i == axis else 0 for i in range(3))
            m[key] = minmod(_nb(U, axis, 1) - U, U - _nb(U, axis, -1))
    else:
        r = order - 1
        M = order
        # x-sweep of the zone averages
        mx = weno1d([_nb(U, 0, o) for o in range(-r, r + 1)], M)
        for a in range(1, M):
            m[(a, 0, 0)] = mx[a - 1]
        # y-sweep of every x-moment that still needs y-moments
        for a in range(0, M - 1):
            src = m[(a, 0, 0)]
            my = weno1d([_nb(src, 1, o) for o in range(-r, r + 1)], M)
            for b in range(1, M - a):
                m[(a, b, 0)] = my[b - 1]
        # z-sweep of every xy-moment that still needs z-moments
        for a in range(0, M - 1):
            for b in range(0, M - 1 - a):
                src = m[(a, b, 0)]
                mz = weno1d([_nb(src, 2, o) for o in range(-r, r + 1)], M)
                for c in range(1, M - a - b):
                    m[(a, b, c)] = mz[c - 1]
    return np.stack([m[mode] for mode in SPATIAL_MODES[:ls]])
