"""Zone moments of the magnetic field from its face-centred normal components
(Sec. III).

Face storage: B[0][k][j][i] is the x-component averaged over the x-face at
x = i dx (the lower x-face of zone (i,j,k)); B[1] and B[2] likewise on the
lower y- and z-faces.

For component d of zone i the face values along axis d at offsets
i-1/2, i+1/2 (and i -+ 3/2, i -+ 5/2) are interpolated by a polynomial in
P_1..P_{M-1} (eq. 21, 25); its zone average is b_0 and its moments b_x, b_xx,
b_xxx are the normal variation.  Candidates: order 2 the single two-face
interpolant (b_0 = mean, b_x = difference); order 3 the stencils S1, S2 of
eq. (22)-(23); order 4 the stencils S1, S2, S3 of eq. (26)-(28).  The oracle
builds each candidate as the interpolant through its face values (the plain
definition; a pin checks the printed formulas against it) and weights them
with the smoothness indicator of eq. (24)/(29).  Linear weights (a reading;
the paper says only "non-linear convex combination"): equal at order 3,
(1, 100, 1) at order 4, eps = 1e-12, omega ~ lambda / (eps + IS)^2.

Remaining moments (a reading of "any suitable reconstruction"): the
zone-centred reconstruction of ``weno.reconstruct`` applied to the b_0 field,
whose pure-normal moments (P_a along the component's own axis) are then
replaced by the values above.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

import numpy as np

from .basis import P, SPATIAL_MODES, N_SPATIAL
from .weno import reconstruct, smoothness_matrix, WENO_EPS

# face offsets (in zone widths, from the zone centre) of each candidate
FACE_STENCILS = {
    2: [[-0.5, 0.5]],
    3: [[-1.5, -0.5, 0.5], [-0.5, 0.5, 1.5]],
    4: [[-2.5, -1.5, -0.5, 0.5], [-1.5, -0.5, 0.5, 1.5], [-0.5, 0.5, 1.5, 2.5]],
}
FACE_LAMBDA = {2: [1.0], 3: [1.0, 1.0], 4: [1.0, 100.0, 1.0]}


def candidate_matrix(offsets, order):
    """Moments (b_0 .. b_{M-1}) of the polynomial in P_0..P_{M-1} through the
    point values at ``offsets``; order 2 has two faces for two moments."""
    V = np.array([[float(P(a, x)) for a in range(order)] for x in offsets])
    return np.linalg.inv(V)


def _nb(arr, axis, o):
    return np.roll(arr, -o, axis=arr.ndim - 1 - axis)


def normal_moments(Bd, d, order):
    """(b_0, .., b_{M-1}) of every zone from the d-faces of component d."""
    # face at offset x - 1/2 + q, i.e. face index i + q for q in -2..3
    def face(off):
        return _nb(Bd, d, int(round(off + 0.5)))
    cands, alphas = [], []
    S = smoothness_matrix(order) if order > 2 else None
    for offs, lam in zip(FACE_STENCILS[order], FACE_LAMBDA[order]):
        Minv = candidate_matrix(offs, order)
        vals = [face(o) for o in offs]
        m = [sum(Minv[a, q] * vals[q] for q in range(order)) for a in range(order)]
        cands.append(m)
        if S is not None:
            IS = sum(S[a, b] * m[a] * m[b] for a in range(order) for b in range(order)
                     if S[a, b] != 0.0)
            alphas.append(lam / (WENO_EPS + IS) ** 2)
    if order == 2:
        return cands[0]
    tot = sum(alphas)
    return [sum(alphas[s] * cands[s][a] for s in range(len(cands))) / tot
            for a in range(order)]


def zone_b_modes(B, order):
    """Spatial modes (L_S, 3, nz, ny, nx) of the zone magnetic field."""
    ls = N_SPATIAL[order]
    out = np.zeros((ls, 3) + B.shape[1:])
    for d in range(3):
        nm = normal_moments(B[d], d, order)
        w = reconstruct(nm[0][None], order)[:, 0]
        for a in range(1, order):
            e = [0, 0, 0]
            e[d] = a
            w[SPATIAL_MODES.index(tuple(e))] = nm[a]
        out[:, d] = w
    return out


def zone_b_mean(B):
    """Arithmetic mean of the two face values of each component (used for
    the CFL speed and for initial energies)."""
    return np.stack([0.5 * (B[d] + _nb(B[d], d, 1)) for d in range(3)])


def divergence(B, dx):
    """Discrete divergence of the face field in every zone."""
    return sum((_nb(B[d], d, 1) - B[d]) / dx[d] for d in range(3))
