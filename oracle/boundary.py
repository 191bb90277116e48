"""Non-periodic boundaries by ghost zones (the paper runs its boundary
problems with reflecting, inflow and outflow boundaries but describes no
boundary treatment; this is the usual finite-volume reading).  GHOST
layers of zones are added outside each bounded face, filled from the
interior zone averages:

* outflow (zero gradient): a ghost zone takes the average of the nearest
  interior zone along the axis;
* reflect (wall): a ghost zone takes the mirror-image zone's average with
  the momentum component normal to the wall negated;
* inflow: a ghost zone takes a given state (the face's inflow state).

The axes are padded in the order x, y, z, each from the array the previous
ones padded, so a zone outside two bounded faces (a corner) takes the later
axis's rule applied to the earlier axis's ghost values (an inflow ghost row
of y holds the inflow state across the x ghosts too; a reflect ghost row of
y mirrors the x ghosts, inflow states included).  The periodic step of
``oracle.step`` then runs on the padded mesh;
the interior results are the bounded step (with GHOST >= the order, no
interior result depends on the padded mesh's periodic wrap).  In the check
mode only the interior and the first ghost layer -- the zones whose
polynomials reach an interior face -- are tested.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from dataclasses import replace

import numpy as np

from .step import compute_dt, step

GHOST = 4
KINDS = ('periodic', 'outflow', 'reflect', 'inflow')


def _source_index(n, lo, hi, g):
    """Interior index and momentum sign of each padded index along an axis
    of n interior zones (lo, hi: the kinds at the lower and upper face)."""
    idx, sgn = [], []
    lo_pad = g if lo != 'periodic' else 0
    hi_pad = g if hi != 'periodic' else 0
    for p in range(-lo_pad, n + hi_pad):
        if p < 0:
            if lo in ('outflow', 'inflow'):     # inflow: overwritten by the caller
                idx.append(0); sgn.append(1.0)
            else:
                idx.append(-1 - p); sgn.append(-1.0)
        elif p >= n:
            if hi in ('outflow', 'inflow'):
                idx.append(n - 1); sgn.append(1.0)
            else:
                idx.append(2 * n - 1 - p); sgn.append(-1.0)
        else:
            idx.append(p); sgn.append(1.0)
    return np.array(idx), np.array(sgn), lo_pad


def _check_kinds(bc):
    for axis in range(3):
        lo, hi = bc[axis]
        if lo not in KINDS or hi not in KINDS:
            raise ValueError('boundary kind %r' % ((lo, hi),))
        if (lo == 'periodic') != (hi == 'periodic'):
            raise ValueError('a periodic axis is periodic on both faces')


def pad(U, bc, g=GHOST, inflow=None):
    """U padded with ghost zones on the bounded faces; bc[axis] = (lower,
    upper) kinds for axis 0 (x), 1 (y), 2 (z); inflow[(axis, side)] (side 0
    lower, 1 upper) the conserved state of each inflow face.  Returns
    (padded U, offsets (x, y, z) of the interior in the padded mesh)."""
    _check_kinds(bc)
    inflow = inflow or {}
    for axis in range(3):
        for side in range(2):
            if bc[axis][side] == 'inflow' and (axis, side) not in inflow:
                raise ValueError('inflow face (%d, %d) without a state' % (axis, side))
    nz, ny, nx = U.shape[1:]
    out = U
    offs = []
    for axis, n in ((0, nx), (1, ny), (2, nz)):
        lo, hi = bc[axis]
        if lo != 'periodic' and n < g:
            raise ValueError('a bounded axis needs at least %d zones' % g)
        idx, sgn, off = _source_index(n, lo, hi, g)
        out = np.take(out, idx, axis=3 - axis)
        shape = [1] * 4
        shape[3 - axis] = len(sgn)
        out = out.copy()
        out[1 + axis] = out[1 + axis] * sgn.reshape(shape[1:])
        for side, sl in ((0, slice(0, off)), (1, slice(off + n, None))):
            if bc[axis][side] == 'inflow':
                st = [slice(None)] * 4
                st[3 - axis] = sl
                out[tuple(st)] = np.asarray(inflow[(axis, side)], dtype=float).reshape(5, 1, 1, 1)
        offs.append(off)
    return out, tuple(offs)


def check_mask(shape, offs, n):
    """Zones of the padded mesh within one zone of the interior along every
    bounded axis."""
    m = np.ones(shape, dtype=bool)
    for axis in range(3):
        o, ni = offs[axis], n[axis]
        if o == 0:
            continue
        p = np.arange(shape[2 - axis]) - o
        keep = (p >= -1) & (p <= ni)
        sl = [None, None, None]
        sl[2 - axis] = slice(None)
        m = m & keep[tuple(sl)]
    return m


def step_bc(U, dt, cfg, bc, inflow=None):
    """One step of the Euler equations with boundaries bc (see pad)."""
    nz, ny, nx = U.shape[1:]
    Up, offs = pad(U, bc, inflow=inflow)
    cfg_p = replace(cfg, zone_size=cfg.spacing(U.shape[1:]),
                    check_mask=check_mask(Up.shape[1:], offs, (nx, ny, nz)))
    Un = step(Up, dt, cfg_p)
    ox, oy, oz = offs
    return Un[:, oz:oz + nz, oy:oy + ny, ox:ox + nx].copy()


def compute_dt_bc(U, cfg, cfl, bc=None, inflow=None):
    """dt of the bounded mesh: the CFL rule over the zones the step reads,
    the interior and the ghost zones; outflow and reflect ghosts copy
    interior states, so only inflow states can add to the interior's."""
    if not inflow:
        return compute_dt(U, cfg, cfl)
    Up, _ = pad(U, bc, inflow=inflow)
    return compute_dt(Up, replace(cfg, zone_size=cfg.spacing(U.shape[1:])), cfl)
