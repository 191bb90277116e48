"""Seeded synthetic initial states shaped like the paper's test problems.

This module is the only code shared by the HIP path's tests/benchmark and the
CPU oracle: it builds initial conserved zone averages and holds none of the
ADER step's arithmetic.  Every state is a pure function of its arguments.

Zone averages are exact for single Fourier modes (product of sinc factors) and
otherwise come from a tensor Gauss-Legendre rule per zone (3 points per axis,
exact to degree 5), in the spirit of initialising by quadrature of the
accuracy of the scheme (Sec. VI).  Conserved variables follow eq. (3):
E = rho v^2 / 2 + P / (gamma - 1) (+ B^2 / 8 pi for MHD, Gaussian units).
"""

import numpy as np

GL3_X, GL3_W = np.polynomial.legendre.leggauss(3)


def _centres(n):
    return (np.arange(n) + 0.5) / n


def _euler_conserved(rho, v, P, gamma):
    U = np.empty((5,) + np.shape(rho))
    U[0] = rho
    U[1:4] = rho * v
    U[4] = 0.5 * rho * (v * v).sum(axis=0) + P / (gamma - 1.0)
    return U


def density_wave(shape, gamma=1.4, amp=0.2, t=0.0):
    """rho = 1 + amp sin(2 pi (x + y + z - 3 t)), v = (1, 1, 1), P = 1 on the
    periodic unit box, exact zone averages.  ``shape`` = (nz, ny, nx).

    The advected density wave of Sec. VI.4 laid along the cube diagonal with
    a wavelength that is periodic on the unit box."""
    nz, ny, nx = shape
    X = _centres(nx)[None, None, :]
    Y = _centres(ny)[None, :, None]
    Z = _centres(nz)[:, None, None]
    sinc = lambda h: np.sin(np.pi * h) / (np.pi * h)  # noqa: E731
    s = sinc(1.0 / nx) * sinc(1.0 / ny) * sinc(1.0 / nz)
    rho = 1.0 + amp * s * np.sin(2.0 * np.pi * (X + Y + Z - 3.0 * t))
    rho = np.broadcast_to(rho, shape)
    U = np.empty((5,) + tuple(shape))
    U[0] = rho
    U[1:4] = rho[None]
    U[4] = 1.0 / (gamma - 1.0) + 1.5 * rho
    return U


def _random_modes(rng, count, kmax):
    modes = []
    while len(modes) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            modes.append((k, rng.uniform(0.0, 2.0 * np.pi)))
    return modes


def _quadrature_average(shape, point_state, gamma, slab=8):
    """Zone averages of conserved variables of a primitive state given at
    points: ``point_state(X, Y, Z) -> (rho, v[3], P)``."""
    nz, ny, nx = shape
    U = np.zeros((5, nz, ny, nx))
    hx, hy, hz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        acc = np.zeros((5, z1 - z0, ny, nx))
        for qz, wz in zip(GL3_X, GL3_W):
            Z = (np.arange(z0, z1) + 0.5 + 0.5 * qz)[:, None, None] * hz
            for qy, wy in zip(GL3_X, GL3_W):
                Y = (np.arange(ny) + 0.5 + 0.5 * qy)[None, :, None] * hy
                for qx, wx in zip(GL3_X, GL3_W):
                    X = (np.arange(nx) + 0.5 + 0.5 * qx)[None, None, :] * hx
                    rho, v, P = point_state(X, Y, Z)
                    shp = (z1 - z0, ny, nx)
                    rho = np.broadcast_to(rho, shp)
                    v = np.broadcast_to(v, (3,) + shp)
                    P = np.broadcast_to(P, shp)
                    acc += (wx * wy * wz / 8.0) * _euler_conserved(rho, v, P, gamma)
        U[:, z0:z1] = acc
    return U


def sedov_modes(shape, seed=1006, gamma=1.4, n_modes=8, amp=0.05, kmax=4,
                p_in=100.0, radius=0.05):
    """Background rho = 1, P = 1 with ``n_modes`` random-phase Fourier modes
    of amplitude ``amp`` in each of rho, u, v, w (integer wave vectors in
    [-kmax, kmax]^3), plus an overpressure sphere P = p_in of ``radius``
    around a seeded centre (periodic distance), sampled at the quadrature
    points: the Sedov-like blast workload on the periodic unit box."""
    rng = np.random.default_rng(seed)
    fields = [_random_modes(rng, n_modes, kmax) for _ in range(4)]
    centre = rng.uniform(0.0, 1.0, size=3)

    def series(modes, X, Y, Z):
        out = 0.0
        for k, ph in modes:
            out = out + amp * np.sin(2.0 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return out

    def state(X, Y, Z):
        rho = 1.0 + series(fields[0], X, Y, Z)
        v = np.stack(np.broadcast_arrays(series(fields[1], X, Y, Z),
                                         series(fields[2], X, Y, Z),
                                         series(fields[3], X, Y, Z)))
        d2 = 0.0
        for A, c in zip((X, Y, Z), centre):
            dd = np.abs(A - c)
            dd = np.minimum(dd, 1.0 - dd)
            d2 = d2 + dd * dd
        P = np.where(d2 < radius * radius, p_in, 1.0)
        return rho, v, P

    return _quadrature_average(tuple(shape), state, gamma)


def random_smooth(shape, seed, gamma=1.4, amp=(0.1, 0.2, 0.1), n_modes=3, kmax=2):
    """Smooth random state (rho, v, P) = background + a few Fourier modes,
    sampled at zone centres (not zone averages: used where only a valid
    smooth state is needed)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    X = _centres(nx)[None, None, :]
    Y = _centres(ny)[None, :, None]
    Z = _centres(nz)[:, None, None]

    def field(a):
        out = np.zeros(tuple(shape))
        for k, ph in _random_modes(rng, n_modes, kmax):
            out = out + a * np.sin(2.0 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return out

    rho = 1.0 + field(amp[0])
    v = np.stack([field(amp[1]) for _ in range(3)])
    P = 1.0 + field(amp[2])
    return _euler_conserved(rho, v, P, gamma)


def blast(shape, p_in=10.0, p_out=0.1, radius=0.2, gamma=1.4):
    """Centred overpressure sphere at rest on the unit box (Sec. VIII.3
    shape), sampled at zone centres."""
    nz, ny, nx = shape
    X = _centres(nx)[None, None, :] - 0.5
    Y = _centres(ny)[None, :, None] - 0.5
    Z = _centres(nz)[:, None, None] - 0.5
    r2 = X * X + Y * Y + Z * Z
    P = np.where(r2 < radius * radius, p_in, p_out)
    P = np.broadcast_to(P, tuple(shape))
    rho = np.ones(tuple(shape))
    return _euler_conserved(rho, np.zeros((3,) + tuple(shape)), P, gamma)
