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


# ---------------------------------------------------------------- MHD ------

FOUR_PI = 4.0 * np.pi


def _mhd_conserved(rho, v, P, Bbar, gamma):
    """Hydro part (5 components) of the MHD state; E includes |Bbar|^2/8pi,
    Bbar the zone field taken as the mean of its two face values."""
    U = _euler_conserved(rho, v, P, gamma)
    U[4] += (Bbar * Bbar).sum(axis=0) / (2.0 * FOUR_PI)
    return U


def face_mean(B):
    """Zone field as the mean of the two face values of each component."""
    return np.stack([0.5 * (B[d] + np.roll(B[d], -1, axis=2 - d)) for d in range(3)])


def _edge_integrals(shape, modes):
    """Line integrals of A = sum a sin(2 pi k.x + phi) along the lower zone
    edges: L[c][k][j][i] = int A_c along the c-edge from the corner
    (i dx, j dy, k dz), exactly."""
    nz, ny, nx = shape
    h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    X = (np.arange(nx) / nx)[None, None, :]
    Y = (np.arange(ny) / ny)[None, :, None]
    Z = (np.arange(nz) / nz)[:, None, None]
    L = np.zeros((3,) + tuple(shape))
    for a, k, ph in modes:
        base = 2.0 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph
        for c in range(3):
            if a[c] == 0.0:
                continue
            if k[c] == 0:
                val = h[c] * np.sin(base)
            else:
                step = 2.0 * np.pi * k[c] * h[c]
                val = (np.cos(base) - np.cos(base + step)) / (2.0 * np.pi * k[c])
            L[c] += a[c] * np.broadcast_to(val, tuple(shape))
    return L


def curl_of_edges(L, shape):
    """Face-averaged B = discrete curl (Stokes) of the edge integrals; the
    discrete divergence vanishes identically."""
    nz, ny, nx = shape
    dx, dy, dz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    Lx, Ly, Lz = L
    up = lambda f, axis: np.roll(f, -1, axis=2 - axis)  # noqa: E731
    Bx = (up(Lz, 1) - Lz - up(Ly, 2) + Ly) / (dy * dz)
    By = (up(Lx, 2) - Lx - up(Lz, 0) + Lz) / (dx * dz)
    Bz = (up(Ly, 0) - Ly - up(Lx, 1) + Lx) / (dx * dy)
    return np.stack([Bx, By, Bz])


def mhd_random_field(shape, seed=2146, gamma=5.0 / 3.0, n_modes=16, kmax=4, b_rms=1.0,
                     p0=0.1, drho=0.05):
    """Ideal-MHD workload: face-centred B from the curl of a random vector
    potential (``n_modes`` Fourier modes, integer k in [-kmax, kmax]^3,
    normal random amplitudes, random phases), scaled to rms |B| = b_rms
    (Gaussian units), so div B = 0 to rounding; rho = 1 + drho * delta with
    delta a smooth random field (16 modes, max |delta| = 1); P = p0; v = 0.
    Returns (U[5], B[3]) with B[d] on the lower d-faces."""
    rng = np.random.default_rng(seed)
    modes = [(rng.normal(size=3), k, ph) for k, ph in _random_modes(rng, n_modes, kmax)]
    B = curl_of_edges(_edge_integrals(shape, modes), shape)
    rms = np.sqrt((B * B).sum(axis=0).mean())
    if rms > 0:        # a mesh too small to carry a curl field (1 zone) keeps B = 0
        B *= b_rms / rms
    nz, ny, nx = shape
    X = _centres(nx)[None, None, :]
    Y = _centres(ny)[None, :, None]
    Z = _centres(nz)[:, None, None]
    delta = np.zeros(tuple(shape))
    for k, ph in _random_modes(rng, 16, kmax):
        delta = delta + rng.normal() * np.sin(2.0 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
    delta /= np.abs(delta).max()
    rho = 1.0 + drho * delta
    v = np.zeros((3,) + tuple(shape))
    P = np.full(tuple(shape), p0)
    return _mhd_conserved(rho, v, P, face_mean(B), gamma), B


def alfven_wave_x(shape, t=0.0, gamma=5.0 / 3.0, eps=0.1, p0=1.0, vx=0.0):
    """Circularly polarised Alfven wave along x (an exact nonlinear solution
    of ideal MHD): rho = 1, P = p0, B_x = sqrt(4 pi), v_y + i v_z =
    eps e^{i phi}, B_y + i B_z = -eps sqrt(4 pi) e^{i phi},
    phi = 2 pi (x - (vx + 1) t).  Zone and face averages are exact."""
    nz, ny, nx = shape
    b0 = np.sqrt(FOUR_PI)
    h = 1.0 / nx
    s = np.sin(np.pi * h) / (np.pi * h)
    xc = _centres(nx)[None, None, :]
    ph = 2.0 * np.pi * (xc - (vx + 1.0) * t)
    shp = tuple(shape)
    rho = np.ones(shp)
    v = np.zeros((3,) + shp)
    v[0] = vx
    v[1] = np.broadcast_to(eps * s * np.cos(ph), shp)
    v[2] = np.broadcast_to(eps * s * np.sin(ph), shp)
    B = np.zeros((3,) + shp)
    B[0] = b0
    B[1] = np.broadcast_to(-eps * b0 * s * np.cos(ph), shp)   # y-faces: x-average over the zone
    B[2] = np.broadcast_to(-eps * b0 * s * np.sin(ph), shp)
    U = _euler_conserved(rho, v, np.full(shp, p0), gamma)
    # exact zone average of rho v^2/2 + B^2/8pi (no sinc on the squares)
    U[4] = p0 / (gamma - 1.0) + 0.5 * vx * vx + 0.5 * eps * eps + (b0 * b0 * (1.0 + eps * eps)) / (2.0 * FOUR_PI)
    U[2] = rho * v[1]
    U[3] = rho * v[2]
    return U, B


def alfven_wave_diagonal(shape, t=0.0, gamma=5.0 / 3.0, eps=0.1, p0=1.0):
    """Torsional (circularly polarised) Alfven wave travelling along the cube
    diagonal n = (1,1,1)/sqrt(3) on the periodic unit box (the Sec. VI.3
    set-up with a wave vector k = 2 pi (1,1,1), periodic on the box):
    rho = 1, P = p0, B = sqrt(4 pi) n + dB, v = dv,
    dv = eps (cos phi e2 + sin phi e3), dB = -sqrt(4 pi) dv, phi = k.x - |k| t.
    The face fields come from the exact edge integrals of the vector
    potential of dB plus the uniform part, so div B = 0 to rounding; zone
    averages are exact.  Returns (U[5], B[3])."""
    nz, ny, nx = shape
    shp = tuple(shape)
    b0 = np.sqrt(FOUR_PI)
    n = np.ones(3) / np.sqrt(3.0)
    e2 = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    e3 = np.cross(n, e2)
    kvec = 2.0 * np.pi * np.ones(3)
    kabs = np.sqrt(kvec @ kvec)
    ph0 = -kabs * t
    alpha = eps * b0 / kabs
    # A = alpha (cos phi e2 + sin phi e3) = alpha e2 sin(phi + pi/2) + alpha e3 sin(phi)
    modes = [(alpha * e2, np.array([1, 1, 1]), ph0 + 0.5 * np.pi),
             (alpha * e3, np.array([1, 1, 1]), ph0)]
    B = curl_of_edges(_edge_integrals(shp, modes), shp)
    for d in range(3):
        B[d] += b0 * n[d]
    X = _centres(nx)[None, None, :]
    Y = _centres(ny)[None, :, None]
    Z = _centres(nz)[:, None, None]
    sinc = lambda h: np.sin(np.pi * h) / (np.pi * h)  # noqa: E731
    s = sinc(1.0 / nx) * sinc(1.0 / ny) * sinc(1.0 / nz)
    phc = 2.0 * np.pi * (X + Y + Z) + ph0
    cos_avg = np.broadcast_to(s * np.cos(phc), shp)
    sin_avg = np.broadcast_to(s * np.sin(phc), shp)
    U = np.zeros((5,) + shp)
    U[0] = 1.0
    for d in range(3):
        U[1 + d] = eps * (e2[d] * cos_avg + e3[d] * sin_avg)
    # |v|^2 = eps^2 and |B|^2 = 4 pi (1 + eps^2) are uniform, so E is exact
    U[4] = p0 / (gamma - 1.0) + 0.5 * eps * eps + b0 * b0 * (1.0 + eps * eps) / (2.0 * FOUR_PI)
    return U, B


ENSEMBLE_SIDES = (32, 48, 64, 96)


def ensemble_shapes(n=64, seed=4096, sides=ENSEMBLE_SIDES):
    """(nz, ny, nx) of n problems, each side drawn independently and
    uniformly from ``sides`` (the uneven batched-ensemble workload)."""
    rng = np.random.default_rng(seed)
    return [tuple(int(s) for s in rng.choice(sides, size=3)) for _ in range(n)]


def ensemble(n=64, seed=4096, sides=ENSEMBLE_SIDES):
    """The batched ensemble: n independent periodic unit-box problems of the
    uneven shapes of ``ensemble_shapes``, each with its own seeded smooth
    random-mode state (``random_smooth`` with seed ``seed + 1 + i``).
    Returns a list of (shape, U)."""
    return [(s, random_smooth(s, seed + 1 + i))
            for i, s in enumerate(ensemble_shapes(n, seed, sides))]


def _spectral_modes(rng, count, kmax, slope=-5.0 / 3.0):
    """count random integer wave vectors in [-kmax, kmax]^3 \\ 0, each with a
    random phase and a random direction of amplitude |k|^slope."""
    ks, amps, phases = [], [], []
    while len(ks) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if not np.any(k != 0):
            continue
        d = rng.normal(size=3)
        ks.append(k)
        amps.append(d / np.linalg.norm(d) * np.linalg.norm(k) ** slope)
        phases.append(rng.uniform(0.0, 2.0 * np.pi))
    return np.array(ks), np.array(amps), np.array(phases)


def _separable_sum(shape, ks, coef, factors):
    """Im sum_m coef_m X_m(i) Y_m(j) Z_m(k) on the mesh, one plane at a time
    as a matrix product (factors(axis, k, n) gives the per-axis factor)."""
    nz, ny, nx = shape
    out = np.empty(tuple(shape))
    FX = np.stack([factors(0, ks[m, 0], nx) for m in range(len(ks))], axis=0)   # (M, nx)
    FY = np.stack([factors(1, ks[m, 1], ny) for m in range(len(ks))], axis=1)   # (ny, M)
    FZ = np.stack([factors(2, ks[m, 2], nz) for m in range(len(ks))], axis=1)   # (nz, M)
    for kz in range(nz):
        out[kz] = ((FY * (coef * FZ[kz])[None, :]) @ FX).imag
    return out


def turbulent_mhd(shape, seed=384, gamma=5.0 / 3.0, n_modes=64, kmax=8, p0=0.6, mach=1.0,
                  b_rms=1.0):
    """Turbulent-like ideal-MHD state on the periodic unit box: velocity and
    vector potential each from ``n_modes`` random Fourier modes (integer
    wave vectors in [-kmax, kmax]^3, random directions, amplitudes |k|^-5/3),
    velocity scaled to rms Mach ``mach`` at rho = 1, P = ``p0``; face B the
    exact face fluxes of curl A (edge line integrals, Stokes), scaled to rms
    |B| = ``b_rms``, so div B = 0 to rounding.  Velocity at zone centres.
    Returns (U[5], B[3]).  Evaluated as sums of separable products, one
    z-plane per matrix product, so 384^3 takes seconds."""
    rng = np.random.default_rng(seed)
    kv, av, pv = _spectral_modes(rng, n_modes, kmax)
    ka, aa, pa = _spectral_modes(rng, n_modes, kmax)
    nz, ny, nx = shape

    def centre(axis, k, n):
        x = (np.arange(n) + 0.5) / n
        return np.exp(2j * np.pi * k * x)

    v = np.stack([_separable_sum(shape, kv, av[:, c] * np.exp(1j * pv), centre) for c in range(3)])
    rms = np.sqrt((v * v).sum(axis=0).mean())
    v *= mach * np.sqrt(gamma * p0) / rms

    # line integrals of A_c along the lower c-edges: the c-factor integrated
    # over the zone, the other two taken at the lower corner
    L = []
    for c in range(3):
        def edge(axis, k, n, c=c):
            x = np.arange(n) / n
            if axis != c:
                return np.exp(2j * np.pi * k * x)
            if k == 0:
                return np.full(n, 1.0 / n, dtype=complex)
            return (np.exp(2j * np.pi * k * (x + 1.0 / n)) - np.exp(2j * np.pi * k * x)) / (2j * np.pi * k)
        L.append(_separable_sum(shape, ka, aa[:, c] * np.exp(1j * pa), edge))
    B = curl_of_edges(np.stack(L), shape)
    rms = np.sqrt((B * B).sum(axis=0).mean())
    if rms > 0:
        B *= b_rms / rms
    rho = np.ones(tuple(shape))
    P = np.full(tuple(shape), p0)
    return _mhd_conserved(rho, v, P, face_mean(B), gamma), B


def isentropic_vortex(n, t=0.0, length=10.0, eps=5.0, gamma=1.4, quad=5):
    """The two-dimensional isentropic vortex of Sec. VI.1 on an n x n mesh
    with one zone in z: shape (1, n, n), the periodic box [0, length]^2 in
    x and y standing for [-length/2, length/2]^2, and lz = length.  Mean
    flow rho = P = 1, v = (1, 1, 0); the vortex adds
        dv = eps / 2 pi exp((1 - r^2) / 2) (-y, x),
        dT = -(gamma - 1) eps^2 / (8 gamma pi^2) exp(1 - r^2)
    at constant entropy (T = P / rho, P / rho^gamma = 1), centred at
    (t, t) (the exact solution at time t: the vortex carried by the mean
    flow, periodically; the nearest periodic image of the centre counts).
    Zone averages of the conserved variables by a quad x quad
    Gauss-Legendre rule per zone."""
    g, w = np.polynomial.legendre.leggauss(quad)
    h = length / n
    edges = np.arange(n) * h
    pts = (edges[:, None] + 0.5 * h * (g[None, :] + 1.0)).ravel()     # (n * quad,)
    wts = np.tile(0.5 * w, n)
    X = pts[None, :] - 0.5 * length
    Y = pts[:, None] - 0.5 * length
    cx = (t + 0.5 * length) % length - 0.5 * length
    dx = (X - cx + 0.5 * length) % length - 0.5 * length
    dy = (Y - cx + 0.5 * length) % length - 0.5 * length
    r2 = dx * dx + dy * dy
    amp = eps / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    vx = 1.0 - amp * dy
    vy = 1.0 + amp * dx
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    P = rho * T
    v = np.stack([vx, vy, np.zeros_like(vx)])
    Uq = _euler_conserved(rho, v, P, gamma)                            # (5, n q, n q)
    Wq = wts[:, None] * wts[None, :]
    Uz = (Uq * Wq).reshape(5, n, quad, n, quad).sum(axis=(2, 4))
    return Uz[:, None, :, :].copy()


def magnetized_vortex(n, t=0.0, length=10.0, kappa=1.0, mu=1.0, gamma=5.0 / 3.0, quad=5):
    """The two-dimensional magnetized isodensity vortex of Sec. VI.2 on an
    n x n mesh with one zone in z: U of shape (5, 1, n, n) and face fields
    B of shape (3, 1, n, n), the periodic box [0, length]^2 standing for
    [-length/2, length/2]^2, lz = length.  Mean flow rho = P = 1, v = (1, 1,
    0), B = 0; the vortex adds
        dv = kappa / 2 pi exp((1 - r^2) / 2) (-y, x),
        dB = mu / 2 pi exp((1 - r^2) / 2) (-y, x),
        dP = (mu / 2 pi)^2 (1 - r^2) exp(1 - r^2) / 8 pi
             - (kappa / 2 pi)^2 exp(1 - r^2) / 2
    (Gaussian units), rho = 1 everywhere, centred at (t, t): the exact
    solution at time t (nearest periodic image of the centre).  The face
    fields are exact face averages, the differences of the potential
    A_z = mu / 2 pi exp((1 - r^2) / 2) at the face's corners divided by the
    edge length, so their discrete divergence vanishes; the zone averages
    of rho v and of E = P / (gamma - 1) + rho |v|^2 / 2 + |B|^2 / 8 pi come
    from a quad x quad Gauss-Legendre rule per zone."""
    h = length / n
    cx = (t + 0.5 * length) % length - 0.5 * length

    def rel(c):
        return (c - 0.5 * length - cx + 0.5 * length) % length - 0.5 * length

    g, w = np.polynomial.legendre.leggauss(quad)
    edges = np.arange(n) * h
    pts = (edges[:, None] + 0.5 * h * (g[None, :] + 1.0)).ravel()
    wts = np.tile(0.5 * w, n)
    dx = rel(pts)[None, :]
    dy = rel(pts)[:, None]
    r2 = dx * dx + dy * dy
    e1 = np.exp(0.5 * (1.0 - r2))
    av = kappa / (2.0 * np.pi) * e1
    ab = mu / (2.0 * np.pi) * e1
    vx, vy = 1.0 - av * dy, 1.0 + av * dx
    bx, by = -ab * dy, ab * dx
    P = (1.0 + (mu / (2.0 * np.pi)) ** 2 * (1.0 - r2) * e1 * e1 / (8.0 * np.pi)
         - 0.5 * (kappa / (2.0 * np.pi)) ** 2 * e1 * e1)
    rho = np.ones_like(P)
    Uq = np.stack([rho, rho * vx, rho * vy, np.zeros_like(rho),
                   P / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
                   + (bx * bx + by * by) / (2.0 * FOUR_PI)])
    Wq = wts[:, None] * wts[None, :]
    U = (Uq * Wq).reshape(5, n, quad, n, quad).sum(axis=(2, 4))[:, None, :, :].copy()
    # A_z at the corners (x_i, y_j) of the mesh, single-valued on the torus
    cxs, cys = rel(edges)[None, :], rel(edges)[:, None]
    Az = mu / (2.0 * np.pi) * np.exp(0.5 * (1.0 - (cxs * cxs + cys * cys)))   # [j][i]
    B = np.zeros((3, 1, n, n))
    B[0, 0] = (np.roll(Az, -1, axis=0) - Az) / h       # B_x = dA_z/dy on x-faces
    B[1, 0] = -(np.roll(Az, -1, axis=1) - Az) / h      # B_y = -dA_z/dx on y-faces
    return U, B


def field_loop(nx, ny, a0=1e-3, radius=0.3, v=(2.0, 1.0), rho=1.0, p=1.0, gamma=5.0 / 3.0):
    """A weak magnetic field loop advected by a uniform flow across the
    periodic box [-1, 1] x [-1/2, 1/2] on nx x ny zones with one zone in z
    (the field-loop test of Sec. VIII, set up after its cited reference):
    A_z = a0 (radius - r) inside r < radius, zero outside, so |B| = a0 in
    the loop; rho, P uniform; v = (2, 1) brings the loop back to its start
    at t = 1.  Face fields are the differences of A_z at the face's corners
    divided by the edge length (discrete div B zero); U of shape
    (5, 1, ny, nx), B of shape (3, 1, ny, nx)."""
    hx, hy = 2.0 / nx, 1.0 / ny
    x = -1.0 + np.arange(nx) * hx
    y = -0.5 + np.arange(ny) * hy
    r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
    Az = np.where(r < radius, a0 * (radius - r), 0.0)    # [j][i] at corner (x_i, y_j)
    B = np.zeros((3, 1, ny, nx))
    B[0, 0] = (np.roll(Az, -1, axis=0) - Az) / hy       # B_x = dA_z/dy on x-faces
    B[1, 0] = -(np.roll(Az, -1, axis=1) - Az) / hx      # B_y = -dA_z/dx on y-faces
    shape = (1, ny, nx)
    vel = np.stack([np.full(shape, v[0]), np.full(shape, v[1]), np.zeros(shape)])
    U = _mhd_conserved(np.full(shape, rho), vel, np.full(shape, p), face_mean(B), gamma)
    return U, B


def mhd_rotor(n, b0=5.0, rho_in=10.0, rho_out=1.0, r0=0.1, r1=0.115, omega=20.0, p=1.0,
              gamma=1.4):
    """The rotor (Sec. VIII) on the periodic unit square, n x n zones and
    one in z: a dense disk (r < r0) spinning at omega about the centre in a
    light medium at rest, with a linear taper of density and angular speed
    over r0 < r < r1, in the uniform field B = (b0, 0, 0) (b0 = 5 in the
    Gaussian units of the step, i.e. 5 / sqrt(4 pi) in Heaviside units, as
    in the usual setup), P = 1.  Point values at the zone centres; U of
    shape (5, 1, n, n), B of shape (3, 1, n, n)."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h - 0.5
    X, Y = np.meshgrid(c, c)                  # [j][i]
    r = np.sqrt(X * X + Y * Y)
    f = np.clip((r1 - r) / (r1 - r0), 0.0, 1.0)
    dens = rho_out + (rho_in - rho_out) * f
    # angular speed: omega inside r0, tapered to zero at r1, zero outside
    w = omega * np.where(r < r0, 1.0, f * r0 / np.maximum(r, 1e-300))
    vx, vy = -w * Y, w * X
    shape = (1, n, n)
    B = np.zeros((3, 1, n, n))
    B[0] = b0
    vel = np.stack([vx.reshape(shape), vy.reshape(shape), np.zeros(shape)])
    U = _mhd_conserved(dens.reshape(shape), vel, np.full(shape, p), face_mean(B), gamma)
    return U, B
