"""Pins of the oracle's MHD pieces: face-B WENO (Sec. III), edge electric
fields and constrained transport (eq. 7-8), and the whole MHD step."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt, step, step_block
from oracle import bweno
from paper_1006_2146_amd import workloads

G = 5.0 / 3.0


def _printed_candidates(order, B):
    """The paper's printed candidates: (22)-(23) at order 3, (26)-(28) at
    order 4.  B maps a face offset (-2.5 .. 2.5) to its value."""
    if order == 3:
        s1 = ((8 * B[-0.5] - B[-1.5] + 5 * B[0.5]) / 12, B[0.5] - B[-0.5],
              (B[0.5] + B[-1.5] - 2 * B[-0.5]) / 2)
        s2 = ((8 * B[0.5] - B[1.5] + 5 * B[-0.5]) / 12, B[0.5] - B[-0.5],
              (B[-0.5] + B[1.5] - 2 * B[0.5]) / 2)
        return [s1, s2]
    s1 = ((9 * B[0.5] + 19 * B[-0.5] - 5 * B[-1.5] + B[-2.5]) / 24,
          (59 * B[0.5] - 57 * B[-0.5] - 3 * B[-1.5] + B[-2.5]) / 60,
          (3 * B[0.5] - 7 * B[-0.5] + 5 * B[-1.5] - B[-2.5]) / 4,
          (B[0.5] - 3 * B[-0.5] + 3 * B[-1.5] - B[-2.5]) / 6)
    s2 = ((-B[1.5] + 13 * B[0.5] + 13 * B[-0.5] - B[-1.5]) / 24,
          (-B[1.5] + 63 * B[0.5] - 63 * B[-0.5] + B[-1.5]) / 60,
          (B[1.5] - B[0.5] - B[-0.5] + B[-1.5]) / 4,
          (B[1.5] - 3 * B[0.5] + 3 * B[-0.5] - B[-1.5]) / 6)
    s3 = ((B[2.5] - 5 * B[1.5] + 19 * B[0.5] + 9 * B[-0.5]) / 24,
          (-B[2.5] + 3 * B[1.5] + 57 * B[0.5] - 59 * B[-0.5]) / 60,
          (-B[2.5] + 5 * B[1.5] - 7 * B[0.5] + 3 * B[-0.5]) / 4,
          (B[2.5] - 3 * B[1.5] + 3 * B[0.5] - B[-0.5]) / 6)
    return [s1, s2, s3]


@pytest.mark.parametrize("order", [3, 4])
def test_face_b_candidates_match_printed_formulas(order):
    # the oracle's interpolants through the face values equal eq. (22)-(23)
    # and (26)-(28) as printed
    rng = np.random.default_rng(order)
    B = {o: rng.normal() for o in (-2.5, -1.5, -0.5, 0.5, 1.5, 2.5)}
    printed = _printed_candidates(order, B)
    for s, offs in enumerate(bweno.FACE_STENCILS[order]):
        Minv = bweno.candidate_matrix(offs, order)
        got = Minv @ np.array([B[o] for o in offs])
        assert np.allclose(got, printed[s], rtol=0, atol=1e-13)


def test_second_order_face_b():
    # Sec. III: b_0 = (B_+ + B_-)/2, b_x = B_+ - B_-
    rng = np.random.default_rng(0)
    Bx = rng.normal(size=(1, 1, 6))
    b0, bx = bweno.normal_moments(Bx, 0, 2)
    assert np.allclose(b0, 0.5 * (Bx + np.roll(Bx, -1, axis=2)))
    assert np.allclose(bx, np.roll(Bx, -1, axis=2) - Bx)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_uniform_mhd_state_is_preserved_bitwise(order):
    n = (4, 5, 6)
    U = np.zeros((5,) + n)
    U[0], U[1], U[2], U[3] = 1.2, 0.1, -0.2, 0.05
    B = np.zeros((3,) + n)
    B[0], B[1], B[2] = 0.5, -0.3, 0.2
    U[4] = 1.5 + 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0] + (B ** 2).sum(0) / (8 * np.pi)
    Un, Bn = step(U, 0.01, OracleConfig(order=order, gamma=G), B)
    assert np.array_equal(Un, U) and np.array_equal(Bn, B)


# The small random-field meshes resolve their k <= 4 modes poorly: at P = 0.1
# the paper's scheme (check mode) meets P <= 0 at check points, so it runs
# at P = 1, and the limit mode (whose scaling then acts) at P = 0.1.
MHD_MODES = [("check", 1.0), ("limit", 0.1)]


@pytest.mark.parametrize("positivity,p0", MHD_MODES)
@pytest.mark.parametrize("order", [2, 3, 4])
def test_div_b_and_conservation(order, positivity, p0):
    U, B = workloads.mhd_random_field((6, 7, 8), seed=order, p0=p0)
    cfg = OracleConfig(order=order, gamma=G, positivity=positivity)
    dx = cfg.spacing(U.shape[1:])
    div0 = np.abs(bweno.divergence(B, dx)).max()
    U1, B1 = U, B
    for _ in range(3):
        U1, B1 = step(U1, compute_dt(U1, cfg, 0.3, B1), cfg, B1)
    scale = np.abs(B).max() / min(dx)
    assert np.abs(bweno.divergence(B1, dx)).max() <= max(div0, 1e-14 * scale) * 10
    assert np.all(np.abs(U1.sum(axis=(1, 2, 3)) - U.sum(axis=(1, 2, 3)))
                  <= 1e-13 * np.abs(U).sum())
    assert np.all(np.abs(B1.sum(axis=(1, 2, 3)) - B.sum(axis=(1, 2, 3))) <= 1e-12 * np.abs(B).sum())
    assert np.abs(B1 - B).max() > 1e-3


@pytest.mark.slow
@pytest.mark.parametrize("order,floor", [(2, 1.7), (3, 2.6)])
def test_design_order_diagonal_alfven_wave(order, floor):
    # Sec. VI.3 / Table III: the torsional Alfven wave along the cube
    # diagonal converges at the design order (error in B_x)
    errs = []
    T = 0.04
    cfg = OracleConfig(order=order, gamma=G)
    for n in (8, 16):
        U, B = workloads.alfven_wave_diagonal((n, n, n))
        t = 0.0
        while t < T - 1e-14:
            dt = min(compute_dt(U, cfg, 0.3, B), T - t)
            U, B = step(U, dt, cfg, B)
            t += dt
        _, Be = workloads.alfven_wave_diagonal((n, n, n), t=T)
        errs.append(np.abs(B[0] - Be[0]).mean())
    assert np.log2(errs[0] / errs[1]) > floor, errs


@pytest.mark.parametrize("positivity,p0", MHD_MODES)
@pytest.mark.parametrize("order", [2, 4])
def test_mhd_step_block_equals_full_step(order, positivity, p0):
    U, B = workloads.mhd_random_field((10, 9, 11), seed=7, p0=p0)
    cfg = OracleConfig(order=order, gamma=G, positivity=positivity)
    dt = compute_dt(U, cfg, 0.3, B)
    Uf, Bf = step(U, dt, cfg, B)
    Ub, Bb = step_block(U, dt, cfg, (8, 2, 9), (3, 2, 4), B)
    iz, iy, ix = np.arange(8, 11) % 10, np.arange(2, 4), np.arange(9, 13) % 11
    pick = lambda A: A[:, iz][:, :, iy][:, :, :, ix]  # noqa: E731
    assert np.array_equal(Ub, pick(Uf)) and np.array_equal(Bb, pick(Bf))


# ------------------------------------------------------ linearized MHD ----

def _random_states(M, seed, vscale=0.5, bscale=2.0):
    from oracle.physics import conserved
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, M)
    v = rng.normal(0.0, vscale, (3, M))
    P = rng.uniform(0.5, 2.0, M)
    B = rng.normal(0.0, bscale, (3, M))
    return conserved(rho, v, P, B, G), (rho, v, P, B)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mhd_jacobian_against_differences_and_wave_speeds(axis):
    # the complex-step Jacobian against central differences of the flux, and
    # its eigenvalues against the closed-form MHD speeds u, u +- c_a,
    # u +- c_s, u +- c_f (Gaussian units)
    from oracle.physics import flux
    from oracle.riemann import mhd_jacobian, seven_wave_slots
    u, (rho, v, P, B) = _random_states(8, axis)
    J = mhd_jacobian(u, axis, G)
    slots = seven_wave_slots(axis)
    for k, s in enumerate(slots):
        h = 1e-6 * max(1.0, np.abs(u[s]).max())
        up, um = u.copy(), u.copy()
        up[s] += h
        um[s] -= h
        fd = (flux(up, axis, G)[slots] - flux(um, axis, G)[slots]) / (2 * h)
        assert np.allclose(J[:, :, k], fd.T, rtol=1e-7, atol=1e-8 * np.abs(J).max())
    a2 = G * P / rho
    ca2 = B[axis] ** 2 / (4 * np.pi * rho)
    b2 = (B * B).sum(axis=0) / (4 * np.pi * rho)
    root = np.sqrt((a2 + b2) ** 2 - 4 * a2 * ca2)
    cf, cs, ca = np.sqrt(0.5 * (a2 + b2 + root)), np.sqrt(0.5 * (a2 + b2 - root)), np.sqrt(ca2)
    un = v[axis]
    speeds = np.sort(np.stack([un - cf, un - ca, un - cs, un, un + cs, un + ca, un + cf]).T, axis=1)
    lam = np.sort(np.linalg.eigvals(J).real, axis=1)
    assert np.allclose(lam, speeds, rtol=0, atol=1e-12)


def test_abs_jacobian_properties():
    # |A|^2 = A^2 and |A| commutes with A; |A| = A when every wave moves
    # to the right (supersonic along the axis)
    from oracle.riemann import frozen_state, mhd_abs_jacobian, mhd_jacobian
    u, _ = _random_states(10, 5)
    ul, ur = u[:, :5], u[:, 5:]
    absA = mhd_abs_jacobian(ul, ur, 1, G)
    A = mhd_jacobian(frozen_state(ul, ur, G).reshape(8, -1), 1, G)
    scale = np.abs(A @ A).max()
    assert np.abs(absA @ absA - A @ A).max() <= 1e-12 * scale
    assert np.abs(absA @ A - A @ absA).max() <= 1e-12 * scale
    fast, _ = _random_states(6, 6, vscale=0.1, bscale=0.3)
    fast[2] = fast[0] * 20.0          # v_y = 20, far above every wave speed
    fast[4] += 0.5 * 400.0 * fast[0]
    absA = mhd_abs_jacobian(fast[:, :3], fast[:, 3:], 1, G)
    A = mhd_jacobian(frozen_state(fast[:, :3], fast[:, 3:], G).reshape(8, -1), 1, G)
    assert np.allclose(absA, A, rtol=0, atol=1e-10 * np.abs(A).max())


def test_linearized_mhd_without_field_is_linearized_euler():
    # with B = 0 the hydro rows of the MHD dissipation are those of the
    # Euler eigen-system (an independent closed form)
    from oracle.physics import conserved
    from oracle.riemann import euler_eigen_dissipation, mhd_abs_jacobian, mhd_dissipation
    _, (rho, v, P, _) = _random_states(8, 7)
    u = conserved(rho, v, P, np.zeros((3, 8)), G)
    ul, ur = u[:, :4], u[:, 4:]
    for axis in range(3):
        D = mhd_dissipation(mhd_abs_jacobian(ul, ur, axis, G), ur - ul, axis)
        De = euler_eigen_dissipation(ul[:5], ur[:5], (ur - ul)[:5], axis, G)
        assert np.allclose(D[:5], De, rtol=1e-12, atol=1e-13 * np.abs(De).max())


def test_linearized_mhd_uniform_state_div_b_and_conservation():
    n = (4, 5, 6)
    U = np.zeros((5,) + n)
    U[0], U[1], U[2], U[3] = 1.2, 0.1, -0.2, 0.05
    B = np.zeros((3,) + n)
    B[0], B[1], B[2] = 0.5, -0.3, 0.2
    U[4] = 1.5 + 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0] + (B ** 2).sum(0) / (8 * np.pi)
    for order in (2, 3):
        cfg = OracleConfig(order=order, gamma=G, riemann="linearized")
        Un, Bn = step(U, 0.01, cfg, B)
        assert np.array_equal(Un, U) and np.array_equal(Bn, B)
    U, B = workloads.mhd_random_field((6, 7, 8), seed=4, p0=1.0)
    cfg = OracleConfig(order=3, gamma=G, riemann="linearized")
    dx = cfg.spacing(U.shape[1:])
    U1, B1 = U, B
    for _ in range(2):
        U1, B1 = step(U1, compute_dt(U1, cfg, 0.3, B1), cfg, B1)
    assert np.abs(bweno.divergence(B1, dx)).max() <= 1e-12 * np.abs(B).max() / min(dx)
    assert np.all(np.abs(U1.sum(axis=(1, 2, 3)) - U.sum(axis=(1, 2, 3))) <= 1e-13 * np.abs(U).sum())
    # less dissipative than HLL but not identical to it
    Uh, Bh = step(U, compute_dt(U, cfg, 0.3, B), OracleConfig(order=3, gamma=G), B)
    Ul, Bl = step(U, compute_dt(U, cfg, 0.3, B), cfg, B)
    assert np.abs(Ul - Uh).max() > 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("order,floor", [(2, 1.7), (3, 2.6)])
def test_design_order_diagonal_alfven_wave_linearized(order, floor):
    errs = []
    T = 0.04
    cfg = OracleConfig(order=order, gamma=G, riemann="linearized")
    for n in (8, 16):
        U, B = workloads.alfven_wave_diagonal((n, n, n))
        t = 0.0
        while t < T - 1e-14:
            dt = min(compute_dt(U, cfg, 0.3, B), T - t)
            U, B = step(U, dt, cfg, B)
            t += dt
        _, Be = workloads.alfven_wave_diagonal((n, n, n), t=T)
        errs.append(np.abs(B[0] - Be[0]).mean())
    assert np.log2(errs[0] / errs[1]) > floor, errs
