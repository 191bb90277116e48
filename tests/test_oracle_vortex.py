"""Pins of the oracle's two-dimensional path (one zone in z) on the
isentropic vortex of Sec. VI.1 (Table I): design order in the density's L1
error against the exact solution (the vortex carried by the mean flow),
and the generator's own exactness (a full crossing of the periodic box
returns the initial state)."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt, step
from paper_1006_2146_amd import workloads


def test_vortex_generator_is_periodic_and_isentropic():
    U0 = workloads.isentropic_vortex(32)
    assert np.array_equal(workloads.isentropic_vortex(32, t=10.0), U0)
    assert np.allclose(workloads.isentropic_vortex(40, t=20.0, length=20.0),
                       workloads.isentropic_vortex(40, length=20.0), rtol=0, atol=1e-13)
    # the mean state away from the vortex, no z velocity
    assert np.all(U0[3] == 0.0)
    assert abs(U0[0, 0, 0, 0] - 1.0) < 1e-4


def _run(n, order, T, length=10.0):
    cfg = OracleConfig(order=order, riemann='hll', lengths=(length, length, length))
    U = workloads.isentropic_vortex(n, length=length)
    t = 0.0
    while t < T - 1e-12:
        dt = min(compute_dt(U, cfg, 0.3), T - t)
        U = step(U, dt, cfg)
        t += dt
    return np.abs(U[0] - workloads.isentropic_vortex(n, t=T, length=length)[0]).mean()


@pytest.mark.slow
@pytest.mark.parametrize("order,floor", [(3, 2.6), (4, 3.7)])
def test_vortex_design_order(order, floor):
    # Table I: the modal ADER-CG with HLL meets its design order in the L1
    # density error; here at t = 0.5 on 32^2 and 64^2 zones (measured 2.81
    # and 4.32); the longer runs of Table I itself are run on the GPU
    e32, e64 = _run(32, order, 0.5), _run(64, order, 0.5)
    assert np.log2(e32 / e64) > floor, (e32, e64)


def test_magnetized_vortex_generator():
    # Sec. VI.2's vortex: the face fields are exact face averages of the
    # field of the printed formula (checked against Gauss quadrature of the
    # point field along each face), their discrete divergence vanishes, the
    # state is periodic over one crossing, and rho = 1
    from oracle.bweno import divergence
    n, L = 24, 10.0
    U, B = workloads.magnetized_vortex(n, length=L)
    h = L / n
    assert np.abs(divergence(B, (h, h, L))).max() <= 1e-14 * np.abs(B).max() / h
    assert np.all(B[2] == 0.0) and np.allclose(U[0], 1.0, rtol=0, atol=1e-14)
    U2, B2 = workloads.magnetized_vortex(n, t=L, length=L)
    assert np.array_equal(U2, U) and np.array_equal(B2, B)
    g, w = np.polynomial.legendre.leggauss(8)

    def point_b(x, y):
        r2 = x * x + y * y
        a = 1.0 / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
        return -a * y, a * x

    for j, i in ((3, 17), (12, 12), (20, 5)):
        x0, y0 = i * h - 0.5 * L, j * h - 0.5 * L
        ys = y0 + 0.5 * h * (g + 1.0)
        xs = x0 + 0.5 * h * (g + 1.0)
        bx = 0.5 * (w * point_b(np.full_like(ys, x0), ys)[0]).sum()
        by = 0.5 * (w * point_b(xs, np.full_like(xs, y0))[1]).sum()
        assert abs(B[0, 0, j, i] - bx) <= 1e-13 and abs(B[1, 0, j, i] - by) <= 1e-13
