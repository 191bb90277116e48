"""Pins of the oracle's SSP Runge-Kutta stepping (Sec. II.d, eq. 18-20):
the stage coefficients against the order conditions, and whole steps
against constant states, conservation and the design order."""

import numpy as np
import pytest
import sympy as sp

from oracle import OracleConfig, compute_dt
from oracle import rk
from tests.test_oracle_step import _density_wave, _random_smooth_state


@pytest.mark.parametrize("scheme,order,stages", [('ssprk2', 2, 2), ('ssprk3', 3, 3),
                                                 ('ssprk54', 4, 5)])
def test_stability_polynomial_matches_exp(scheme, order, stages):
    # for dU/dt = z U the step multiplies U by a polynomial R(z) of degree
    # "stages"; an order-p scheme has R(z) = exp(z) + O(z^(p+1)).  This pins
    # every printed coefficient of (18)-(20): exactly for (18)-(19); the
    # 14-digit decimals of (20) satisfy the order conditions to about 1e-10,
    # so a wrong digit down to the ninth decimal place fails.
    z = sp.Symbol('z')
    R = sp.expand(rk.ssp_step(sp.Float(1, 30), 1, lambda V: z * V, scheme))
    poly = sp.Poly(R, z)
    assert poly.degree() == stages
    c = [float(poly.coeff_monomial(z ** k)) for k in range(stages + 1)]
    tol = 1e-9 if scheme == 'ssprk54' else 1e-15
    for k in range(order + 1):
        assert abs(c[k] - 1.0 / float(sp.factorial(k))) < tol, (k, c[k])
    if stages > order:
        assert abs(c[order + 1] - 1.0 / float(sp.factorial(order + 1))) > 1e-6


@pytest.mark.parametrize("order", [2, 3, 4])
def test_rk_constant_state_and_conservation(order):
    cfg = OracleConfig(order=order, riemann='hll')
    U = np.zeros((5, 5, 6, 7))
    U[:] = np.array([1.3, 0.2, -0.1, 0.3, 2.5])[:, None, None, None]
    Un = rk.step_rk(U, 0.01, cfg)
    # L vanishes on a constant state; the printed weights of the last stage of
    # (20) sum to 1 - 1e-14, (18)-(19) exactly to 1
    assert np.allclose(Un, U, rtol=(3e-14 if order == 4 else 1e-15), atol=0)
    U = _random_smooth_state(8, 3)
    dt = compute_dt(U, cfg, 0.3)
    Un = rk.step_rk(U, dt, cfg)
    tot0, tot1 = U.sum(axis=(1, 2, 3)), Un.sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(U).sum(axis=(1, 2, 3)))
    assert not np.allclose(Un, U)


def test_rk_stage_is_the_ader_flux_of_a_frozen_polynomial():
    # with the predictor bypassed, L(U) is the ADER update's flux divergence
    # with all evolutionary modes zero: one forward-Euler stage of L equals
    # an ADER step whose predictor returns the spatial polynomial unchanged
    import sys
    from oracle import predictor as pr
    st = sys.modules['oracle.step']
    cfg = OracleConfig(order=3, riemann='hll')
    U = _random_smooth_state(7, 9)
    dt = compute_dt(U, cfg, 0.3)
    orig = pr.predict_modal
    try:
        def frozen(what, order, *a, **k):
            out = np.zeros((pr.N_SPACETIME[order],) + what.shape[1:])
            out[:pr.N_SPATIAL[order]] = what
            return out
        st.predict_modal = frozen
        ref = st.step(U, dt, cfg)
    finally:
        st.predict_modal = orig
    got = U + dt * rk.spatial_operator(U, cfg)
    assert np.allclose(got, ref, rtol=0, atol=1e-14 * np.abs(U).max())


def _run_rk(U, cfg, T, cfl=0.3):
    t = 0.0
    while t < T - 1e-14:
        dt = min(compute_dt(U, cfg, cfl), T - t)
        U = rk.step_rk(U, dt, cfg)
        t += dt
    return U


@pytest.mark.slow
@pytest.mark.parametrize("order,sizes,T", [(2, (16, 32), 0.02), (3, (8, 16), 0.05),
                                           (4, (8, 16), 0.05)])
def test_rk_design_order_density_wave(order, sizes, T):
    cfg = OracleConfig(order=order, riemann='hll')
    errs = []
    for n in sizes:
        U = _run_rk(_density_wave(n, 0.0), cfg, T)
        errs.append(np.abs(U[0] - _density_wave(n, T)[0]).mean())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.6, (errs, rate)


# ------------------------------------------------------------------- MHD --

G53 = 5.0 / 3.0


@pytest.mark.parametrize("order", [2, 3, 4])
def test_rk_mhd_div_b_conservation_and_constant_state(order):
    from oracle.bweno import divergence
    from paper_1006_2146_amd import workloads
    cfg = OracleConfig(order=order, gamma=G53, riemann='hll')
    U, B = workloads.mhd_random_field((7, 8, 9), seed=order)
    dt = compute_dt(U, cfg, 0.3, B)
    Un, Bn = rk.step_rk_mhd(U, B, dt, cfg)
    dx = cfg.spacing(U.shape[1:])
    assert np.abs(divergence(Bn, dx)).max() <= 1e-12 * np.abs(Bn).max() / min(dx)
    tot0, tot1 = U.sum(axis=(1, 2, 3)), Un.sum(axis=(1, 2, 3))
    # (the random field starts at rest: the momenta sum to zero)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(U).sum())
    assert np.allclose(Bn.sum(axis=(1, 2, 3)), B.sum(axis=(1, 2, 3)), rtol=0, atol=1e-11)
    # a uniform magnetised flow stays uniform
    Uc = np.zeros((5, 4, 5, 6))
    Uc[:] = np.array([1.1, 0.2, -0.3, 0.1, 3.0])[:, None, None, None]
    Bc = np.zeros((3, 4, 5, 6))
    Bc[:] = np.array([0.4, -0.2, 0.7])[:, None, None, None]
    Un, Bn = rk.step_rk_mhd(Uc, Bc, 0.01, cfg)
    tol = 3e-14 if order == 4 else 1e-15
    assert np.allclose(Un, Uc, rtol=tol, atol=0) and np.allclose(Bn, Bc, rtol=tol, atol=0)


def test_rk_mhd_stage_is_the_ader_step_of_a_frozen_polynomial():
    import sys
    from oracle import predictor as pr
    from paper_1006_2146_amd import workloads
    st = sys.modules['oracle.step']
    cfg = OracleConfig(order=3, gamma=G53, riemann='linearized')
    U, B = workloads.mhd_random_field((6, 7, 8), seed=11)
    dt = compute_dt(U, cfg, 0.3, B)
    orig = st.predict_modal
    try:
        def frozen(what, order, *a, **k):
            out = np.zeros((pr.N_SPACETIME[order],) + what.shape[1:])
            out[:pr.N_SPATIAL[order]] = what
            return out
        st.predict_modal = frozen
        Ur, Br = st.step(U, dt, cfg, B)
    finally:
        st.predict_modal = orig
    LU, LB = rk.mhd_operator((U, B), cfg)
    assert np.allclose(U + dt * LU, Ur, rtol=0, atol=1e-14 * np.abs(U).max())
    assert np.allclose(B + dt * LB, Br, rtol=0, atol=1e-14 * np.abs(B).max())


@pytest.mark.slow
@pytest.mark.parametrize("order,floor", [(2, 1.7), (3, 2.6)])
def test_rk_mhd_design_order_alfven_wave(order, floor):
    from paper_1006_2146_amd import workloads
    errs = []
    T = 0.04
    cfg = OracleConfig(order=order, gamma=G53)
    for n in (8, 16):
        U, B = workloads.alfven_wave_diagonal((n, n, n))
        t = 0.0
        while t < T - 1e-14:
            dt = min(compute_dt(U, cfg, 0.3, B), T - t)
            U, B = rk.step_rk_mhd(U, B, dt, cfg)
            t += dt
        _, Be = workloads.alfven_wave_diagonal((n, n, n), t=T)
        errs.append(np.abs(B[0] - Be[0]).mean())
    assert np.log2(errs[0] / errs[1]) > floor, errs
