"""Pins of the oracle's non-stiff source terms (modal form: Sec. IV source
modes eq. 34, 43, 52, evolution eq. 30, 36, 45, space-time averages eq. 35,
44, 53; nodal form: App. A-C; update eq. 6)."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt, step
from oracle.predictor import gravity_source
from tests.test_oracle_step import _density_wave

G = (0.3, -0.2, 0.5)


def _uniform(rho, v, p, shape=(4, 5, 6), gamma=1.4):
    U = np.zeros((5,) + shape)
    U[0] = rho
    U[1:4] = (rho * np.asarray(v))[:, None, None, None]
    U[4] = p / (gamma - 1.0) + 0.5 * rho * float(np.dot(v, v))
    return U


FORMS = ["modal", "nodal"]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("order", [2, 3, 4])
def test_uniform_gravity_is_exact(order, form):
    # a uniform state under uniform gravity: v(t) = v + g t, rho and p
    # constant, E gains m.g t + rho |g|^2 t^2 / 2 -- a quadratic in time the
    # scheme reproduces at every order (this pins the tau modes of the
    # sources and the weights of the space-time averages)
    cfg = OracleConfig(order=order, form=form, riemann='hll', source=gravity_source(G))
    rho, v, p = 1.3, np.array([0.2, -0.1, 0.3]), 2.0
    dt = 0.05
    Un = step(_uniform(rho, v, p), dt, cfg)
    ve = v + np.array(G) * dt
    ref = _uniform(rho, ve, p)
    assert np.abs(Un - ref).max() < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("order", [2, 3, 4])
def test_linear_damping_local_error_order(order, form):
    # S = -kappa u on a state at rest (uniform fluxes): one step must agree
    # with exp(-kappa dt) to O(dt^(M+1)); a wrong coefficient anywhere in the
    # source modes, the evolution terms or the average lowers the order
    kappa = 1.0
    cfg = OracleConfig(order=order, form=form, riemann='hll', source=lambda u: -kappa * u)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        U = _uniform(1.0, [0.0, 0.0, 0.0], 1.0, shape=(3, 3, 3))
        errs.append(abs(step(U, dt, cfg)[0, 0, 0, 0] - np.exp(-kappa * dt)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > order + 1 - 0.2, (errs, rates)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_zero_source_is_the_plain_step(order):
    U = _density_wave(6, 0.0)
    plain = OracleConfig(order=order, riemann='hll')
    zero = OracleConfig(order=order, riemann='hll', source=lambda u: np.zeros_like(u))
    dt = compute_dt(U, plain, 0.3)
    assert np.array_equal(step(U, dt, zero), step(U, dt, plain))


@pytest.mark.slow
@pytest.mark.parametrize("order,sizes,T", [(2, (16, 32), 0.02), (3, (8, 16), 0.05),
                                           (4, (8, 16), 0.05)])
def test_gravity_design_order_density_wave(order, sizes, T):
    # the density wave under uniform gravity: v and p stay uniform, and the
    # profile moves by v t + g t^2 / 2, i.e. the plain wave at the time
    # t' = t + (gx + gy + gz) t^2 / 6 along its diagonal phase
    cfg = OracleConfig(order=order, riemann='hll', source=gravity_source(G))
    t_eff = T + sum(G) * T * T / 6.0
    errs = []
    for n in sizes:
        U = _density_wave(n, 0.0)
        t = 0.0
        while t < T - 1e-14:
            dt = min(compute_dt(U, cfg, 0.3), T - t)
            U = step(U, dt, cfg)
            t += dt
        errs.append(np.abs(U[0] - _density_wave(n, t_eff)[0]).mean())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.6, (errs, rate)
