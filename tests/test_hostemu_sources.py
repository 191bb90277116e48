"""CPU parity of the kernel source's affine source term (host build of the
per-zone code) against the oracle's predictor with a source (Sec. IV: the
source modes eq. 34, 43, 52 in the evolution eq. 30, 36, 45 and the
space-time averages eq. 35, 44, 53; App. A-C in the nodal form) and eq. (6)
with dt S-bar: uniform gravity, linear damping of the momentum, and a random
affine source, orders 2-4, both forms, FP64 point and deviation forms at the
FP64 bar, the mixed path within its FP32 bound."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt as oracle_dt, step as oracle_step
from paper_1006_2146_amd import workloads
from tests import hostemu
from tests.test_hostemu_parity import both, close


@pytest.fixture(scope="module", autouse=True)
def _built():
    hostemu.load()


def gravity(g):
    A = np.zeros((5, 5))
    A[1:4, 0] = g
    A[4, 1:4] = g
    return A, np.zeros(5)


def damping(k):
    A = np.zeros((5, 5))
    A[1, 1] = A[2, 2] = A[3, 3] = -k
    return A, np.zeros(5)


def random_affine(seed):
    rng = np.random.default_rng(seed)
    return 0.4 * rng.standard_normal((5, 5)), 0.2 * rng.standard_normal(5)


SOURCES = {"gravity": gravity((0.3, -0.2, 0.5)), "damping": damping(0.7),
           "affine": random_affine(11)}


def oracle_fn(A, b):
    def source(u):
        return np.tensordot(A, u, axes=(1, 0)) + b.reshape((5,) + (1,) * (u.ndim - 1))
    return source


def _run(U0, order, form, name, nsteps, precision, positivity="check"):
    A, b = SOURCES[name]
    cfg = OracleConfig(order=order, form=form, riemann="hll", source=oracle_fn(A, b),
                       positivity=positivity)
    U = U0
    out = []
    limited.clear()
    for _ in range(nsteps):
        dt = oracle_dt(U, cfg, 0.3)
        e, o = both(lambda: hostemu.step(U, dt, order, form, precision=precision,
                                         positivity=positivity, source=(A, b)),
                    lambda: oracle_step(U, dt, cfg))
        if e is None:
            break
        out.append((e, o))
        limited.append(hostemu.last_limited)
        U = o
    return out


limited = []   # scaled zone polynomials per step of the last _run (limit mode)

ORDERS = [(2, "modal"), (2, "nodal"), (3, "modal"), (3, "nodal"), (4, "modal"), (4, "nodal")]


@pytest.mark.parametrize("name", sorted(SOURCES))
@pytest.mark.parametrize("precision", ["fp64", "fp64dev"])
@pytest.mark.parametrize("order,form", ORDERS)
def test_source_parity(order, form, precision, name):
    U0 = workloads.random_smooth((5, 6, 7), seed=order + 3)
    pairs = _run(U0, order, form, name, 2, precision)
    assert len(pairs) == 2
    for e, o in pairs:
        ok, err = close(e, o)
        assert ok, err


@pytest.mark.parametrize("order,form", ORDERS)
def test_source_mixed_within_fp32_bound(order, form):
    # the mixed path's FP32 bulk: the step's change resolved to ~1e-6
    U0 = workloads.random_smooth((5, 6, 7), seed=order + 3)
    for e, o in _run(U0, order, form, "affine", 1, "mixed"):
        d = np.abs(e - o).reshape(5, -1).max(axis=1)
        assert np.all(d <= 2e-6 * np.abs(o).reshape(5, -1).max(axis=1)), d


@pytest.mark.parametrize("order,form", ORDERS)
def test_source_limit_mode_parity(order, form):
    # the limit mode where the scaling acts: a blast with a source
    U0 = workloads.blast((8, 8, 8), p_in=100.0, p_out=0.1, radius=0.25)
    pairs = _run(U0, order, form, "damping", 3, "fp64", positivity="limit")
    assert len(pairs) == 3
    for e, o in pairs:
        ok, err = close(e, o)
        assert ok, err
    assert sum(limited) > 0, limited


def test_uniform_gravity_exact_in_the_host_build():
    # a uniform state under uniform gravity changes by exactly the
    # quadratic in time of the exact solution (oracle pin restated for the
    # kernel code): velocity + g dt, energy + m.g dt + rho |g|^2 dt^2 / 2
    g = np.array([0.3, -0.2, 0.5])
    rho, v, p, gam = 1.3, np.array([0.2, -0.1, 0.3]), 2.0, 1.4
    U = np.zeros((5, 4, 5, 6))
    U[0] = rho
    U[1:4] = (rho * v)[:, None, None, None]
    U[4] = p / (gam - 1.0) + 0.5 * rho * v.dot(v)
    dt = 0.05
    for order, form in ORDERS:
        out = hostemu.step(U, dt, order, form, source=gravity(g))
        ve = v + g * dt
        ref = U.copy()
        ref[1:4] = (rho * ve)[:, None, None, None]
        ref[4] = p / (gam - 1.0) + 0.5 * rho * ve.dot(ve)
        assert np.abs(out - ref).max() < 1e-14 * np.abs(ref).max(), (order, form)
