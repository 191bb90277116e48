"""The affine source term of the Euler equations on the GPU through the C
ABI (ader_set_source) against the oracle's predictor with a source (Sec. IV:
source modes eq. 34, 43, 52; evolution eq. 30, 36, 45; space-time averages
eq. 35, 44, 53; App. A-C in the nodal form) and eq. (6) with dt S-bar: FP64
parity per step, the mixed path within its FP32 bound, the limit mode, a
batch against solo runs, graph replays, and the argument checks."""

import ctypes

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt as oracle_dt, step as oracle_step
from oracle.positivity import NonPhysical
from paper_1006_2146_amd import ader, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


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
ORDERS = [(2, "modal"), (2, "nodal"), (3, "modal"), (3, "nodal"), (4, "modal"), (4, "nodal")]
FORM = {"modal": ader.ADER_MODAL, "nodal": ader.ADER_NODAL}
POS = {"check": ader.ADER_POSITIVITY_CHECK, "limit": ader.ADER_POSITIVITY_LIMIT}


def oracle_fn(A, b):
    def source(u):
        return np.tensordot(A, u, axes=(1, 0)) + b.reshape((5,) + (1,) * (u.ndim - 1))
    return source


def close(a, b, tol=1e-12):
    err = np.abs(a - b).sum(axis=(1, 2, 3)) / np.abs(b).sum(axis=(1, 2, 3))
    mx = np.abs(a - b).reshape(5, -1).max(axis=1) / np.abs(b).reshape(5, -1).max(axis=1)
    return bool(np.all(err <= tol) and np.all(mx <= tol)), (err, mx)


def _steps(U0, order, form, name, nsteps, precision=ader.ADER_FP64, positivity="check",
           lengths=(1.0, 0.9, 1.2)):
    A, b = SOURCES[name]
    cfg = OracleConfig(order=order, form=form, riemann="hll", lengths=lengths,
                       source=oracle_fn(A, b), positivity=positivity)
    out = []
    with ader.Solver(U0.shape[1:], lengths=lengths, order=order, form=FORM[form],
                     precision=precision, positivity=POS[positivity]) as s:
        s.set_source(A, b)
        s.set_state(U0)
        U = U0
        for it in range(nsteps):
            say("source", name, order, form, precision, positivity, "step", it)
            dt = s.compute_dt(0.3)
            assert abs(dt - oracle_dt(U, cfg, 0.3)) <= 1e-14 * dt
            s.step(dt)
            s.synchronize()
            Ug = s.get_state()
            Uo = oracle_step(U, dt, cfg)
            out.append((Ug, Uo))
            U = Uo
            s.set_state(U)
    return out


@pytest.mark.parametrize("name", sorted(SOURCES))
@pytest.mark.parametrize("order,form", ORDERS)
def test_source_parity_fp64(order, form, name):
    U0 = workloads.random_smooth((7, 9, 10), seed=order + 3)
    for Ug, Uo in _steps(U0, order, form, name, 2):
        ok, err = close(Ug, Uo)
        assert ok, err


@pytest.mark.parametrize("order,form", ORDERS)
def test_source_mixed_within_fp32_bound(order, form):
    U0 = workloads.random_smooth((7, 9, 10), seed=order + 3)
    for Ug, Uo in _steps(U0, order, form, "affine", 1, precision=ader.ADER_MIXED):
        d = np.abs(Ug - Uo).reshape(5, -1).max(axis=1)
        assert np.all(d <= 2e-6 * np.abs(Uo).reshape(5, -1).max(axis=1)), d


@pytest.mark.parametrize("order,form", ORDERS)
def test_source_limit_mode_parity(order, form):
    # a blast where the limit mode's scaling acts, with a damping source
    U0 = workloads.blast((8, 8, 8), p_in=100.0, p_out=0.1, radius=0.25)
    for Ug, Uo in _steps(U0, order, form, "damping", 2, positivity="limit",
                         lengths=(1.0, 1.0, 1.0)):
        ok, err = close(Ug, Uo)
        assert ok, err


def test_source_check_mode_flags_like_the_oracle():
    # the paper's scheme meets P <= 0 at a check point in the second step
    # of this blast: both sides step the first and flag the second
    U0 = workloads.blast((10, 10, 10), p_in=100.0, p_out=0.1, radius=0.25)
    A, b = SOURCES["damping"]
    cfg = OracleConfig(order=3, riemann="hll", source=oracle_fn(A, b))
    dt0 = oracle_dt(U0, cfg, 0.3)
    U1 = oracle_step(U0, dt0, cfg)
    dt1 = oracle_dt(U1, cfg, 0.3)
    with pytest.raises(NonPhysical):
        oracle_step(U1, dt1, cfg)
    with ader.Solver((10, 10, 10), order=3) as s:
        s.set_source(A, b)
        s.set_state(U0)
        s.step(dt0)
        s.synchronize()
        ok, err = close(s.get_state(), U1)
        assert ok, err
        s.set_state(U1)
        s.step(dt1)
        with pytest.raises(ader.AderError) as e:
            s.synchronize()
        assert e.value.code == ader.ADER_ESTATE


def test_uniform_gravity_exact():
    # uniform state, uniform gravity: velocity + g dt and energy + m.g dt +
    # rho |g|^2 dt^2 / 2, exactly, at every order and form
    g = np.array([0.3, -0.2, 0.5])
    rho, v, p, gam = 1.3, np.array([0.2, -0.1, 0.3]), 2.0, 1.4
    U = np.zeros((5, 4, 5, 6))
    U[0] = rho
    U[1:4] = (rho * v)[:, None, None, None]
    U[4] = p / (gam - 1.0) + 0.5 * rho * v.dot(v)
    dt = 0.05
    ve = v + g * dt
    ref = U.copy()
    ref[1:4] = (rho * ve)[:, None, None, None]
    ref[4] = p / (gam - 1.0) + 0.5 * rho * ve.dot(ve)
    for order, form in ORDERS:
        for prec in (ader.ADER_FP64, ader.ADER_MIXED):
            say("gravity exact", order, form, prec)
            with ader.Solver((4, 5, 6), order=order, form=FORM[form], precision=prec) as s:
                s.set_source(*gravity(g))
                s.set_state(U)
                s.step(dt)
                out = s.get_state()
            tol = 1e-14 if prec == ader.ADER_FP64 else 1e-7
            assert np.abs(out - ref).max() < tol * np.abs(ref).max(), (order, form, prec)


def test_source_batch_equals_solo_and_graph_replays():
    # every problem of a batch takes the source; each equals its solo run
    # bitwise; graph replays equal eager steps, and a new source is taken up
    shapes = [(6, 7, 9), (8, 8, 8), (5, 9, 6)]
    states = [workloads.random_smooth(sh, seed=20 + q) for q, sh in enumerate(shapes)]
    A, b = SOURCES["affine"]
    A2, b2 = SOURCES["gravity"]
    import torch
    stream = torch.cuda.Stream()   # graph capture needs a stream of its own
    res = {}
    for graph in (False, True):
        with ader.BatchSolver(shapes, order=3, stream=stream.cuda_stream if graph else None) as bs:
            if graph:
                ader.ader_set_graph(bs.ctx, True)
            bs.set_source(A, b)
            for q, U in enumerate(states):
                bs.set_state(q, U)
            for _ in range(3):
                bs.step_cfl(0.3)
            bs.set_source(A2, b2)
            for _ in range(2):
                bs.step_cfl(0.3)
            res[graph] = [bs.get_state(q) for q in range(len(shapes))]
    for q in range(len(shapes)):
        assert np.array_equal(res[False][q], res[True][q]), q
    for q, (sh, U) in enumerate(zip(shapes, states)):
        say("solo", q)
        with ader.Solver(sh, order=3) as s:
            s.set_source(A, b)
            s.set_state(U)
            for _ in range(3):
                s.step_cfl(0.3)
            s.set_source(A2, b2)
            for _ in range(2):
                s.step_cfl(0.3)
            assert np.array_equal(s.get_state(), res[False][q]), q


def test_source_removed_equals_no_source():
    U0 = workloads.random_smooth((6, 6, 6), seed=2)
    outs = []
    for set_then_clear in (False, True):
        with ader.Solver((6, 6, 6), order=4) as s:
            if set_then_clear:
                s.set_source(*SOURCES["affine"])
                s.set_source(None)
            s.set_state(U0)
            s.step_cfl(0.3)
            outs.append(s.get_state())
    assert np.array_equal(outs[0], outs[1])


def test_source_errors():
    A, b = SOURCES["affine"]
    with ader.Solver((4, 4, 4), system=ader.ADER_MHD, gamma=5.0 / 3.0) as s:
        with pytest.raises(ader.AderError) as e:
            s.set_source(A, b)
        assert e.value.code == ader.ADER_EUNSUPPORTED
    with ader.Solver((4, 4, 4)) as s:
        bad = A.copy()
        bad[2, 3] = np.nan
        with pytest.raises(ader.AderError) as e:
            s.set_source(bad, b)
        assert e.value.code == ader.ADER_EINVAL
        lib = ader.load()
        bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        assert lib.ader_set_source(s.ctx, None, bp) == ader.ADER_EINVAL
        # the SSP-RK scheme has no source term
        s.set_source(A, b)
        s.set_state(workloads.random_smooth((4, 4, 4), seed=1))
        ader.ader_set_scheme(s.ctx, ader.ADER_SCHEME_SSPRK)
        with pytest.raises(ader.AderError) as e:
            s.step(1e-3)
        assert e.value.code == ader.ADER_EUNSUPPORTED
