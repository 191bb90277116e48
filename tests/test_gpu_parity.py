"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  FP64 bar, per conserved variable and per step (each
step compared from the GPU's own previous state): relative L1 <= 1e-12,
element-wise max |U_gpu - U_oracle| <= 1e-12 max |U|, and the step's
increment U^{n+1} - U^n within 1e-10 relative L1 where it is not tiny.

Positivity: the default (check) mode is the paper's scheme; where a check
point has rho <= 0 or P <= 0 the oracle raises NonPhysical and the library
must report ADER_ESTATE at the same step.  The limit mode (opt-in scaling)
is tested against the oracle's limit mode."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt as oracle_dt, step as oracle_step, step_block
from oracle.positivity import NonPhysical
from paper_1006_2146_amd import ader, workloads

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12

RS = {"hll": ader.ADER_HLL, "linearized": ader.ADER_LINEARIZED}
FORM = {"modal": ader.ADER_MODAL, "nodal": ader.ADER_NODAL}

CASES = [(2, "modal", "hll"), (2, "nodal", "hll"), (2, "modal", "linearized"),
         (3, "modal", "hll"), (3, "modal", "linearized"), (3, "nodal", "hll"),
         (3, "nodal", "linearized"), (4, "modal", "hll"), (4, "modal", "linearized"),
         (4, "nodal", "hll")]


def rel_l1(a, b):
    num = np.abs(a - b).sum(axis=(1, 2, 3))
    den = np.abs(b).sum(axis=(1, 2, 3))
    return num / den


def parity(got, ref, prev=None, tol=TOL_FP64):
    """The FP64 bar: per-variable relative L1 and element-wise max error
    within tol (the max against each variable's max |U|, floored at tol of
    the largest variable's, for variables that vanish), and, given the
    previous state, the increment within 1e-10 relative L1 wherever it is
    at least 1e-6 of the state."""
    err = rel_l1(got, ref)
    amax = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)
    scale = np.maximum(amax, tol * amax.max())
    mx = np.abs(got - ref).reshape(ref.shape[0], -1).max(axis=1) / scale
    ok = np.all(err <= tol) and np.all(mx <= tol)
    inc = None
    if prev is not None:
        d_ref = ref - prev
        size = np.abs(d_ref).sum(axis=(1, 2, 3))
        big = size >= 1e-6 * np.abs(ref).sum(axis=(1, 2, 3))
        inc = np.abs((got - prev) - d_ref).sum(axis=(1, 2, 3)) / np.maximum(size, 1e-300)
        ok = ok and np.all(inc[big] <= 1e-10)
    return bool(ok), (err, mx, inc)


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _solver(shape, order, form, rs, lengths=(1.0, 1.0, 1.0), precision=ader.ADER_FP64,
            positivity="check"):
    return ader.Solver(shape, lengths=lengths, order=order, form=FORM[form], riemann=RS[rs],
                       precision=precision, positivity=POS[positivity])


POS = {"check": ader.ADER_POSITIVITY_CHECK, "limit": ader.ADER_POSITIVITY_LIMIT}


def gpu_flagged(s):
    """Wait for the solver's queued work: True if it reported ADER_ESTATE
    (a non-positive check point in the check mode)."""
    try:
        s.synchronize()
    except ader.AderError as e:
        if e.code != ader.ADER_ESTATE:
            raise
        return True
    return False


def oracle_or_none(fn):
    try:
        return fn()
    except NonPhysical:
        return None


def _check_steps(U0, order, form, rs, nsteps, cfl=0.3, lengths=(1.0, 1.0, 1.0), tag="",
                 positivity="check"):
    """Steps GPU and oracle; returns the number of steps both took (fewer
    than nsteps where both found a non-positive check point)."""
    shape = U0.shape[1:]
    cfg = OracleConfig(order=order, form=form, riemann=rs, lengths=lengths,
                       positivity=positivity)
    with _solver(shape, order, form, rs, lengths, positivity=positivity) as s:
        s.set_state(U0)
        U = U0
        for it in range(nsteps):
            say(tag, "order", order, form, rs, positivity, "shape", shape, "step", it)
            dt_gpu = s.compute_dt(cfl)
            dt_ref = oracle_dt(U, cfg, cfl)
            assert abs(dt_gpu - dt_ref) <= 1e-14 * dt_ref
            s.step(dt_gpu)
            flagged = gpu_flagged(s)
            Uo = oracle_or_none(lambda: oracle_step(U, dt_gpu, cfg))
            assert flagged == (Uo is None), (it, "GPU flag", flagged, "oracle raised", Uo is None)
            if flagged:
                return it
            Ug = s.get_state()
            ok, err = parity(Ug, Uo, U)
            assert ok, (it, err)
            U = Ug
    return nsteps


@pytest.mark.parametrize("order,form,rs", CASES)
def test_parity_smooth_ragged(order, form, rs):
    U0 = workloads.random_smooth((9, 14, 21), seed=order)
    _check_steps(U0, order, form, rs, 2, lengths=(1.0, 0.8, 1.3), tag="smooth")


@pytest.mark.parametrize("positivity", ["check", "limit"])
@pytest.mark.parametrize("order,form,rs", CASES)
def test_parity_blast_positivity(order, form, rs, positivity):
    # 1000:1 blast: the paper's scheme (check mode) meets P <= 0 at check
    # points within three steps and both sides report it at the same step;
    # in the limit mode the scaling is active in many zones
    U0 = workloads.blast((12, 12, 12), p_in=100.0, p_out=0.1, radius=0.25)
    n = _check_steps(U0, order, form, rs, 3, tag="blast", positivity=positivity)
    assert (n < 3) if positivity == "check" else (n == 3)


@pytest.mark.parametrize("order,form,rs", CASES)
def test_limit_mode_inactive_is_check_mode(order, form, rs):
    # where the scaling does not act, the limit mode is bit-identical to the
    # paper's scheme; on the blast it counts the zones it scales
    U0 = workloads.random_smooth((9, 14, 21), seed=order + 40)
    out = {}
    for pos in ("check", "limit"):
        say("limit-inactive", order, form, rs, pos)
        with _solver(U0.shape[1:], order, form, rs, positivity=pos) as s:
            s.set_state(U0)
            s.step(0.2 * s.compute_dt(0.3))
            assert not gpu_flagged(s)
            out[pos] = s.get_state()
            assert s.limited_zones() == 0
    assert np.array_equal(out["check"], out["limit"])
    with _solver((12, 12, 12), order, form, rs, positivity="limit") as s:
        s.set_state(workloads.blast((12, 12, 12), p_in=100.0, p_out=0.1, radius=0.25))
        for _ in range(3):      # the paper's scheme meets P <= 0 within three steps
            s.step_cfl(0.3)
        assert not gpu_flagged(s)
        assert s.limited_zones() > 0
        assert s.limited_zones() == 0    # read and restarted


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 1), (3, 1, 2), (1, 5, 4)])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_parity_degenerate_meshes(shape, order):
    U0 = workloads.random_smooth(shape, seed=3)
    _check_steps(U0, order, "modal", "hll", 1, tag="tiny")


def test_constant_state_bitwise():
    U0 = np.zeros((5, 6, 7, 9))
    U0[:] = np.array([1.3, 0.2, -0.1, 0.3, 2.5])[:, None, None, None]
    for order in (2, 3, 4):
        for rs in ("hll", "linearized"):
            say("constant", order, rs)
            with _solver((6, 7, 9), order, "modal", rs) as s:
                s.set_state(U0)
                s.step(0.01)
                assert np.array_equal(s.get_state(), U0)


def test_conservation_and_translation():
    for order in (2, 3, 4):
        U0 = workloads.random_smooth((10, 9, 8), seed=11)
        say("conservation", order)
        with _solver((10, 9, 8), order, "modal", "linearized") as s:
            s.set_state(U0)
            for _ in range(3):
                s.step_cfl(0.3)
            U = s.get_state()
            tot0, tot1 = U0.sum(axis=(1, 2, 3)), U.sum(axis=(1, 2, 3))
            assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(U0).sum(axis=(1, 2, 3)))
        # exact translation by one zone at unit Courant number (linearized)
        rng = np.random.default_rng(order)
        n = (6, 5, 8)
        rho = rng.uniform(0.8, 1.2, size=n)
        U0 = np.zeros((5,) + n)
        U0[0] = rho
        U0[1] = 4.0 * rho
        U0[4] = 0.01 / 0.4 + 0.5 * 16.0 * rho
        say("translation", order)
        with _solver(n, order, "modal", "linearized") as s:
            s.set_state(U0)
            s.step((1.0 / 8) / 4.0)
            assert np.allclose(s.get_state()[0], np.roll(rho, 1, axis=2), rtol=0, atol=1e-9)


def test_config1_density_wave_full():
    # 32^3, order 2 nodal, minmod, HLL, CFL 0.4, 10 steps, parity every step
    U0 = workloads.density_wave((32, 32, 32))
    _check_steps(U0, 2, "nodal", "hll", 10, cfl=0.4, tag="config1")


@pytest.mark.parametrize("rs", ["hll", "linearized"])
def test_config2_full_size_sampled(rs):
    # 128^3 Sedov-mode workload, order 3 modal, one CFL 0.3 step on the GPU;
    # the oracle recomputes sampled blocks (two around the blast centre).
    # The 100:1 overpressure sphere puts P <= 0 at check points of the first
    # reconstruction: the paper's scheme (check mode) is undefined there and
    # both sides say so; the workload runs in the limit mode.
    shape = (128, 128, 128)
    U0 = workloads.sedov_modes(shape)
    centre_zone = tuple(int(c) for c in np.argwhere(U0[4] == U0[4].max())[0])
    near = tuple((c - 6) % 128 for c in centre_zone)
    with _solver(shape, 3, "modal", rs) as s:
        s.set_state(U0)
        say("config2", rs, "check mode step_cfl")
        s.step_cfl(0.3)
        assert gpu_flagged(s)
        dt = s.dt()
    with pytest.raises(NonPhysical):
        step_block(U0, dt, OracleConfig(order=3, riemann=rs), near, (12, 12, 12))
    cfg = OracleConfig(order=3, riemann=rs, positivity="limit")
    with _solver(shape, 3, "modal", rs, positivity="limit") as s:
        s.set_state(U0)
        say("config2", rs, "limit mode step_cfl")
        s.step_cfl(0.3)
        assert not gpu_flagged(s)
        Ug = s.get_state()
        dt = s.dt()
        assert s.limited_zones() > 0
    assert abs(dt - oracle_dt(U0, cfg, 0.3)) <= 1e-14 * dt
    origins = [(0, 0, 0), (125, 3, 64), (60, 127, 17),
               tuple((c - 2) % 128 for c in centre_zone), near]
    for o in origins:
        b = 12 if o == near else 4
        ref = step_block(U0, dt, cfg, o, (b, b, b))
        iz = np.arange(o[0], o[0] + b) % 128
        iy = np.arange(o[1], o[1] + b) % 128
        ix = np.arange(o[2], o[2] + b) % 128
        got = Ug[:, iz][:, :, iy][:, :, :, ix]
        ok, err = parity(got, ref)
        assert ok, (o, err)


# ----------------------------------------------------------------- MHD ------

G53 = 5.0 / 3.0
MHD_CASES = [(2, "modal"), (2, "nodal"), (3, "modal"), (3, "nodal"), (4, "modal"), (4, "nodal")]


def _mhd_solver(shape, order, form, lengths=(1.0, 1.0, 1.0), precision=ader.ADER_FP64, rs="hll",
                positivity="check"):
    return ader.Solver(shape, lengths=lengths, gamma=G53, order=order, form=FORM[form],
                       riemann=RS[rs], precision=precision, system=ader.ADER_MHD,
                       positivity=POS[positivity])


# The small random-field meshes resolve their k <= 4 modes poorly: at P = 0.1
# the paper's scheme (check mode) meets P <= 0 at check points, so it runs
# at P = 1, and the limit mode (whose scaling then acts) at P = 0.1.
MHD_MODES = [("check", 1.0), ("limit", 0.1)]


def _check_steps_mhd(U0, B0, order, form, nsteps, cfl=0.3, lengths=(1.0, 1.0, 1.0), tag="",
                     rs="hll", positivity="check"):
    shape = U0.shape[1:]
    cfg = OracleConfig(order=order, form=form, gamma=G53, lengths=lengths, riemann=rs,
                       positivity=positivity)
    with _mhd_solver(shape, order, form, lengths, rs=rs, positivity=positivity) as s:
        s.set_state(U0, B0)
        U, B = U0, B0
        for it in range(nsteps):
            say(tag, "mhd order", order, form, rs, positivity, "shape", shape, "step", it)
            dt_gpu = s.compute_dt(cfl)
            assert abs(dt_gpu - oracle_dt(U, cfg, cfl, B)) <= 1e-14 * dt_gpu
            s.step(dt_gpu)
            assert not gpu_flagged(s)
            Ug, Bg = s.get_state()
            Uo, Bo = oracle_step(U, dt_gpu, cfg, B)
            ok, err = parity(Ug, Uo, U)
            okb, errb = parity(Bg, Bo, B)
            assert ok and okb, (it, err, errb)
            U, B = Ug, Bg
    return U, B


@pytest.mark.parametrize("positivity,p0", MHD_MODES)
@pytest.mark.parametrize("rs", ["hll", "linearized"])
@pytest.mark.parametrize("order,form", MHD_CASES)
def test_parity_mhd_random_field_ragged(order, form, rs, positivity, p0):
    U0, B0 = workloads.mhd_random_field((7, 9, 10), seed=order, p0=p0)
    _check_steps_mhd(U0, B0, order, form, 2, lengths=(1.0, 0.9, 1.2), tag="mhd-random", rs=rs,
                     positivity=positivity)


@pytest.mark.parametrize("rs", ["hll", "linearized"])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_parity_mhd_alfven_and_div_b(order, rs):
    from oracle.bweno import divergence
    U0, B0 = workloads.alfven_wave_diagonal((8, 8, 8))
    U, B = _check_steps_mhd(U0, B0, order, "modal", 3, tag="mhd-alfven", rs=rs)
    dx = (1.0 / 8,) * 3
    assert np.abs(divergence(B, dx)).max() <= 1e-12 * np.abs(B).max() / dx[0]
    assert np.all(np.abs(U.sum(axis=(1, 2, 3)) - U0.sum(axis=(1, 2, 3))) <= 1e-13 * np.abs(U0).sum())


@pytest.mark.parametrize("positivity,p0", MHD_MODES)
def test_mhd_linearized_layouts(positivity, p0):
    # the linearized MHD flux in every layout that carries full edge states
    U0, B0 = workloads.mhd_random_field((6, 7, 8), seed=31, p0=p0)
    cfg = OracleConfig(order=3, gamma=G53, riemann="linearized", positivity=positivity)
    for layout in (ader.ADER_LAYOUT_ZONE, ader.ADER_LAYOUT_SPLIT, ader.ADER_LAYOUT_SPLIT2,
                   ader.ADER_LAYOUT_PAIR, ader.ADER_LAYOUT_PAIR2, ader.ADER_LAYOUT_PAIR_SPLIT):
        with _mhd_solver((6, 7, 8), 3, "modal", rs="linearized", positivity=positivity) as s:
            ader.ader_set_layout(s.ctx, layout)
            s.set_state(U0, B0)
            say("mhd linearized layout", layout, positivity)
            dt = s.compute_dt(0.3)
            s.step(dt)
            assert not gpu_flagged(s)
            Ug, Bg = s.get_state()
        Uo, Bo = oracle_step(U0, dt, cfg, B0)
        ok, err = parity(Ug, Uo, U0)
        okb, errb = parity(Bg, Bo, B0)
        assert ok and okb, (layout, err, errb)


def test_config3_mhd_full_size_sampled():
    # 128^3 MHD, order 4, HLL, CT: one CFL 0.3 step on the GPU, sampled blocks
    # recomputed by the oracle
    shape = (128, 128, 128)
    U0, B0 = workloads.mhd_random_field(shape)
    cfg = OracleConfig(order=4, gamma=G53)
    with _mhd_solver(shape, 4, "modal") as s:
        s.set_state(U0, B0)
        say("config3", "step_cfl")
        s.step_cfl(0.3)
        assert not gpu_flagged(s)
        Ug, Bg = s.get_state()
        dt = s.dt()
    assert abs(dt - oracle_dt(U0, cfg, 0.3, B0)) <= 1e-14 * dt
    for o in [(0, 0, 0), (100, 37, 127), (64, 64, 64)]:
        Ur, Br = step_block(U0, dt, cfg, o, (3, 3, 3), B0)
        iz = np.arange(o[0], o[0] + 3) % 128
        iy = np.arange(o[1], o[1] + 3) % 128
        ix = np.arange(o[2], o[2] + 3) % 128
        pick = lambda A: A[:, iz][:, :, iy][:, :, :, ix]  # noqa: E731
        ok, err = parity(pick(Ug), Ur)
        okb, errb = parity(pick(Bg), Br)
        assert ok and okb, (o, err, errb)


# --------------------------------------------------------- predictor layouts --

LAYOUTS = [ader.ADER_LAYOUT_ZONE, ader.ADER_LAYOUT_SPLIT, ader.ADER_LAYOUT_SPLIT2,
           ader.ADER_LAYOUT_ZONE2, ader.ADER_LAYOUT_ZONE_2W, ader.ADER_LAYOUT_PAIR,
           ader.ADER_LAYOUT_PAIR2, ader.ADER_LAYOUT_PAIR_SPLIT, ader.ADER_LAYOUT_FUSED]


def _skip_unbuilt(layout, order, mhd=False):
    if layout == ader.ADER_LAYOUT_ZONE and order == 4 and not mhd:
        pytest.skip("the Euler one-lane-per-zone predictor is not built in FP64 at order 4 (a "
                    "run of it did not finish, cause not found); the lane-split layout runs "
                    "there")
    if layout == ader.ADER_LAYOUT_FUSED and (order != 3 or mhd):
        pytest.skip("the fused reconstruction+predictor is built for Euler at order 3")
    if layout == ader.ADER_LAYOUT_ZONE2 and order > 3:
        pytest.skip("the one-lane-per-zone instance with its own facial pass is built for "
                    "orders 2 and 3")
    if layout == ader.ADER_LAYOUT_ZONE_2W and (order > 3 or mhd):
        pytest.skip("the two-wave one-lane-per-zone instance is built for Euler at orders 2-3")
    if layout in (ader.ADER_LAYOUT_PAIR, ader.ADER_LAYOUT_PAIR2, ader.ADER_LAYOUT_PAIR_SPLIT) \
            and (order < 3 or not mhd):
        pytest.skip("the pair layout is built for MHD at orders 3-4")
    if layout in (ader.ADER_LAYOUT_PAIR, ader.ADER_LAYOUT_PAIR2) and order == 4:
        pytest.skip("the one-kernel pair layout is switched off at order 4 (wrong results "
                    "in the modal form, cause not found); the two-kernel form is used")


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("order,rs", [(3, "hll"), (4, "linearized")])
def test_parity_layouts_euler(layout, order, rs):
    _skip_unbuilt(layout, order)
    # every predictor layout against the oracle: smooth ragged mesh (check
    # mode), a blast in the limit mode (the scaling and its exact pass
    # active) and the same blast in the check mode (reported at the same
    # step by both sides)
    blast = workloads.blast((12, 12, 12), p_in=100.0, p_out=0.1, radius=0.25)
    for tag, U0, lengths, steps, pos in (
            ("smooth", workloads.random_smooth((9, 14, 21), seed=order + 7), (1.0, 0.8, 1.3), 2,
             "check"),
            ("blast", blast, (1.0, 1.0, 1.0), 2, "limit"),
            ("blast", blast, (1.0, 1.0, 1.0), 3, "check")):
        cfg = OracleConfig(order=order, riemann=rs, lengths=lengths, positivity=pos)
        with _solver(U0.shape[1:], order, "modal", rs, lengths, positivity=pos) as s:
            ader.ader_set_layout(s.ctx, layout)
            assert ader.ader_get_layout(s.ctx) == layout
            s.set_state(U0)
            U = U0
            for it in range(steps):
                say("layout", layout, tag, pos, order, rs, "step", it)
                dt = s.compute_dt(0.3)
                s.step(dt)
                flagged = gpu_flagged(s)
                Uo = oracle_or_none(lambda: oracle_step(U, dt, cfg))
                assert flagged == (Uo is None), (tag, pos, it)
                if flagged:
                    break
                Ug = s.get_state()
                ok, err = parity(Ug, Uo, U)
                assert ok, (tag, pos, it, err)
                U = Ug


@pytest.mark.parametrize("positivity,p0", MHD_MODES)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("order", [3, 4])
def test_parity_layouts_mhd(layout, order, positivity, p0):
    _skip_unbuilt(layout, order, mhd=True)
    U0, B0 = workloads.mhd_random_field((7, 9, 10), seed=order + 20, p0=p0)
    cfg = OracleConfig(order=order, gamma=G53, lengths=(1.0, 0.9, 1.2), positivity=positivity)
    with _mhd_solver((7, 9, 10), order, "modal", lengths=(1.0, 0.9, 1.2),
                     positivity=positivity) as s:
        ader.ader_set_layout(s.ctx, layout)
        s.set_state(U0, B0)
        U, B = U0, B0
        for it in range(2):
            say("mhd layout", layout, order, positivity, "step", it)
            dt = s.compute_dt(0.3)
            s.step(dt)
            assert not gpu_flagged(s)
            Ug, Bg = s.get_state()
            Uo, Bo = oracle_step(U, dt, cfg, B)
            ok, err = parity(Ug, Uo, U)
            okb, errb = parity(Bg, Bo, B)
            assert ok and okb, (it, err, errb)
            U, B = Ug, Bg


def test_layout_errors():
    with _solver((4, 4, 4), 2, "modal", "hll") as s:
        assert ader.load().ader_set_layout(s.ctx, ader.ADER_LAYOUT_SPLIT) == ader.ADER_EUNSUPPORTED
        assert ader.load().ader_set_layout(s.ctx, 9) == ader.ADER_EINVAL
        assert ader.ader_get_layout(s.ctx) == ader.ADER_LAYOUT_ZONE
        ader.ader_set_layout(s.ctx, ader.ADER_LAYOUT_ZONE2)
        assert ader.ader_get_layout(s.ctx) == ader.ADER_LAYOUT_ZONE2
    with _solver((4, 4, 4), 4, "modal", "hll") as s:
        assert ader.load().ader_set_layout(s.ctx, ader.ADER_LAYOUT_ZONE2) == ader.ADER_EUNSUPPORTED
        assert ader.load().ader_set_layout(s.ctx, ader.ADER_LAYOUT_ZONE) == ader.ADER_EUNSUPPORTED
        assert ader.ader_get_layout(s.ctx) == ader.ADER_LAYOUT_SPLIT
        assert ader.load().ader_set_layout(s.ctx, ader.ADER_LAYOUT_ZONE_2W) == \
            ader.ADER_EUNSUPPORTED
    with _mhd_solver((4, 4, 4), 3, "modal") as s:
        assert ader.load().ader_set_layout(s.ctx, ader.ADER_LAYOUT_ZONE_2W) == \
            ader.ADER_EUNSUPPORTED
        assert ader.ader_get_layout(s.ctx) == ader.ADER_LAYOUT_PAIR
    with _mhd_solver((4, 4, 4), 4, "modal") as s:
        for lay in (ader.ADER_LAYOUT_PAIR, ader.ADER_LAYOUT_PAIR2):
            assert ader.load().ader_set_layout(s.ctx, lay) == ader.ADER_EUNSUPPORTED
        assert ader.ader_get_layout(s.ctx) == ader.ADER_LAYOUT_PAIR_SPLIT


# ----------------------------------------- turbulent MHD, linearized, order 4 --

def test_turbulent_mhd_linearized_order4_parity():
    # the turbulent-like MHD workload (64-mode k^-5/3 velocity and vector
    # potential, rms Mach 1) at a size the oracle steps whole.  Its k <= 8
    # modes on 10..14 zones take the paper's scheme to P <= 0 at check points:
    # both sides flag that in the check mode, and step it in the limit mode.
    U0, B0 = workloads.turbulent_mhd((10, 12, 14), seed=7)
    cfg = OracleConfig(order=4, gamma=G53, riemann="linearized")
    dt = oracle_dt(U0, cfg, 0.3, B0)
    with pytest.raises(NonPhysical):
        oracle_step(U0, dt, cfg, B0)
    with _mhd_solver(U0.shape[1:], 4, "modal", rs="linearized") as s:
        s.set_state(U0, B0)
        say("turbulent mhd order 4 check mode")
        s.step(s.compute_dt(0.3))
        assert gpu_flagged(s)
    _check_steps_mhd(U0, B0, 4, "modal", 2, tag="turbulent", rs="linearized", positivity="limit")


def test_config5_turbulent_mhd_384_mixed():
    # 384^3 MHD, order 4, linearized flux, CT, FP32 bulk with FP64 update: one
    # CFL step on the GPU; sampled blocks against the FP64 oracle at the
    # mixed path's per-step accuracy, div B at round-off over the whole mesh,
    # conserved totals, and the device memory within one GPU
    from oracle.bweno import divergence
    shape = (384, 384, 384)
    say("config5 generate")
    U0, B0 = workloads.turbulent_mhd(shape)
    cfg = OracleConfig(order=4, gamma=G53, riemann="linearized")
    with _mhd_solver(shape, 4, "modal", precision=ader.ADER_MIXED, rs="linearized") as s:
        s.set_state(U0, B0)
        say("config5 step")
        s.step_cfl(0.3)
        assert not gpu_flagged(s)
        Ug, Bg = s.get_state()
        dt = s.dt()
        assert ader.ader_device_bytes(s.ctx) < 200e9
    assert abs(dt - oracle_dt(U0, cfg, 0.3, B0)) <= 1e-14 * dt
    dx = (1.0 / 384,) * 3
    assert np.abs(divergence(Bg, dx)).max() <= 1e-12 * np.abs(Bg).max() / dx[0]
    tot0, tot1 = U0.sum(axis=(1, 2, 3)), Ug.sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot1 - tot0) <= 1e-12 * np.abs(U0).sum(axis=(1, 2, 3)))
    for o in [(0, 0, 0), (200, 383, 17)]:
        say("config5 oracle block", o)
        Ur, Br = step_block(U0, dt, cfg, o, (2, 2, 2), B0)
        iz = np.arange(o[0], o[0] + 2) % 384
        iy = np.arange(o[1], o[1] + 2) % 384
        ix = np.arange(o[2], o[2] + 2) % 384
        pick = lambda A: A[:, iz][:, :, iy][:, :, :, ix]  # noqa: E731
        # FP32 bulk: the step's change is resolved to ~1e-6 relative
        assert np.all(rel_l1(pick(Ug), Ur) <= 1e-6), o
        assert np.all(rel_l1(pick(Bg), Br) <= 1e-6), o
