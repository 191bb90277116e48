"""CPU parity of the kernel source (host build of the per-zone kernel code)
against the oracle: the same FP64 bar as the GPU parity tests, so logic
errors in the generated scheme code or the kernels show up before any GPU
run.  Each FP64 case runs in both forms: the point form of the FP64 path and
the deviation form of the mixed path evaluated in double, which checks the
deviation algebra exactly (its FP32 accuracy is tested separately)."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt as oracle_dt, step as oracle_step
from paper_1006_2146_amd import workloads
from tests import hostemu

CASES = [(2, "modal", "hll"), (2, "nodal", "hll"), (2, "modal", "linearized"),
         (3, "modal", "hll"), (3, "modal", "linearized"), (3, "nodal", "hll"),
         (3, "nodal", "linearized"), (4, "modal", "hll"), (4, "modal", "linearized"),
         (4, "nodal", "hll")]


def rel_l1(a, b):
    return np.abs(a - b).sum(axis=(1, 2, 3)) / np.abs(b).sum(axis=(1, 2, 3))


@pytest.fixture(scope="module", autouse=True)
def _built():
    hostemu.load()


def _steps(U0, order, form, rs, nsteps, lengths=(1.0, 1.0, 1.0), cfl=0.3, precision="fp64"):
    cfg = OracleConfig(order=order, form=form, riemann=rs, lengths=lengths)
    U = U0
    for it in range(nsteps):
        dt = hostemu.compute_dt(U, cfl, lengths)
        assert abs(dt - oracle_dt(U, cfg, cfl)) <= 1e-14 * dt
        Ue = hostemu.step(U, dt, order, form, rs, precision=precision, lengths=lengths)
        Uo = oracle_step(U, dt, cfg)
        err = rel_l1(Ue, Uo)
        assert np.all(err <= 1e-12), (it, err)
        U = Ue
    return U


FORMS = ["fp64", "fp64dev"]


@pytest.mark.parametrize("precision", FORMS)
@pytest.mark.parametrize("order,form,rs", CASES)
def test_kernel_source_smooth(order, form, rs, precision):
    _steps(workloads.random_smooth((7, 9, 11), seed=order), order, form, rs, 2,
           lengths=(1.0, 0.8, 1.3), precision=precision)


@pytest.mark.parametrize("precision", FORMS)
@pytest.mark.parametrize("order,form,rs", CASES)
def test_kernel_source_blast(order, form, rs, precision):
    _steps(workloads.blast((10, 10, 10), p_in=100.0, p_out=0.1, radius=0.25), order, form, rs, 3,
           precision=precision)


@pytest.mark.parametrize("precision", FORMS)
@pytest.mark.parametrize("order", [2, 3, 4])
def test_kernel_source_tiny_meshes(order, precision):
    for shape in [(1, 1, 1), (2, 3, 1), (3, 1, 2)]:
        _steps(workloads.random_smooth(shape, seed=3), order, "modal", "hll", 1, precision=precision)


MHD_CASES = [(2, "modal"), (2, "nodal"), (3, "modal"), (3, "nodal"), (4, "modal"), (4, "nodal")]


def _steps_mhd(U0, B0, order, form, nsteps, lengths=(1.0, 1.0, 1.0), cfl=0.3, precision="fp64",
               rs="hll"):
    cfg = OracleConfig(order=order, form=form, gamma=5.0 / 3.0, lengths=lengths, riemann=rs)
    U, B = U0, B0
    for it in range(nsteps):
        dt = hostemu.compute_dt_mhd(U, B, cfl, lengths)
        assert abs(dt - oracle_dt(U, cfg, cfl, B)) <= 1e-14 * dt
        Ue, Be = hostemu.step_mhd(U, B, dt, order, form, precision=precision, lengths=lengths,
                                  riemann=rs)
        Uo, Bo = oracle_step(U, dt, cfg, B)
        err = rel_l1(Ue, Uo)
        errb = rel_l1(Be, Bo)
        assert np.all(err <= 1e-12) and np.all(errb <= 1e-12), (it, err, errb)
        U, B = Ue, Be
    return U, B


@pytest.mark.parametrize("rs", ["hll", "linearized"])
@pytest.mark.parametrize("precision", FORMS)
@pytest.mark.parametrize("order,form", MHD_CASES)
def test_kernel_source_mhd_random_field(order, form, precision, rs):
    U0, B0 = workloads.mhd_random_field((6, 7, 8), seed=order)
    _steps_mhd(U0, B0, order, form, 2, lengths=(1.0, 0.9, 1.2), precision=precision, rs=rs)


@pytest.mark.parametrize("rs", ["hll", "linearized"])
@pytest.mark.parametrize("precision", FORMS)
@pytest.mark.parametrize("order", [2, 3, 4])
def test_kernel_source_mhd_alfven(order, precision, rs):
    U0, B0 = workloads.alfven_wave_diagonal((6, 6, 6))
    _steps_mhd(U0, B0, order, "modal", 2, precision=precision, rs=rs)


def test_kernel_source_mhd_eigensystem():
    # the kernel source's analytic eigen-system (Roe-Balsara vectors) against
    # the oracle's |A| from its definition, on random face pairs and axes
    from oracle.physics import conserved
    from oracle.riemann import mhd_abs_jacobian, mhd_dissipation
    rng = np.random.default_rng(3)
    G = 5.0 / 3.0

    def state():
        return conserved(rng.uniform(0.5, 2.0), rng.normal(0, 0.5, 3), rng.uniform(0.5, 2.0),
                         rng.normal(0, 2.0, 3), G)
    for _ in range(30):
        ul, ur = state(), state()
        du = rng.normal(0, 1, 8)
        for axis in range(3):
            Do = mhd_dissipation(mhd_abs_jacobian(ul[:, None], ur[:, None], axis, G),
                                 du[:, None], axis)[:, 0]
            Dk = hostemu.mhd_dissipation(ul, ur, du, axis, G)
            assert np.abs(Dk - Do).max() <= 1e-12 * np.abs(Do).max()


# ------------------------------------------------ SSP-RK (Sec. II.d), Euler --

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp64dev", 1e-12), ("mixed", 1e-7)])
@pytest.mark.parametrize("rs", ["hll", "linearized"])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_kernel_source_rk(order, rs, precision, tol):
    # the RK side-packet and stage-combination kernels, built for the host,
    # against the oracle's SSP-RK steps (a smooth ragged mesh, then a blast
    # where the positivity scaling acts)
    from oracle import rk as ork
    for U0, lengths in ((workloads.random_smooth((7, 9, 11), seed=order + 5), (1.0, 0.8, 1.3)),
                        (workloads.blast((8, 8, 8), p_in=100.0, p_out=0.1, radius=0.25),
                         (1.0, 1.0, 1.0))):
        cfg = OracleConfig(order=order, riemann=rs, lengths=lengths)
        U = U0
        for it in range(2):
            dt = hostemu.compute_dt(U, 0.3, lengths)
            Ue = hostemu.step_rk(U, dt, order, rs, precision=precision, lengths=lengths)
            err = rel_l1(Ue, ork.step_rk(U, dt, cfg))
            assert np.all(err <= tol), (it, err)
            U = Ue


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp64dev", 1e-12), ("mixed", 1e-6)])
@pytest.mark.parametrize("rs", ["hll", "linearized"])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_kernel_source_rk_mhd(order, rs, precision, tol):
    # the MHD RK side packets (the predictor kernel with the predictor
    # bypassed) and the stage combinations of U and of the face fields,
    # built for the host, against the oracle's MHD SSP-RK steps
    from oracle import rk as ork
    from oracle.bweno import divergence
    U0, B0 = workloads.mhd_random_field((6, 7, 8), seed=order + 70)
    cfg = OracleConfig(order=order, gamma=5.0 / 3.0, riemann=rs)
    U, B = U0, B0
    for it in range(2):
        dt = hostemu.compute_dt_mhd(U, B, 0.3)
        Ue, Be = hostemu.step_rk_mhd(U, B, dt, order, rs, precision=precision)
        Uo, Bo = ork.step_rk_mhd(U, B, dt, cfg)
        assert np.all(rel_l1(Ue, Uo) <= tol) and np.all(rel_l1(Be, Bo) <= tol), it
        dx = cfg.spacing(U.shape[1:])
        assert np.abs(divergence(Be, dx)).max() <= 1e-12 * np.abs(Be).max() / min(dx)
        U, B = Ue, Be
