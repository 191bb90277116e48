"""CPU parity of the kernel source (host build of ader_kernels.h) against the
oracle: the same FP64 bar as the GPU parity tests, so logic errors in the
generated scheme code or the kernels show up before any GPU run."""

import numpy as np
import pytest

from oracle import OracleConfig, compute_dt as oracle_dt, step as oracle_step
from paper_1006_2146_amd import workloads
from tests import hostemu

CASES = [(2, "modal", "hll"), (2, "nodal", "hll"), (2, "modal", "linearized"),
         (3, "modal", "hll"), (3, "modal", "linearized"),
         (4, "modal", "hll"), (4, "modal", "linearized")]


def rel_l1(a, b):
    return np.abs(a - b).sum(axis=(1, 2, 3)) / np.abs(b).sum(axis=(1, 2, 3))


@pytest.fixture(scope="module", autouse=True)
def _built():
    hostemu.load()


def _steps(U0, order, form, rs, nsteps, lengths=(1.0, 1.0, 1.0), cfl=0.3):
    cfg = OracleConfig(order=order, form=form, riemann=rs, lengths=lengths)
    U = U0
    for it in range(nsteps):
        dt = hostemu.compute_dt(U, cfl, lengths)
        assert abs(dt - oracle_dt(U, cfg, cfl)) <= 1e-14 * dt
        Ue = hostemu.step(U, dt, order, form, rs, lengths=lengths)
        Uo = oracle_step(U, dt, cfg)
        err = rel_l1(Ue, Uo)
        assert np.all(err <= 1e-12), (it, err)
        U = Ue
    return U


@pytest.mark.parametrize("order,form,rs", CASES)
def test_kernel_source_smooth(order, form, rs):
    _steps(workloads.random_smooth((7, 9, 11), seed=order), order, form, rs, 2,
           lengths=(1.0, 0.8, 1.3))


@pytest.mark.parametrize("order,form,rs", CASES)
def test_kernel_source_blast(order, form, rs):
    _steps(workloads.blast((10, 10, 10), p_in=100.0, p_out=0.1, radius=0.25), order, form, rs, 3)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_kernel_source_tiny_meshes(order):
    for shape in [(1, 1, 1), (2, 3, 1), (3, 1, 2)]:
        _steps(workloads.random_smooth(shape, seed=3), order, "modal", "hll", 1)
