"""Plain FP64 CPU oracle for one ADER-CG time step on a periodic 3D mesh.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library under ``paper_1006_2146_amd/``) never calls it, and this package
shares no code, tables or helpers with that path.

Everything here follows Balsara, Meyer, Dumbser, Du & Xu, "Efficient
Implementation of ADER Schemes for Euler and Magnetohydrodynamical Flows on
Structured Meshes" (arXiv:1006.2146).  Each function names the section and
equation it restates.  Arrays are numpy float64 in the layout
``U[var][z][y][x]`` (x fastest), and every stage is vectorised over zones with
``numpy.roll`` for the periodic neighbours, so a reader can hold each line
against the paper.

Modules
-------
basis     -- Hermite/temporal basis (eq. 9, 13), mode orderings (eq. 10-16)
physics   -- Euler / ideal-MHD conserved fluxes in Gaussian units (eq. 3)
weno      -- zone-centred WENO / minmod reconstruction (Sec. II.1)
bweno     -- WENO zone-averaging of face-centred B (Sec. III)
predictor -- ADER-CG space-time predictor, modal (Sec. IV) and nodal (App. A, B)
faces     -- barycentre states and face/edge space-time averages (Sec. V, App. D)
riemann   -- HLL (eq. 17, 56) and linearized Riemann fluxes at frozen states
step      -- whole step: dt by CFL, flux-difference update (eq. 6), CT (eq. 8)
linadv    -- the same step for linear advection of five components (test system)

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` except the choices the paper leaves open (WENO
linear weights and epsilon, the CFL convention, the frozen state of the
linearized solver), which are documented readings with no paper value to pin
against.
"""

from .step import OracleConfig, compute_dt, step, step_block  # noqa: F401
