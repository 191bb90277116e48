"""The kernel source's per-zone code (host build) under the address and
undefined-behaviour sanitizers: a child process with the sanitizer runtime
preloaded runs steps of every path the host build covers -- Euler at orders
2-4 in both forms, FP64 and mixed, both Riemann solvers, SSP-RK, MHD, the
source term and the positivity limit mode, on ragged and one-zone meshes --
and must finish with no sanitizer report.  Its results must also equal the
optimised host build's to rounding."""

import os
import subprocess
import sys

import numpy as np

from tests import hostemu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from tests import hostemu
from paper_1006_2146_amd import workloads

out = {}
U = workloads.random_smooth((5, 6, 7), seed=3)
U1 = workloads.random_smooth((1, 1, 1), seed=4)
for order in (2, 3, 4):
    for form in ("modal", "nodal"):
        for prec in ("fp64", "mixed"):
            for rs in ("hll", "linearized"):
                out["e%d%s%s%s" % (order, form, prec, rs)] = hostemu.step(
                    U, 2e-3, order, form, riemann=rs, precision=prec)
    out["one%d" % order] = hostemu.step(U1, 1e-3, order)
    out["rk%d" % order] = hostemu.step_rk(U, 2e-3, order)
    Um, Bm = workloads.mhd_random_field((4, 5, 6), seed=order, p0=1.0)
    Un, Bn = hostemu.step_mhd(Um, Bm, 1e-3, order, gamma=5.0 / 3.0)
    out["m%d" % order] = np.concatenate([Un, Bn])
A = 0.3 * np.eye(5)
out["src"] = hostemu.step(U, 2e-3, 3, source=(A, np.full(5, 0.1)))
blast = workloads.blast((8, 8, 8), p_in=100.0, p_out=0.1, radius=0.25)
out["lim"] = hostemu.step(blast, 1e-3, 3, positivity="limit")
np.savez(OUTPUT, **out)
print("sanitized run done", flush=True)
"""


def _run(env_extra, path):
    env = dict(os.environ)
    env.update(env_extra)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    code = "OUTPUT = %r\n" % path + SCRIPT
    return subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                          text=True, timeout=1500)


def test_kernel_source_under_sanitizers(tmp_path):
    san = hostemu.build_sanitized()
    rt = hostemu.sanitizer_runtime()
    r = _run({"LD_PRELOAD": rt, "ADER_HOSTEMU_LIB": san,
              "ASAN_OPTIONS": "detect_leaks=0",
              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
             str(tmp_path / "san.npz"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "sanitized run done" in r.stdout
    # the same steps in the optimised build
    hostemu.build()
    r2 = _run({}, str(tmp_path / "opt.npz"))
    assert r2.returncode == 0, r2.stderr[-4000:]
    a, b = np.load(tmp_path / "san.npz"), np.load(tmp_path / "opt.npz")
    assert sorted(a.files) == sorted(b.files)
    for k in a.files:
        tol = 1e-6 if "mixed" in k else 1e-12
        assert np.abs(a[k] - b[k]).max() <= tol * np.abs(b[k]).max(), k
