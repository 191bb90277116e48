"""Host (CPU) build of the HIP kernel source, for CPU tests of the kernel
logic.  Test infrastructure: the product path never loads it."""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "ader_hostemu.hip")
LIB = os.path.join(HERE, "libader_hostemu.so")
DEPS = [SRC] + [os.path.join(ROOT, "paper_1006_2146_amd", "csrc", f)
                for f in ("zone_ops.h", "physics_device.h", os.path.join("generated", "ader_scheme.h"))]

_lib = None

# precision: "fp64" (the FP64 path), "mixed" (FP32 deviation form, the mixed
# path), "fp64dev" (the deviation form in double)
PRECISION = {"fp64": 0, "mixed": 1, "fp64dev": 2}


# The same source built with the address and undefined-behaviour sanitizers
# on the host code (there is no device code in this build), for the CPU
# test that runs the kernel code under them in a child process.
SAN_LIB = os.path.join(HERE, "libader_hostemu_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-fno-omit-frame-pointer"]


def build_sanitized(force=False):
    stale = force or not os.path.exists(SAN_LIB) or any(
        os.path.getmtime(d) > os.path.getmtime(SAN_LIB) for d in DEPS)
    if stale:
        tmp = "%s.tmp%d" % (SAN_LIB, os.getpid())
        subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O0", "-std=c++17", "-fPIC",
                        "-shared"] + SAN_FLAGS + ["-o", tmp, SRC], check=True)
        os.replace(tmp, SAN_LIB)
    return SAN_LIB


def sanitizer_runtime():
    """The clang address-sanitizer runtime the sanitized build needs preloaded."""
    clang = os.path.join(os.path.dirname(os.path.realpath(subprocess.check_output(
        ["bash", "-c", "command -v hipcc"], text=True).strip())), "..", "lib", "llvm", "bin",
        "clang")
    res = subprocess.check_output([clang, "-print-resource-dir"], text=True).strip()
    return os.path.join(res, "lib", "linux", "libclang_rt.asan-x86_64.so")


def build(force=False):
    stale = force or not os.path.exists(LIB) or any(
        os.path.getmtime(d) > os.path.getmtime(LIB) for d in DEPS)
    if stale:
        tmp = "%s.tmp%d" % (LIB, os.getpid())   # parallel test workers build apart
        subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                        "-fPIC", "-shared", "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        # ADER_HOSTEMU_LIB: another build of the same source (the sanitized one)
        path = os.environ.get("ADER_HOSTEMU_LIB")
        if not path:
            path = LIB
            build()
        lib = ctypes.CDLL(path)
        D, I = ctypes.c_double, ctypes.c_int
        DP = ctypes.POINTER(ctypes.c_double)
        lib.hostemu_step.argtypes = [DP, I, I, I, D, D, D, D, I, I, I, I, D]
        lib.hostemu_step.restype = I
        lib.hostemu_step_rk.argtypes = [DP, I, I, I, D, D, D, D, I, I, I, D]
        lib.hostemu_step_rk_mhd.argtypes = [DP, DP, I, I, I, D, D, D, D, I, I, I, D]
        lib.hostemu_step_rk_mhd.restype = I
        lib.hostemu_step_rk.restype = I
        lib.hostemu_dt.argtypes = [DP, I, I, I, D, D, D, D, D]
        lib.hostemu_dt.restype = D
        lib.hostemu_step_mhd.argtypes = [DP, DP, I, I, I, D, D, D, D, I, I, I, I, D]
        lib.hostemu_step_mhd.restype = I
        lib.hostemu_mhd_dissipation.argtypes = [DP, DP, DP, I, D, DP]
        lib.hostemu_dt_mhd.argtypes = [DP, DP, I, I, I, D, D, D, D, D]
        lib.hostemu_dt_mhd.restype = D
        lib.hostemu_set_source.argtypes = [DP, DP]
        lib.hostemu_set_source.restype = None
        lib.hostemu_set_positivity.argtypes = [I]
        lib.hostemu_set_positivity.restype = None
        lib.hostemu_pos_status.argtypes = [ctypes.POINTER(I), ctypes.POINTER(ctypes.c_uint)]
        lib.hostemu_pos_status.restype = None
        _lib = lib
    return _lib


class NonPhysical(ArithmeticError):
    """The check mode met rho <= 0 or P <= 0 at a check point."""


# positivity: "check" (the paper's scheme: report, change nothing) or
# "limit" (the scaling safeguard)
POSITIVITY = {"check": 0, "limit": 1}

last_limited = 0   # scaled zone polynomials of the last step (limit mode)


def _begin(positivity):
    load().hostemu_set_positivity(POSITIVITY[positivity])


def _end():
    global last_limited
    bad = ctypes.c_int(0)
    lim = ctypes.c_uint(0)
    load().hostemu_pos_status(ctypes.byref(bad), ctypes.byref(lim))
    last_limited = lim.value
    if bad.value:
        raise NonPhysical("rho <= 0 or P <= 0 at a check point")


def _spacing(U, lengths):
    nz, ny, nx = U.shape[1:]
    return nx, ny, nz, lengths[0] / nx, lengths[1] / ny, lengths[2] / nz


def step(U, dt, order, form="modal", riemann="hll", precision="fp64",
         lengths=(1.0, 1.0, 1.0), gamma=1.4, positivity="check", source=None):
    """One ADER step; ``source`` = (A, b) adds the affine source A u + b."""
    out = np.ascontiguousarray(U, dtype=np.float64).copy()
    nx, ny, nz, dx, dy, dz = _spacing(out, lengths)
    _begin(positivity)
    lib = load()
    if source is not None:
        A = np.ascontiguousarray(source[0], dtype=np.float64).reshape(25)
        b = np.ascontiguousarray(source[1], dtype=np.float64).reshape(5)
        lib.hostemu_set_source(_dp(A), _dp(b))
    try:
        lib.hostemu_step(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nx, ny, nz,
                         dx, dy, dz, gamma, order, 1 if form == "nodal" else 0,
                         1 if riemann == "linearized" else 0, PRECISION[precision], dt)
    finally:
        lib.hostemu_set_source(None, None)
    _end()
    return out


def step_rk(U, dt, order, riemann="hll", precision="fp64", lengths=(1.0, 1.0, 1.0),
            gamma=1.4, positivity="check"):
    """One SSP-RK step (Euler) of the host build of the RK kernels."""
    out = np.ascontiguousarray(U, dtype=np.float64).copy()
    nx, ny, nz, dx, dy, dz = _spacing(out, lengths)
    _begin(positivity)
    load().hostemu_step_rk(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nx, ny, nz,
                           dx, dy, dz, gamma, order, 1 if riemann == "linearized" else 0,
                           PRECISION[precision], dt)
    _end()
    return out


def compute_dt(U, cfl, lengths=(1.0, 1.0, 1.0), gamma=1.4):
    U = np.ascontiguousarray(U, dtype=np.float64)
    nx, ny, nz, dx, dy, dz = _spacing(U, lengths)
    return load().hostemu_dt(U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nx, ny, nz,
                             dx, dy, dz, gamma, cfl)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def step_mhd(U, B, dt, order, form="modal", precision="fp64", lengths=(1.0, 1.0, 1.0),
             gamma=5.0 / 3.0, riemann="hll", positivity="check"):
    Uo = np.ascontiguousarray(U, dtype=np.float64).copy()
    Bo = np.ascontiguousarray(B, dtype=np.float64).copy()
    nx, ny, nz, dx, dy, dz = _spacing(Uo, lengths)
    _begin(positivity)
    load().hostemu_step_mhd(_dp(Uo), _dp(Bo), nx, ny, nz, dx, dy, dz, gamma, order,
                            1 if form == "nodal" else 0, 1 if riemann == "linearized" else 0,
                            PRECISION[precision], dt)
    _end()
    return Uo, Bo


def step_rk_mhd(U, B, dt, order, riemann="hll", precision="fp64", lengths=(1.0, 1.0, 1.0),
                gamma=5.0 / 3.0, positivity="check"):
    """One SSP-RK step of ideal MHD of the host build of the RK kernels."""
    Uo = np.ascontiguousarray(U, dtype=np.float64).copy()
    Bo = np.ascontiguousarray(B, dtype=np.float64).copy()
    nx, ny, nz, dx, dy, dz = _spacing(Uo, lengths)
    _begin(positivity)
    load().hostemu_step_rk_mhd(_dp(Uo), _dp(Bo), nx, ny, nz, dx, dy, dz, gamma, order,
                               1 if riemann == "linearized" else 0, PRECISION[precision], dt)
    _end()
    return Uo, Bo


def compute_dt_mhd(U, B, cfl, lengths=(1.0, 1.0, 1.0), gamma=5.0 / 3.0):
    U = np.ascontiguousarray(U, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    nx, ny, nz, dx, dy, dz = _spacing(U, lengths)
    return load().hostemu_dt_mhd(_dp(U), _dp(B), nx, ny, nz, dx, dy, dz, gamma, cfl)


def mhd_dissipation(ubl, ubr, du, axis, gamma=5.0 / 3.0):
    """|A| du of the kernel source's analytic MHD eigen-system (one face)."""
    out = np.zeros(8)
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (ubl, ubr, du)]
    load().hostemu_mhd_dissipation(_dp(args[0]), _dp(args[1]), _dp(args[2]), axis, gamma, _dp(out))
    return out
