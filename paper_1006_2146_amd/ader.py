"""Thin ctypes binding of libader_hip.so (include/ader.h), same names as the
C ABI.  Argument marshalling only: every step of the path runs in the HIP
kernels.  Raises if the library is missing; there is no CPU fallback."""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libader_hip.so")

ADER_OK = 0
ADER_EINVAL = -1
ADER_EUNSUPPORTED = -2
ADER_ENOMEM = -3
ADER_EDEVICE = -4
ADER_ESTATE = -5
ADER_ESEQ = -6

ADER_EULER, ADER_MHD, ADER_LINADV = 0, 1, 2
ADER_BC_PERIODIC, ADER_BC_OUTFLOW, ADER_BC_REFLECT, ADER_BC_INFLOW = 0, 1, 2, 3
ADER_HLL, ADER_LINEARIZED = 0, 1
ADER_MODAL, ADER_NODAL = 0, 1
ADER_FP64, ADER_MIXED = 0, 1

# every symbol include/ader.h declares
EXPORTS = [
    "ader_create", "ader_set_gamma", "ader_set_order", "ader_set_riemann",
    "ader_set_precision", "ader_set_state", "ader_bind_device_state",
    "ader_get_state", "ader_compute_dt", "ader_step", "ader_step_cfl",
    "ader_get_dt", "ader_synchronize", "ader_set_timing", "ader_stage_times",
    "ader_device_bytes", "ader_strerror", "ader_destroy",
    "ader_batch_create", "ader_batch_size", "ader_batch_set_state", "ader_batch_get_state",
    "ader_batch_step_cfl", "ader_set_graph", "ader_autotune", "ader_get_launch",
    "ader_set_launch", "ader_set_layout", "ader_get_layout", "ader_set_recon", "ader_get_recon",
    "ader_set_flux_mode", "ader_get_flux_mode",
    "ader_set_scheme", "ader_get_scheme",
    "ader_set_positivity", "ader_get_positivity", "ader_limited_zones", "ader_diagnostics",
    "ader_diagnostics_noalloc", "ader_set_source", "ader_set_advection", "ader_set_boundary",
    "ader_set_inflow",
]
ADER_SCHEME_ADER, ADER_SCHEME_SSPRK = 0, 1
ADER_POSITIVITY_CHECK, ADER_POSITIVITY_LIMIT = 0, 1
ADER_PROBE_FP32_FMA, ADER_PROBE_FP64_FMA, ADER_PROBE_HBM_COPY = 0, 1, 2
ADER_RECON_SWEEPS, ADER_RECON_TILED, ADER_RECON_COLUMNS, ADER_RECON_MARCH = 0, 1, 2, 3
ADER_FLUX_SEPARATE, ADER_FLUX_FUSED = 0, 1
ADER_LAYOUT_ZONE, ADER_LAYOUT_SPLIT, ADER_LAYOUT_SPLIT2, ADER_LAYOUT_ZONE2 = 0, 1, 2, 3
ADER_LAYOUT_ZONE_2W, ADER_LAYOUT_PAIR, ADER_LAYOUT_PAIR2 = 4, 5, 6
ADER_LAYOUT_PAIR_SPLIT, ADER_LAYOUT_FUSED = 7, 8
LAUNCH_CLASSES = ["dt", "recon", "predict", "flux", "update"]
STAGES = ["dt", "recon", "predict", "flux", "update"]


class ader_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double)]


class AderError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, strerror(code), code))


_lib = None


def load():
    """Load libader_hip.so (raises FileNotFoundError if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            "libader_hip.so is not built; run `python -m paper_1006_2146_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ader_create": ([ctypes.POINTER(ader_mesh), I, I, P, ctypes.POINTER(P)], I),
        "ader_set_gamma": ([P, D], I),
        "ader_set_order": ([P, I, I], I),
        "ader_set_riemann": ([P, I], I),
        "ader_set_precision": ([P, I], I),
        "ader_set_state": ([P, DP, DP], I),
        "ader_bind_device_state": ([P, P, P], I),
        "ader_get_state": ([P, DP, DP], I),
        "ader_compute_dt": ([P, D, DP], I),
        "ader_step": ([P, D], I),
        "ader_step_cfl": ([P, D], I),
        "ader_get_dt": ([P, DP], I),
        "ader_synchronize": ([P], I),
        "ader_set_timing": ([P, I], I),
        "ader_stage_times": ([P, DP, ctypes.POINTER(ctypes.c_int)], I),
        "ader_device_bytes": ([P, DP], I),
        "ader_strerror": ([I], ctypes.c_char_p),
        "ader_destroy": ([P], None),
        "ader_batch_create": ([I, ctypes.POINTER(ader_mesh), I, I, P, ctypes.POINTER(P)], I),
        "ader_batch_size": ([P, ctypes.POINTER(I)], I),
        "ader_batch_set_state": ([P, I, DP, DP], I),
        "ader_batch_get_state": ([P, I, DP, DP], I),
        "ader_batch_step_cfl": ([P, D, DP], I),
        "ader_set_graph": ([P, I], I),
        "ader_autotune": ([P, I], I),
        "ader_get_launch": ([P, ctypes.POINTER(I), ctypes.POINTER(I)], I),
        "ader_set_launch": ([P, ctypes.POINTER(I), ctypes.POINTER(I)], I),
        "ader_set_layout": ([P, I], I),
        "ader_get_layout": ([P, ctypes.POINTER(I)], I),
        "ader_set_recon": ([P, I], I),
        "ader_get_recon": ([P, ctypes.POINTER(I)], I),
        "ader_set_flux_mode": ([P, I], I),
        "ader_get_flux_mode": ([P, ctypes.POINTER(I)], I),
        "ader_set_scheme": ([P, I], I),
        "ader_get_scheme": ([P, ctypes.POINTER(I)], I),
        "ader_set_positivity": ([P, I], I),
        "ader_get_positivity": ([P, ctypes.POINTER(I)], I),
        "ader_limited_zones": ([P, ctypes.POINTER(ctypes.c_longlong)], I),
        "ader_diagnostics": ([P, DP, DP], I),
        "ader_diagnostics_noalloc": ([P, DP, DP], I),
        "ader_set_source": ([P, DP, DP], I),
        "ader_set_advection": ([P, D, D, D], I),
        "ader_set_boundary": ([P, ctypes.POINTER(I)], I),
        "ader_set_inflow": ([P, I, ctypes.POINTER(ctypes.c_double)], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(code):
    return load().ader_strerror(code).decode()


def _check(rc, where):
    if rc != ADER_OK:
        raise AderError(rc, where)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --- one Python function per C entry point -----------------------------------

def ader_create(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, system=ADER_EULER, device=0, stream=None):
    lib = load()
    mesh = ader_mesh(nx, ny, nz, lx, ly, lz)
    out = ctypes.c_void_p()
    rc = lib.ader_create(ctypes.byref(mesh), system, device,
                         ctypes.c_void_p(stream) if stream else None, ctypes.byref(out))
    _check(rc, "ader_create")
    return out


def ader_set_gamma(ctx, gamma):
    _check(load().ader_set_gamma(ctx, gamma), "ader_set_gamma")


def ader_set_order(ctx, order, form=ADER_MODAL):
    _check(load().ader_set_order(ctx, order, form), "ader_set_order")


def ader_set_riemann(ctx, riemann):
    _check(load().ader_set_riemann(ctx, riemann), "ader_set_riemann")


def ader_set_precision(ctx, precision):
    _check(load().ader_set_precision(ctx, precision), "ader_set_precision")


def ader_set_state(ctx, U, B=None):
    U = np.ascontiguousarray(U, dtype=np.float64)
    if B is not None:
        B = np.ascontiguousarray(B, dtype=np.float64)
    _check(load().ader_set_state(ctx, _dptr(U), None if B is None else _dptr(B)),
           "ader_set_state")


def ader_bind_device_state(ctx, device_ptr, b_device_ptr=None):
    _check(load().ader_bind_device_state(ctx, ctypes.c_void_p(device_ptr),
                                         ctypes.c_void_p(b_device_ptr) if b_device_ptr else None),
           "ader_bind_device_state")


def ader_get_state(ctx, shape, with_b=False):
    U = np.empty(shape, dtype=np.float64)
    B = np.empty((3,) + tuple(shape[1:]), dtype=np.float64) if with_b else None
    _check(load().ader_get_state(ctx, _dptr(U), None if B is None else _dptr(B)), "ader_get_state")
    return (U, B) if with_b else U


def ader_compute_dt(ctx, cfl, want_host=True):
    if not want_host:
        _check(load().ader_compute_dt(ctx, cfl, None), "ader_compute_dt")
        return None
    dt = ctypes.c_double()
    _check(load().ader_compute_dt(ctx, cfl, ctypes.byref(dt)), "ader_compute_dt")
    return dt.value


def ader_step(ctx, dt):
    _check(load().ader_step(ctx, dt), "ader_step")


def ader_step_cfl(ctx, cfl):
    _check(load().ader_step_cfl(ctx, cfl), "ader_step_cfl")


def ader_get_dt(ctx, n=1):
    """dt of the latest step; a list of n values for a batch of n problems."""
    dt = (ctypes.c_double * n)()
    _check(load().ader_get_dt(ctx, dt), "ader_get_dt")
    return dt[0] if n == 1 else list(dt)


def ader_synchronize(ctx):
    _check(load().ader_synchronize(ctx), "ader_synchronize")


def ader_set_timing(ctx, enable):
    _check(load().ader_set_timing(ctx, 1 if enable else 0), "ader_set_timing")


def ader_stage_times(ctx):
    """{stage: (milliseconds, launches)} since the previous call."""
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int * len(STAGES))()
    _check(load().ader_stage_times(ctx, ms, cnt), "ader_stage_times")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}


def ader_device_bytes(ctx):
    b = ctypes.c_double()
    _check(load().ader_device_bytes(ctx, ctypes.byref(b)), "ader_device_bytes")
    return b.value


def ader_set_scheme(ctx, scheme):
    _check(load().ader_set_scheme(ctx, scheme), "ader_set_scheme")


def ader_get_scheme(ctx):
    v = ctypes.c_int()
    _check(load().ader_get_scheme(ctx, ctypes.byref(v)), "ader_get_scheme")
    return v.value


def ader_set_positivity(ctx, mode):
    _check(load().ader_set_positivity(ctx, mode), "ader_set_positivity")


def ader_get_positivity(ctx):
    v = ctypes.c_int()
    _check(load().ader_get_positivity(ctx, ctypes.byref(v)), "ader_get_positivity")
    return v.value


def ader_limited_zones(ctx, n=1):
    """Per problem, the zone polynomials the limit mode scaled since the
    previous call (a list of n counts)."""
    out = (ctypes.c_longlong * n)()
    _check(load().ader_limited_zones(ctx, out), "ader_limited_zones")
    return list(out)


def ader_diagnostics(ctx, n=1):
    """(totals[n][8], max_abs_divB[n]) of the current state."""
    tot = np.empty((n, 8), dtype=np.float64)
    div = np.empty(n, dtype=np.float64)
    _check(load().ader_diagnostics(ctx, _dptr(tot), _dptr(div)), "ader_diagnostics")
    return tot, div


def ader_set_boundary(ctx, bc):
    """Kinds of the faces x-, x+, y-, y+, z-, z+ (ADER_BC_*), before the
    first state is set."""
    arr = (ctypes.c_int * 6)(*[int(x) for x in bc])
    _check(load().ader_set_boundary(ctx, arr), "ader_set_boundary")


def ader_set_inflow(ctx, face, state):
    """Conserved state (5 values) of inflow face `face` (0..5: x-, x+, y-,
    y+, z-, z+)."""
    arr = np.ascontiguousarray(state, dtype=np.float64).reshape(5)
    _check(load().ader_set_inflow(ctx, int(face), _dptr(arr)), "ader_set_inflow")


def ader_set_advection(ctx, a):
    """Velocity (ax, ay, az) of a linear-advection context."""
    _check(load().ader_set_advection(ctx, float(a[0]), float(a[1]), float(a[2])),
           "ader_set_advection")


def ader_set_source(ctx, A=None, b=None):
    """The affine source S(u) = A u + b (A 5 x 5, b 5 or None); A None
    removes it."""
    if A is None:
        _check(load().ader_set_source(ctx, None, None), "ader_set_source")
        return
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(25)
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64).reshape(5)
    _check(load().ader_set_source(ctx, _dptr(A), None if bb is None else _dptr(bb)),
           "ader_set_source")


def ader_diagnostics_noalloc(ctx, n=1):
    """ader_diagnostics with the library's fixed scratch (no allocation)."""
    tot = np.empty((n, 8), dtype=np.float64)
    div = np.empty(n, dtype=np.float64)
    _check(load().ader_diagnostics_noalloc(ctx, _dptr(tot), _dptr(div)),
           "ader_diagnostics_noalloc")
    return tot, div


_probe = None


def load_probe():
    """The measurement library (include/ader_probe.h), apart from the step
    library's ABI."""
    global _probe
    if _probe is None:
        path = os.path.join(_HERE, "libader_probe.so")
        if not os.path.exists(path):
            raise FileNotFoundError("libader_probe.so is not built")
        _probe = ctypes.CDLL(path)
        _probe.ader_probe_peak.argtypes = [ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double)]
        _probe.ader_probe_peak.restype = ctypes.c_int
        _probe.ader_probe_face_eval.argtypes = [ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_double)]
        _probe.ader_probe_face_eval.restype = ctypes.c_int
    return _probe


def ader_probe_peak(kind, device=0):
    """Measured peak of `kind` (ADER_PROBE_*): TFLOP/s for the FMA probes,
    GB/s (read + write) for the HBM copy."""
    v = ctypes.c_double()
    _check(load_probe().ader_probe_peak(device, kind, ctypes.byref(v)), "ader_probe_peak")
    return v.value


def ader_probe_face_eval(order, device=0):
    """VALU against MFMA on the side-point evaluation of order 3 or 4
    (include/ader_probe.h)."""
    out = (ctypes.c_double * 6)()
    _check(load_probe().ader_probe_face_eval(device, order, out), "ader_probe_face_eval")
    keys = ("valu_useful_tflops", "mfma_useful_tflops", "valu_ms", "mfma_ms",
            "mfma_dense_tflops", "max_rel_diff")
    return dict(zip(keys, out))


def ader_destroy(ctx):
    if ctx:
        load().ader_destroy(ctx)


def ader_batch_create(meshes, system=ADER_EULER, device=0, stream=None):
    """meshes: sequence of (nx, ny, nz, lx, ly, lz)."""
    lib = load()
    arr = (ader_mesh * len(meshes))(*[ader_mesh(*m) for m in meshes])
    out = ctypes.c_void_p()
    rc = lib.ader_batch_create(len(meshes), arr, system, device,
                               ctypes.c_void_p(stream) if stream else None, ctypes.byref(out))
    _check(rc, "ader_batch_create")
    return out


def ader_batch_size(ctx):
    n = ctypes.c_int()
    _check(load().ader_batch_size(ctx, ctypes.byref(n)), "ader_batch_size")
    return n.value


def ader_batch_set_state(ctx, i, U, B=None):
    U = np.ascontiguousarray(U, dtype=np.float64)
    if B is not None:
        B = np.ascontiguousarray(B, dtype=np.float64)
    _check(load().ader_batch_set_state(ctx, i, _dptr(U), None if B is None else _dptr(B)),
           "ader_batch_set_state")


def ader_batch_get_state(ctx, i, shape, with_b=False):
    U = np.empty(shape, dtype=np.float64)
    B = np.empty((3,) + tuple(shape[1:]), dtype=np.float64) if with_b else None
    _check(load().ader_batch_get_state(ctx, i, _dptr(U), None if B is None else _dptr(B)),
           "ader_batch_get_state")
    return (U, B) if with_b else U


def ader_batch_step_cfl(ctx, cfl, n=None):
    """One CFL step of every problem; with n, returns the n dt values taken."""
    if n is None:
        _check(load().ader_batch_step_cfl(ctx, cfl, None), "ader_batch_step_cfl")
        return None
    dts = np.empty(n, dtype=np.float64)
    _check(load().ader_batch_step_cfl(ctx, cfl, _dptr(dts)), "ader_batch_step_cfl")
    return dts


def ader_set_graph(ctx, enable):
    _check(load().ader_set_graph(ctx, 1 if enable else 0), "ader_set_graph")


def ader_autotune(ctx, reps=3):
    _check(load().ader_autotune(ctx, reps), "ader_autotune")


def ader_get_launch(ctx):
    """{class: (threads per block, blocks per CU)}."""
    k = len(LAUNCH_CLASSES)
    b = (ctypes.c_int * k)()
    g = (ctypes.c_int * k)()
    _check(load().ader_get_launch(ctx, b, g), "ader_get_launch")
    return {name: (b[i], g[i]) for i, name in enumerate(LAUNCH_CLASSES)}


def ader_set_layout(ctx, layout):
    _check(load().ader_set_layout(ctx, layout), "ader_set_layout")


def ader_get_layout(ctx):
    out = ctypes.c_int()
    _check(load().ader_get_layout(ctx, ctypes.byref(out)), "ader_get_layout")
    return out.value


def ader_set_recon(ctx, mode):
    _check(load().ader_set_recon(ctx, mode), "ader_set_recon")


def ader_get_recon(ctx):
    out = ctypes.c_int()
    _check(load().ader_get_recon(ctx, ctypes.byref(out)), "ader_get_recon")
    return out.value


def ader_set_flux_mode(ctx, mode):
    _check(load().ader_set_flux_mode(ctx, mode), "ader_set_flux_mode")


def ader_get_flux_mode(ctx):
    out = ctypes.c_int()
    _check(load().ader_get_flux_mode(ctx, ctypes.byref(out)), "ader_get_flux_mode")
    return out.value


def ader_set_launch(ctx, shapes):
    """shapes: {class: (threads per block, blocks per CU)} for every class."""
    k = len(LAUNCH_CLASSES)
    b = (ctypes.c_int * k)(*[shapes[n][0] for n in LAUNCH_CLASSES])
    g = (ctypes.c_int * k)(*[shapes[n][1] for n in LAUNCH_CLASSES])
    _check(load().ader_set_launch(ctx, b, g), "ader_set_launch")


def _configure(ctx, gamma, order, form, riemann, precision, positivity):
    ader_set_gamma(ctx, gamma)
    ader_set_order(ctx, order, form)
    ader_set_riemann(ctx, riemann)
    ader_set_precision(ctx, precision)
    ader_set_positivity(ctx, positivity)


class BatchSolver:
    """Owner of a batch context of independent problems (marshalling only).
    shapes: (nz, ny, nx) per problem; lengths: one (lx, ly, lz) or one per
    problem."""

    def __init__(self, shapes, lengths=(1.0, 1.0, 1.0), gamma=1.4, order=3, form=ADER_MODAL,
                 riemann=ADER_HLL, precision=ADER_FP64, device=0, stream=None,
                 system=ADER_EULER, positivity=ADER_POSITIVITY_CHECK, boundary=None):
        if lengths and not isinstance(lengths[0], (tuple, list)):
            lengths = [lengths] * len(shapes)
        self.shapes = [tuple(s) for s in shapes]
        self.mhd = system == ADER_MHD
        meshes = [(s[2], s[1], s[0]) + tuple(L) for s, L in zip(self.shapes, lengths)]
        self.ctx = ader_batch_create(meshes, system=system, device=device, stream=stream)
        try:
            if boundary is not None:
                ader_set_boundary(self.ctx, boundary)
            _configure(self.ctx, gamma, order, form, riemann, precision, positivity)
        except Exception:
            self.close()
            raise

    def __len__(self):
        return len(self.shapes)

    def set_state(self, i, U, B=None):
        ader_batch_set_state(self.ctx, i, U, B)

    def get_state(self, i):
        return ader_batch_get_state(self.ctx, i, (5,) + self.shapes[i], with_b=self.mhd)

    def step_cfl(self, cfl, want_dts=False):
        return ader_batch_step_cfl(self.ctx, cfl, len(self) if want_dts else None)

    def step(self, dt):
        ader_step(self.ctx, dt)

    def dts(self):
        return ader_get_dt(self.ctx, len(self))

    def limited_zones(self):
        return ader_limited_zones(self.ctx, len(self))

    def set_source(self, A=None, b=None):
        ader_set_source(self.ctx, A, b)

    def set_advection(self, a):
        ader_set_advection(self.ctx, a)

    def diagnostics(self):
        return ader_diagnostics(self.ctx, len(self))

    def synchronize(self):
        ader_synchronize(self.ctx)

    def close(self):
        if self.ctx:
            ader_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Convenience owner of one context (still marshalling only)."""

    def __init__(self, shape, lengths=(1.0, 1.0, 1.0), gamma=1.4, order=3,
                 form=ADER_MODAL, riemann=ADER_HLL, precision=ADER_FP64,
                 device=0, stream=None, system=ADER_EULER, positivity=ADER_POSITIVITY_CHECK,
                 boundary=None):
        nz, ny, nx = shape
        self.shape = (5, nz, ny, nx)
        self.mhd = system == ADER_MHD
        self.ctx = ader_create(nx, ny, nz, *lengths, system=system, device=device, stream=stream)
        try:
            if boundary is not None:
                ader_set_boundary(self.ctx, boundary)
            _configure(self.ctx, gamma, order, form, riemann, precision, positivity)
        except Exception:
            self.close()
            raise

    def set_state(self, U, B=None):
        ader_set_state(self.ctx, U, B)

    def get_state(self):
        """U (Euler) or (U, B) (MHD)."""
        return ader_get_state(self.ctx, self.shape, with_b=self.mhd)

    def compute_dt(self, cfl):
        return ader_compute_dt(self.ctx, cfl)

    def step(self, dt):
        ader_step(self.ctx, dt)

    def step_cfl(self, cfl):
        ader_step_cfl(self.ctx, cfl)

    def dt(self):
        return ader_get_dt(self.ctx)

    def limited_zones(self):
        return ader_limited_zones(self.ctx)[0]

    def set_source(self, A=None, b=None):
        ader_set_source(self.ctx, A, b)

    def set_advection(self, a):
        ader_set_advection(self.ctx, a)

    def diagnostics(self):
        """(totals[8], max |div B|) of the current state."""
        tot, div = ader_diagnostics(self.ctx, 1)
        return tot[0], div[0]

    def synchronize(self):
        ader_synchronize(self.ctx)

    def close(self):
        if self.ctx:
            ader_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
