#!/usr/bin/env python3
"""Throughput of the MI355X ADER-CG step: the batched ensemble of 64 uneven
Euler problems (order 3, HLL), mixed precision against FP64.

One "step" is the whole hot path on the device for every problem of the
batch: dt by CFL per problem (wavefront max reduction), third-order WENO
reconstruction, the ADER-CG space-time predictor, face-side quadrature,
Riemann fluxes and the FP64 update, each stage one persistent launch over
all problems, the step replayed from a hipGraph.  The states stay resident
in HBM; torch is used for device buffers and streams only.

Prints ONE JSON line (rank 0, one GPU): the headline is the batched
ensemble in mixed precision with its FP64 line and their ratio beside it.
Extra fields: the other workloads (the 32^3 density wave, the 128^3
Sedov-mode Euler runs, the 128^3 MHD random field, the 384^3 turbulent MHD
run), per-stage device times, conserved-total drift and max |div B| per
workload, the roofline of the dominant kernel, ADER against SSP-RK, and the
CPU oracle baseline (one core and all cores).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SHAPE = (128, 128, 128)
CFL = 0.3
WORKLOAD = "sedov-modes-128^3"
# Published MI355X peaks: HBM3E 8 TB/s; vector FP64 78.6 TFLOP/s and FP32
# 157.3 TFLOP/s.  The FP32 figure counts packed FP32 instructions, which this
# build does not emit; without them one FP32 FMA issues per lane per clock:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s, reported
# beside the published fraction as the figure this code can reach.
PUBLISHED_TFLOPS = {"f64": 78.6, "f32": 157.3}
NONPACKED_TFLOPS = {"f64": 78.6, "f32": 78.6}
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per zone-update: the FP64 state read once and
# written once (Euler 5, MHD 8 variables)
STATE_BYTES_PER_ZONE = {"euler": 80, "mhd": 128}
RECON_NAMES = ["sweeps", "tiled", "columns", "march"]
FLUX_NAMES = ["separate", "fused-update"]
LAYOUT_NAMES = {0: "zone", 1: "split", 2: "split-2waves", 3: "zone-prescan", 4: "zone-2waves",
                5: "pair", 6: "pair-2waves", 7: "pair-2kernels", 8: "fused-recon"}
METRIC = "zone-updates/sec, 3D ADER-WENO3/4 Euler+MHD; mixed-prec batched vs FP64"
ENSEMBLE_WORKLOAD = ("ensemble-64-uneven: 64 periodic unit-box Euler problems, sides drawn from "
                     "{32,48,64,96} per axis (seed 4096), smooth random modes, gamma 1.4; "
                     "order 3 modal ADER-WENO, HLL, CFL 0.3, per-problem dt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


class Tuning:
    """Launch shapes and predictor layout per run, autotuned on the GPU, or
    read back from a file an earlier run wrote (so that a profiled run uses
    the tuned configuration without the tuner's own trial launches)."""

    def __init__(self, path):
        self.path = path
        self.saved = {}
        self.reuse = bool(path) and os.path.exists(path)
        if self.reuse:
            with open(path) as fh:
                self.saved = json.load(fh)

    def apply(self, ader, ctx, key):
        if self.reuse:
            cfg = self.saved[key]
            ader.ader_set_launch(ctx, {k: tuple(v) for k, v in cfg["launch"].items()})
            ader.ader_set_layout(ctx, cfg["layout"])
            ader.ader_set_recon(ctx, cfg["recon"])
            ader.ader_set_flux_mode(ctx, cfg.get("flux", -1))
        else:
            ader.ader_autotune(ctx, 4)
            self.saved[key] = {"launch": ader.ader_get_launch(ctx),
                               "layout": ader.ader_get_layout(ctx),
                               "recon": ader.ader_get_recon(ctx),
                               "flux": ader.ader_get_flux_mode(ctx)}

    def write(self):
        if self.path and not self.reuse:
            with open(self.path, "w") as fh:
                json.dump(self.saved, fh, indent=1)


TUNE = Tuning(None)


def kernel_source_hash():
    """sha256 over the kernel sources (file name and bytes, in name order)."""
    import glob
    import hashlib
    csrc = os.path.join(HERE, "paper_1006_2146_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(csrc, "*.hip")) +
                   [os.path.join(csrc, "generated", "ader_scheme.h")])
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, profile="traffic_ensemble64_o3.md", tag="ensemble"):
    """HBM bytes per launch of `kernel` from a committed counter summary, if
    it was taken on these kernel sources; else None."""
    path = os.path.join(HERE, "profiles", profile)
    if not os.path.exists(path):
        return None
    value, digest = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_bytes_per_launch %s %s:" % (kernel, tag)):
                value = float(line.rsplit(":", 1)[1])
            if line.startswith("kernel sources: sha256 "):
                digest = line.split()[-1]
    return value if value is not None and digest == kernel_source_hash() else None


def flop_counts():
    path = os.path.join(HERE, "paper_1006_2146_amd", "csrc", "generated", "flop_counts.json")
    with open(path) as fh:
        return json.load(fh)["counts"]


def conservation(tot0, div0, tot1, div1, mhd, steps):
    """Drift of the device totals (ader_diagnostics) over a run: per
    conserved quantity |T_end - T_start| / max(|mass|, |energy|) at the
    start, the largest over the problems of a batch; and max |div B| before
    and after (MHD)."""
    tot0, tot1 = np.atleast_2d(tot0), np.atleast_2d(tot1)
    nq = 8 if mhd else 5
    scale = np.maximum(np.abs(tot0[:, 0]), np.abs(tot0[:, 4]))[:, None]
    drift = (np.abs(tot1 - tot0)[:, :nq] / scale).max(axis=0)
    out = {"steps": steps, "total_drift_rel": [float(x) for x in drift],
           "quantities": ["rho", "mx", "my", "mz", "E", "Bx", "By", "Bz"][:nq],
           "scale": "max(|total mass|, |total energy|) at the start, per problem"}
    if mhd:
        out["max_abs_divB_start"] = float(np.max(div0))
        out["max_abs_divB_end"] = float(np.max(div1))
    return out


def run_variant(ader, torch, U0, precision, riemann, steps, warmup, order=3, B0=None, key="",
                form=None, positivity=None):
    """Autotune the launch shapes, time `steps` graph-replayed CFL steps
    (wall clock between synchronisations), then take a separate eager pass
    with per-stage HIP events for the stage breakdown."""
    nz, ny, nx = SHAPE
    N = nx * ny * nz
    stream = torch.cuda.Stream()
    mhd = B0 is not None
    pos = ader.ADER_POSITIVITY_CHECK if positivity is None else positivity
    s = ader.Solver(SHAPE, order=order, riemann=riemann, precision=precision,
                    stream=stream.cuda_stream, gamma=5.0 / 3.0 if mhd else 1.4,
                    system=ader.ADER_MHD if mhd else ader.ADER_EULER,
                    form=ader.ADER_MODAL if form is None else form, positivity=pos)
    try:
        with torch.cuda.stream(stream):
            dU = torch.from_numpy(U0).to("cuda")            # resident state, 5 x N doubles
            dB = torch.from_numpy(B0).to("cuda") if mhd else None
        stream.synchronize()
        ader.ader_bind_device_state(s.ctx, dU.data_ptr(), dB.data_ptr() if mhd else None)
        tot0, div0 = s.diagnostics()
        TUNE.apply(ader, s.ctx, key)
        ader.ader_set_graph(s.ctx, True)
        for _ in range(warmup):
            s.step_cfl(CFL)
        s.synchronize()
        s.limited_zones()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(CFL)
        s.synchronize()                                  # raises on an unphysical state
        t1 = time.perf_counter()
        limited = s.limited_zones()
        # stage breakdown: eager steps with events around each stage
        ader.ader_set_timing(s.ctx, True)
        for _ in range(steps):
            s.step_cfl(CFL)
        stages = ader.ader_stage_times(s.ctx)
        ader.ader_set_timing(s.ctx, False)
        s.synchronize()
        tot1, div1 = s.diagnostics()
        finite = bool(torch.isfinite(dU).all().item())
        launch = ader.ader_get_launch(s.ctx)
        layout = LAYOUT_NAMES[ader.ader_get_layout(s.ctx)]
        recon_mode = RECON_NAMES[ader.ader_get_recon(s.ctx)]
        flux_mode = FLUX_NAMES[ader.ader_get_flux_mode(s.ctx)]
    finally:
        s.close()
    wall = t1 - t0
    out = {
        "zone_updates_per_s": N * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "launch": launch,
        "predict_layout": layout,
        "recon_mode": recon_mode,
        "flux_mode": flux_mode,
        "finite": finite,
        "positivity": "limit" if pos == ader.ADER_POSITIVITY_LIMIT else "check",
        "conservation": conservation(tot0, div0, tot1, div1, mhd, warmup + 2 * steps),
    }
    if pos == ader.ADER_POSITIVITY_LIMIT:
        out["limited_zone_polynomials_per_step"] = limited / steps
    return out


def run_turbulent(ader, torch, steps, warmup):
    """384^3 turbulent-like MHD, order 4, linearized flux, CT, FP32 bulk with
    FP64 update: graph-replayed CFL steps with the launch configuration tuned
    on the 128^3 MHD run (tuning at this size would take minutes)."""
    from paper_1006_2146_amd import workloads
    shape = (384, 384, 384)
    t0 = time.perf_counter()
    U0, B0 = workloads.turbulent_mhd(shape)
    log("turbulent MHD generated in %.1f s" % (time.perf_counter() - t0))
    zones = int(np.prod(shape))
    stream = torch.cuda.Stream()
    s = ader.Solver(shape, order=4, riemann=ader.ADER_LINEARIZED, precision=ader.ADER_MIXED,
                    stream=stream.cuda_stream, gamma=5.0 / 3.0, system=ader.ADER_MHD)
    try:
        with torch.cuda.stream(stream):
            dU = torch.from_numpy(U0).to("cuda")
            dB = torch.from_numpy(B0).to("cuda")
        stream.synchronize()
        del U0, B0
        ader.ader_bind_device_state(s.ctx, dU.data_ptr(), dB.data_ptr())
        tot0, div0 = s.diagnostics()
        cfg = TUNE.saved.get("mhd-o4-mixed-lin")
        if cfg:
            ader.ader_set_launch(s.ctx, {k: tuple(v) for k, v in cfg["launch"].items()})
            ader.ader_set_layout(s.ctx, cfg["layout"])
            ader.ader_set_recon(s.ctx, cfg["recon"])
        ader.ader_set_graph(s.ctx, True)
        for _ in range(warmup):
            s.step_cfl(CFL)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(CFL)
        s.synchronize()
        t1 = time.perf_counter()
        ader.ader_set_timing(s.ctx, True)
        s.step_cfl(CFL)
        stages = ader.ader_stage_times(s.ctx)
        ader.ader_set_timing(s.ctx, False)
        s.synchronize()
        tot1, div1 = s.diagnostics()
        out = {"workload": "turbulent-mhd-384^3: 64-mode k^-5/3 velocity (rms Mach 1) and vector "
                           "potential, rho 1, P 0.6, rms |B| 1; order 4 modal, linearized, CT, "
                           "gamma 5/3, FP32 bulk / FP64 update",
               "zones": zones, "steps": steps,
               "zone_updates_per_s": zones * steps / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
               "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
               "device_gb": ader.ader_device_bytes(s.ctx) / 1e9,
               "predict_layout": LAYOUT_NAMES[ader.ader_get_layout(s.ctx)],
               "finite": bool(torch.isfinite(dU).all().item()),
               "conservation": conservation(tot0, div0, tot1, div1, True, warmup + steps + 1)}
    finally:
        s.close()
    log("turbulent MHD %.3e zone-updates/s" % out["zone_updates_per_s"])
    return out


# Table V (one 2.53 GHz Nehalem core, 97^3 blast problems): ADER-WENO over
# RK-WENO speed at the same order and Riemann solver, Euler
PAPER_ADER_OVER_RK = {"euler-hll": {2: 198817 / 126935, 3: 75105 / 37049, 4: 21065 / 8623},
                      "euler-linearized": {2: 154674 / 92448, 3: 67025 / 31598, 4: 20348 / 8119},
                      "mhd-hll": {2: 118280 / 72047, 3: 46418 / 21791, 4: 12076 / 3778}}


def run_schemes(ader, torch, U0, steps, warmup, Um=None, Bm=None):
    """ADER-CG against SSP-RK (Sec. II.d) on the same 128^3 workloads, HLL,
    orders 2-4: Euler (Sedov modes) mixed and FP64, and MHD (random field)
    mixed; each autotuned, graph-replayed CFL steps at the same CFL."""
    nz, ny, nx = SHAPE
    N = nx * ny * nz
    out = {"workload": WORKLOAD + " (Euler, positivity limit mode) and mhd-random-field-128^3 "
           "(MHD), HLL, CFL %.2f; SSP-RK2/RK3/SSP(5,4) at orders 2/3/4" % CFL,
           "paper_ader_over_rk": {"euler-hll": PAPER_ADER_OVER_RK["euler-hll"],
                                  "mhd-hll": PAPER_ADER_OVER_RK["mhd-hll"]},
           "paper_hardware": "Intel Nehalem 2.53 GHz, one core (Table V)"}
    cases = [("mixed", ader.ADER_MIXED, False), ("fp64", ader.ADER_FP64, False)]
    if Um is not None:
        cases.append(("mhd-mixed", ader.ADER_MIXED, True))
    for prec_name, prec, mhd in cases:
        for order in (2, 3, 4):
            res = {}
            for sname, scheme in (("ader", ader.ADER_SCHEME_ADER), ("rk", ader.ADER_SCHEME_SSPRK)):
                stream = torch.cuda.Stream()
                s = ader.Solver(SHAPE, order=order, riemann=ader.ADER_HLL, precision=prec,
                                stream=stream.cuda_stream, gamma=5.0 / 3.0 if mhd else 1.4,
                                system=ader.ADER_MHD if mhd else ader.ADER_EULER,
                                positivity=ader.ADER_POSITIVITY_CHECK if mhd
                                else ader.ADER_POSITIVITY_LIMIT)
                try:
                    ader.ader_set_scheme(s.ctx, scheme)
                    with torch.cuda.stream(stream):
                        dU = torch.from_numpy(Um if mhd else U0).to("cuda")
                        dB = torch.from_numpy(Bm).to("cuda") if mhd else None
                    stream.synchronize()
                    ader.ader_bind_device_state(s.ctx, dU.data_ptr(), dB.data_ptr() if mhd else None)
                    ader.ader_autotune(s.ctx, 2)
                    ader.ader_set_graph(s.ctx, True)
                    for _ in range(warmup):
                        s.step_cfl(CFL)
                    s.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(steps):
                        s.step_cfl(CFL)
                    s.synchronize()
                    res[sname] = N * steps / (time.perf_counter() - t0)
                finally:
                    s.close()
            out["%s-o%d" % (prec_name, order)] = {
                "ader_zone_updates_per_s": res["ader"], "rk_zone_updates_per_s": res["rk"],
                "ader_over_rk": res["ader"] / res["rk"]}
            log("schemes %s order %d: ADER %.3e, RK %.3e zone-updates/s (ratio %.2f)"
                % (prec_name, order, res["ader"], res["rk"], res["ader"] / res["rk"]))
    return out


def run_density_wave(ader, torch, steps=10):
    """The 32^3 density wave (rho = 1 + 0.2 sin 2 pi (x + y + z), v = (1, 1, 1),
    P = 1), second-order nodal predictor with minmod slopes, HLL, FP64, CFL
    0.4: `steps` graph-replayed steps (after one warm-up)."""
    from paper_1006_2146_amd import workloads
    shape = (32, 32, 32)
    U0 = workloads.density_wave(shape)
    stream = torch.cuda.Stream()
    s = ader.Solver(shape, order=2, form=ader.ADER_NODAL, riemann=ader.ADER_HLL,
                    precision=ader.ADER_FP64, stream=stream.cuda_stream)
    try:
        s.set_state(U0)
        tot0, div0 = s.diagnostics()
        ader.ader_set_graph(s.ctx, True)
        s.step_cfl(0.4)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(0.4)
        s.synchronize()
        t1 = time.perf_counter()
        tot1, div1 = s.diagnostics()
    finally:
        s.close()
    return {"workload": "density-wave-32^3, order 2 nodal, minmod, HLL, FP64, CFL 0.4",
            "steps": steps, "zone_updates_per_s": 32 ** 3 * steps / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / steps,
            "conservation": conservation(tot0, div0, tot1, div1, False, steps + 1)}


def run_host_roundtrip(ader, U0, steps):
    """The same 128^3 mixed HLL run through the host-buffer entry points:
    ader_set_state from host memory, `steps` CFL steps, ader_get_state back
    to host memory, all inside the timed region (the PCIe-inclusive rate; the
    headline value keeps the state resident)."""
    nz, ny, nx = SHAPE
    N = nx * ny * nz
    s = ader.Solver(SHAPE, order=3, riemann=ader.ADER_HLL, precision=ader.ADER_MIXED,
                    positivity=ader.ADER_POSITIVITY_LIMIT)
    try:
        cfg = TUNE.saved.get("mixed-hll")
        if cfg:
            ader.ader_set_launch(s.ctx, {k: tuple(v) for k, v in cfg["launch"].items()})
            ader.ader_set_layout(s.ctx, cfg["layout"])
            ader.ader_set_recon(s.ctx, cfg["recon"])
            ader.ader_set_flux_mode(s.ctx, cfg.get("flux", -1))
        s.set_state(U0)
        s.step_cfl(CFL)
        s.synchronize()
        t0 = time.perf_counter()
        s.set_state(U0)
        for _ in range(steps):
            s.step_cfl(CFL)
        out = s.get_state()
        t1 = time.perf_counter()
        t2 = time.perf_counter()
        s.set_state(U0)
        s.synchronize()
        t3 = time.perf_counter()
        s.get_state()
        t4 = time.perf_counter()
    finally:
        s.close()
    assert np.isfinite(out).all()
    return {"steps": steps, "zone_updates_per_s": N * steps / (t1 - t0),
            "set_state_ms": 1e3 * (t3 - t2), "get_state_ms": 1e3 * (t4 - t3),
            "note": "set_state from host, %d CFL steps (eager), get_state to host, all timed"
                    % steps}


def ensemble_sample_accuracy(ader, q, shape, U):
    """Problem q of the ensemble, one CFL step from its initial state: the
    mixed and FP64 paths against the FP64 oracle (relative L1 per variable,
    the largest), and the local truncation error of the order-3 step
    estimated by the FP64 order-4 step from the same state with the same
    dt (the mixed error over it is the bound's ratio)."""
    from oracle import OracleConfig, step as oracle_step
    res = {}
    for name, prec, order in (("fp64", ader.ADER_FP64, 3), ("mixed", ader.ADER_MIXED, 3),
                              ("fp64-o4", ader.ADER_FP64, 4)):
        with ader.Solver(shape, order=order, precision=prec) as s:
            s.set_state(U)
            if "dt" not in res:
                res["dt"] = s.compute_dt(CFL)
            s.step(res["dt"])
            res[name] = s.get_state()
    ref = oracle_step(U, res["dt"], OracleConfig(order=3, riemann="hll"))

    def rel(a, b):
        return float((np.abs(a - b).sum(axis=(1, 2, 3)) / np.abs(b).sum(axis=(1, 2, 3))).max())

    trunc = rel(res["fp64"], res["fp64-o4"])
    mixed = rel(res["mixed"], ref)
    return {"problem": q, "shape": list(shape), "steps": 1,
            "fp64_l1_rel_vs_oracle": rel(res["fp64"], ref), "mixed_l1_rel_vs_oracle": mixed,
            "trunc_l1_rel_estimate": trunc, "mixed_over_trunc": mixed / trunc,
            "trunc_estimate": "order-3 minus order-4 FP64 step from the same state and dt"}


def run_ensemble(ader, torch, steps, warmup, sample=True):
    """The batched ensemble: 64 uneven problems, order 3, HLL, mixed
    precision and FP64, one persistent launch per stage, graph-replayed,
    autotuned; conserved totals and a sampled problem against the oracle."""
    from paper_1006_2146_amd import workloads
    ens = workloads.ensemble()
    shapes = [s for s, _ in ens]
    zones = int(sum(np.prod(s) for s in shapes))
    out = {"workload": ENSEMBLE_WORKLOAD, "zones": zones, "problems": len(shapes)}
    for name, prec in (("mixed", ader.ADER_MIXED), ("fp64", ader.ADER_FP64)):
        stream = torch.cuda.Stream()
        with ader.BatchSolver(shapes, order=3, precision=prec, stream=stream.cuda_stream) as b:
            for i, (_, U) in enumerate(ens):
                b.set_state(i, U)
            tot0, div0 = b.diagnostics()
            TUNE.apply(ader, b.ctx, "ensemble-" + name)
            ader.ader_set_graph(b.ctx, True)
            for _ in range(warmup):
                b.step_cfl(CFL)
            b.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                b.step_cfl(CFL)
            b.synchronize()
            t1 = time.perf_counter()
            ader.ader_set_timing(b.ctx, True)
            for _ in range(steps):
                b.step_cfl(CFL)
            stages = ader.ader_stage_times(b.ctx)
            ader.ader_set_timing(b.ctx, False)
            b.synchronize()
            tot1, div1 = b.diagnostics()
            out[name] = {"zone_updates_per_s": zones * steps / (t1 - t0),
                         "ms_per_step": 1e3 * (t1 - t0) / steps,
                         "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
                         "launch": ader.ader_get_launch(b.ctx),
                         "predict_layout": LAYOUT_NAMES[ader.ader_get_layout(b.ctx)],
                         "recon_mode": RECON_NAMES[ader.ader_get_recon(b.ctx)],
                         "flux_mode": FLUX_NAMES[ader.ader_get_flux_mode(b.ctx)],
                         "conservation": conservation(tot0, div0, tot1, div1, False,
                                                      warmup + 2 * steps)}
        log("ensemble", name, "%.3e zone-updates/s" % out[name]["zone_updates_per_s"])
    out["mixed_over_fp64"] = out["mixed"]["zone_updates_per_s"] / out["fp64"]["zone_updates_per_s"]
    if sample:
        q = int(np.argmin([np.prod(sh) for sh in shapes]))
        log("ensemble sample accuracy, problem", q, shapes[q])
        out["sample_accuracy"] = ensemble_sample_accuracy(ader, q, shapes[q], ens[q][1])
    return out


# Algorithmic HBM bytes per zone of the memory-bound stages of the order-3
# Euler step (5 variables; b = 4 bytes per bulk value in the mixed path, 8 in
# FP64; state and fluxes always double):
#   recon  (x, y, z WENO sweeps): U read once per sweep (3 x 40 B), the 9
#          higher modes written once (45 b), and the moments the later
#          sweeps read back (y reads (1,0,0): 5 b; z reads (1,0,0) and
#          (0,1,0): 10 b);
#   flux   three faces' two side packets (2 x 3 x 15 b), U of the zone (40 B),
#          F written (3 x 5 doubles = 120 B);
#   update U and the zone's own F read (40 + 120 B), U written (40 B);
#   flux with the update fused (one kernel): the six side packets (90 b),
#          the averages read (40 B: the predictor's copy in the mixed path)
#          and U written (40 B); the fluxes stay on chip.
def hbm_bytes_per_zone(b, fused=False):
    if fused:
        return {"recon": 120 + 45 * b + 15 * b, "flux": 90 * b + 40 + 40}
    return {"recon": 120 + 45 * b + 15 * b, "flux": 90 * b + 40 + 120, "update": 200}


def hbm_stages(pv, N, dtype, probes):
    b = 8 if dtype == "f64" else 4
    out = {}
    fused = pv.get("flux_mode") == "fused-update"
    for stage, per_zone in hbm_bytes_per_zone(b, fused).items():
        ms = pv["stage_ms_per_step"][stage]
        gbs = per_zone * N / (ms * 1e-3) / 1e9
        out[stage] = {"bytes_per_zone": per_zone, "ms": ms, "achieved_gbs": gbs,
                      "frac_of_8tbs": gbs / HBM_PEAK_GBS}
        if probes:
            out[stage]["frac_of_copy"] = gbs / probes["hbm_copy_gbs"]
    return out


def accuracy(ader, U0, order, riemann, steps, B0=None, trunc_order=None, form=None,
             positivity=None):
    """Untimed accuracy pass of the mixed path: the FP64 path takes `steps`
    CFL steps, the mixed path repeats them with the same dt sequence, and the
    relative L1 distance (largest over the variables) is reported.  With
    trunc_order, the FP64 result at that higher order on the same steps
    estimates the truncation error of the scheme at this resolution."""
    mhd = B0 is not None
    kw = dict(order=order, riemann=riemann, gamma=5.0 / 3.0 if mhd else 1.4,
              system=ader.ADER_MHD if mhd else ader.ADER_EULER,
              form=ader.ADER_MODAL if form is None else form,
              positivity=ader.ADER_POSITIVITY_CHECK if positivity is None else positivity)

    def run(precision, dts=None, order_=None, form_=None):
        args = dict(kw, order=order_ or order)
        if form_ is not None:
            args["form"] = form_
        with ader.Solver(SHAPE, precision=precision, **args) as s:
            s.set_state(U0, B0) if mhd else s.set_state(U0)
            out = []
            for q in range(steps):
                if dts is None:
                    out.append(s.compute_dt(CFL))
                    s.step(out[-1])
                else:
                    s.step(dts[q])
            st = s.get_state()
        return (st if mhd else (st,)), out

    ref, dts = run(ader.ADER_FP64)
    mix, _ = run(ader.ADER_MIXED, dts)

    def rel(a, b):
        return float(max((np.abs(x - y).sum(axis=(1, 2, 3)) / np.abs(y).sum(axis=(1, 2, 3))).max()
                         for x, y in zip(a, b)))

    res = {"steps": steps, "l1_rel_vs_fp64": rel(mix, ref)}
    if trunc_order:
        hi, _ = run(ader.ADER_FP64, dts, trunc_order, ader.ADER_MODAL)
        res["trunc_rel_estimate"] = rel(ref, hi)
        res["trunc_estimate"] = "order-%d FP64 result on the same steps" % trunc_order
        res["ratio"] = res["l1_rel_vs_fp64"] / res["trunc_rel_estimate"]
    return res


def _oracle_task(task):
    """One oracle step (order 3, HLL, FP64) of a box x box x box sub-box of
    ensemble problem q from its initial state (ghost zones computed, only
    the sub-box counted); returns (zones, seconds of the step)."""
    q, box = task
    from oracle import OracleConfig, compute_dt, step_block
    from paper_1006_2146_amd import workloads
    shape = workloads.ensemble_shapes()[q]
    U = workloads.random_smooth(shape, 4096 + 1 + q)
    cfg = OracleConfig(order=3, riemann="hll", zone_size=(1.0 / shape[2], 1.0 / shape[1],
                                                          1.0 / shape[0]))
    dt = compute_dt(U, cfg, CFL)
    t0 = time.perf_counter()
    step_block(U, dt, cfg, (0, 0, 0), (box, box, box))
    return float(box ** 3), time.perf_counter() - t0


def cpu_baseline(box=40):
    """The FP64 oracle, as it stands, on a bounded sample of the ensemble
    workload: one step of a box^3 periodic sub-box of one problem per
    process.  First one process alone (one core), then one process per
    available core (at most 16), all at once; the all-core value is the sum
    of the concurrent processes' rates."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    z, t = _oracle_task((0, box))
    one = z / t
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_task, [(q % 64, box) for q in range(cores)], chunksize=1)
    wall = time.perf_counter() - t0
    rate = sum(zq / tq for zq, tq in res)
    return {"value": float(rate), "unit": "zone-updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": float(one),
            "sample": "one order-3 HLL FP64 oracle step (numpy) of a %d^3 periodic sub-box of "
                      "each of %d ensemble problems, one process per core, concurrently "
                      "(%.1f s wall; %.1f s on one core alone for one sub-box)"
                      % (box, cores, wall, t)}


PREDICT_KERNELS = {("f32", "zone"): "k_predict<float,3,0,true,1>",
                   ("f32", "zone-prescan"): "k_predict<float,3,0,false,1>",
                   ("f32", "zone-2waves"): "k_predict<float,3,0,true,2>",
                   ("f32", "split"): "k_predict_split<float,3,0,1>",
                   ("f32", "split-2waves"): "k_predict_split<float,3,0,2>",
                   ("f64", "zone"): "k_predict<double,3,0,true,1>",
                   ("f64", "zone-prescan"): "k_predict<double,3,0,false,1>",
                   ("f64", "zone-2waves"): "k_predict<double,3,0,true,2>",
                   ("f64", "split"): "k_predict_split<double,3,0,1>",
                   ("f64", "split-2waves"): "k_predict_split<double,3,0,2>",
                   ("f32", "fused-recon"): "k_recon_predict<float,3,0,4>",
                   ("f64", "fused-recon"): "k_recon_predict<double,3,0,4>"}


def roofline_of(run, zones, dtype):
    """Roofline of the dominant kernel (the order-3 predictor with the face
    quadrature: ALU-bound) from its HIP-event time per launch, and of the
    whole step against the algorithmic state traffic (HBM)."""
    fc = flop_counts()["M3"]
    # the method's work as the generated code evaluates it: predictor and
    # face-side quadrature; the positivity check and the deviation form's
    # extra terms are not counted
    flops_zone = fc["predictor"] + fc["faces"]
    pred_ms = run["stage_ms_per_step"]["predict"]
    achieved = flops_zone * zones / (pred_ms * 1e-3) / 1e12
    kernel = PREDICT_KERNELS.get((dtype, run["predict_layout"]),
                                 "k_predict (%s)" % run["predict_layout"])
    step_gbs = STATE_BYTES_PER_ZONE["euler"] * zones / (run["ms_per_step"] * 1e-3) / 1e9
    return {"bound": "alu", "kernel": kernel, "achieved": achieved,
            "peak": PUBLISHED_TFLOPS[dtype], "unit": "TFLOP/s",
            "frac": achieved / PUBLISHED_TFLOPS[dtype],
            "traffic": recorded_traffic(kernel),
            "traffic_unit": "HBM bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "flops_per_zone": flops_zone,
            "flops_basis": "order-3 modal predictor (%d) + face quadrature (%d) per zone, as "
                           "the generated code evaluates them%s" % (
                               fc["predictor"], fc["faces"],
                               "; this kernel also reconstructs (WENO in LDS), whose work is "
                               "not counted" if run["predict_layout"] == "fused-recon" else ""),
            "zones_per_launch": zones, "launch_ms": pred_ms,
            "peak_basis": "published MI355X vector FP32 (packed) / FP64",
            "peak_nonpacked": NONPACKED_TFLOPS[dtype],
            "frac_nonpacked": achieved / NONPACKED_TFLOPS[dtype],
            "nonpacked_basis": "256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz: FP32 without "
                               "packed instructions, as this library is compiled",
            "whole_step": {"bound": "hbm", "bytes_per_zone": STATE_BYTES_PER_ZONE["euler"],
                           "achieved_gbs": step_gbs, "peak_gbs": HBM_PEAK_GBS,
                           "frac": step_gbs / HBM_PEAK_GBS,
                           "basis": "FP64 state read once and written once per zone-update"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants",
                    default="fp64-hll,fp64-lin,mixed-hll,mixed-lin,fp64-hll-nodal,mixed-hll-nodal",
                    help="order-3 Euler runs on the 128^3 Sedov-mode workload (positivity "
                         "limit mode): {fp64,mixed}-{hll,lin}[-nodal]; '' for none")
    ap.add_argument("--mhd-variants", default="fp64,mixed,mixed-lin",
                    help="order-4 MHD runs on the 128^3 random-field workload: fp64, mixed "
                         "(HLL), fp64-lin, mixed-lin (linearized); '' for none")
    ap.add_argument("--only-ensemble", action="store_true",
                    help="the headline ensemble alone (for profiling)")
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the ADER vs SSP-RK comparison (orders 2-4)")
    ap.add_argument("--no-turbulent", action="store_true",
                    help="skip the 384^3 turbulent MHD run (order 4, linearized, mixed)")
    ap.add_argument("--turbulent-steps", type=int, default=10)
    ap.add_argument("--tune-file", default=None,
                    help="reuse the launch shapes and layouts in this file if it exists, "
                         "else autotune and write them there")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the FMA and HBM-copy peak probes")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the untimed mixed-vs-FP64 accuracy passes")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the headline ensemble and print the other runs' JSON only "
                         "(for profiling the 128^3 workloads)")
    ap.add_argument("--only-probes", action="store_true",
                    help="the peak probes and the VALU/MFMA comparison alone (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (a reference kernel "
                         "of known traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # the CPU oracle first, before anything touches the GPU
    baseline = None
    if not args.no_cpu_baseline and not args.only_ensemble and not args.only_probes:
        log("cpu baseline (oracle, all cores)")
        baseline = cpu_baseline()
        log("cpu baseline", baseline)

    import torch
    from paper_1006_2146_amd import ader, workloads

    global TUNE
    TUNE = Tuning(args.tune_file)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    ader.load()
    probes = None
    if not args.no_probes and not args.only_ensemble:
        log("peak probes")
        probes = {"fp32_fma_tflops": ader.ader_probe_peak(ader.ADER_PROBE_FP32_FMA),
                  "fp64_fma_tflops": ader.ader_probe_peak(ader.ADER_PROBE_FP64_FMA),
                  "hbm_copy_gbs": ader.ader_probe_peak(ader.ADER_PROBE_HBM_COPY)}
        # VALU against MFMA on the predictor's side-point evaluation (FP32)
        probes["face_eval_valu_vs_mfma"] = {
            "order%d" % o: ader.ader_probe_face_eval(o) for o in (3, 4)}
        log("probes", probes)
        if args.only_probes:
            print(json.dumps({"peak_probes": probes}))
            return

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d bytes" % nbytes)

    ensemble = None
    if not args.no_ensemble:
        log("batched ensemble (headline)")
        ensemble = run_ensemble(ader, torch, args.steps, args.warmup,
                                sample=not args.no_accuracy and not args.only_ensemble)

    variants, mhd_variants = {}, {}
    small = roundtrip = schemes = turbulent = None
    if not args.only_ensemble:
        log("density wave 32^3")
        small = run_density_wave(ader, torch)
        U0 = None
        if args.variants:
            log("building the Sedov-mode workload", SHAPE)
            U0 = workloads.sedov_modes(SHAPE)
        table = {"fp64-hll": (ader.ADER_FP64, ader.ADER_HLL),
                 "fp64-lin": (ader.ADER_FP64, ader.ADER_LINEARIZED),
                 "mixed-hll": (ader.ADER_MIXED, ader.ADER_HLL),
                 "mixed-lin": (ader.ADER_MIXED, ader.ADER_LINEARIZED)}
        for name in (args.variants.split(",") if args.variants else []):
            # "-nodal": the nodal predictor of App. B instead of the modal one;
            # the 100:1 overpressure sphere needs the positivity limit mode
            prec, rs = table[name.replace("-nodal", "")]
            form = ader.ADER_NODAL if name.endswith("-nodal") else ader.ADER_MODAL
            log("variant", name, "warmup", args.warmup, "steps", args.steps)
            variants[name] = run_variant(ader, torch, U0, prec, rs, args.steps, args.warmup,
                                         key=name, form=form,
                                         positivity=ader.ADER_POSITIVITY_LIMIT)
            log("variant", name, "%.3e zone-updates/s" % variants[name]["zone_updates_per_s"])
        Um = Bm = None
        if args.mhd_variants:
            log("building the MHD workload", SHAPE)
            Um, Bm = workloads.mhd_random_field(SHAPE)
            for name in args.mhd_variants.split(","):
                prec = ader.ADER_FP64 if name.startswith("fp64") else ader.ADER_MIXED
                rs = ader.ADER_LINEARIZED if name.endswith("-lin") else ader.ADER_HLL
                log("mhd variant", name)
                mhd_variants["mhd-o4-" + name] = run_variant(ader, torch, Um, prec, rs,
                                                             args.steps, args.warmup, order=4,
                                                             B0=Bm, key="mhd-o4-" + name)
                log("mhd variant", name, "%.3e zone-updates/s"
                    % mhd_variants["mhd-o4-" + name]["zone_updates_per_s"])
        for name in ([] if args.no_accuracy else variants):
            if name.startswith("mixed"):
                log("accuracy", name)
                base = name.replace("-nodal", "")
                rs = ader.ADER_HLL if base.endswith("hll") else ader.ADER_LINEARIZED
                form = ader.ADER_NODAL if name.endswith("-nodal") else ader.ADER_MODAL
                variants[name]["accuracy"] = accuracy(ader, U0, 3, rs, 10, trunc_order=4,
                                                      form=form,
                                                      positivity=ader.ADER_POSITIVITY_LIMIT)
        for name in ([] if args.no_accuracy else mhd_variants):
            if "mixed" in name:
                log("accuracy", name)
                rs = ader.ADER_LINEARIZED if name.endswith("-lin") else ader.ADER_HLL
                mhd_variants[name]["accuracy"] = accuracy(ader, Um, 4, rs, 3, B0=Bm)
        if "mixed-hll" in variants:
            log("host round trip")
            roundtrip = run_host_roundtrip(ader, U0, args.steps)
        if not args.no_schemes and U0 is not None:
            log("ADER vs SSP-RK")
            schemes = run_schemes(ader, torch, U0, max(3, min(args.steps, 10)), 1, Um, Bm)
        if not args.no_turbulent and args.mhd_variants:
            log("turbulent MHD 384^3")
            del Um, Bm
            turbulent = run_turbulent(ader, torch, args.turbulent_steps, 1)

    if ensemble is None:
        TUNE.write()
        print(json.dumps({"sedov_variants": variants, "mhd_variants": mhd_variants,
                          "density_wave_32": small}))
        return
    head = ensemble["mixed"]
    zones = ensemble["zones"]
    roofline = roofline_of(head, zones, "f32")
    if probes:
        roofline["peak_measured"] = probes["fp32_fma_tflops"]
        roofline["frac_measured"] = roofline["achieved"] / probes["fp32_fma_tflops"]

    out = {
        "metric": METRIC,
        "value": head["zone_updates_per_s"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ENSEMBLE_WORKLOAD, "system": "euler", "problems": 64,
                   "zones": zones, "order": 3, "form": "modal", "riemann": "hll",
                   "precision": "mixed",
                   "precision_detail": "FP32 bulk in deviation form; FP64 state, fluxes, "
                                       "update and dt",
                   "positivity": "check (the paper's scheme)", "cfl": CFL,
                   "steps_replayed_as": "hipGraph", "launch": "autotuned",
                   "fp64_value": ensemble["fp64"]["zone_updates_per_s"],
                   "mixed_over_fp64": ensemble["mixed_over_fp64"]},
        "roofline": roofline,
        "hbm_stages": hbm_stages(head, zones, "f32", probes),
        "peak_probes": probes,
        "ensemble": ensemble,
        "density_wave_32": small,
        "sedov_variants": {"workload": WORKLOAD + ", order 3, positivity limit mode (the 100:1 "
                                                  "overpressure sphere makes the paper's scheme "
                                                  "meet P <= 0 in the first step)",
                           **variants},
        "mhd_variants": {"workload": "mhd-random-field-128^3, order 4 modal, CT, gamma 5/3; "
                                     "HLL, or linearized (-lin)",
                         **mhd_variants},
        "turbulent_mhd": turbulent,
        "ader_vs_ssprk": schemes,
        "host_roundtrip": roundtrip,
    }
    for prec in ("fp64", "mixed"):
        if prec + "-hll" in variants and prec + "-hll-nodal" in variants:
            out.setdefault("nodal_over_modal", {})[prec + "-hll"] = (
                variants[prec + "-hll-nodal"]["zone_updates_per_s"] /
                variants[prec + "-hll"]["zone_updates_per_s"])
    if baseline is not None:
        out["cpu_baseline"] = baseline
    TUNE.write()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
