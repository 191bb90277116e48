#!/usr/bin/env python3
"""Throughput of the MI355X ADER-CG step on the 128^3 Sedov-mode Euler workload.

One "step" is the whole hot path on the device: dt by CFL (wavefront max
reduction), third-order WENO reconstruction, the ADER-CG space-time
predictor, face-side quadrature, Riemann fluxes and the FP64 update.  The
state stays resident in HBM (a torch tensor bound zero-copy to the library;
torch is used for the device buffer and the stream only).

Prints ONE JSON line (rank 0, one GPU).  Extra fields: the four variants
(FP64 / mixed x HLL / linearized), per-stage device times, the roofline of
the dominant kernel and the CPU oracle baseline.

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
# Vector ALU peaks from the unit counts and clock: 256 CUs x 4 SIMDs x 16
# lanes x 2 flops per FMA x 2.4 GHz = 78.6 TFLOP/s, for FP64 and for FP32 as
# compiled here (without packed FP32 instructions, so one FP32 FMA per lane
# per clock); the published FP32 vector figure, 157.3, counts packed FP32.
PEAK_TFLOPS = {"f64": 78.6, "f32": 78.6}
PUBLISHED_TFLOPS = {"f64": 78.6, "f32": 157.3}
HBM_PEAK_GBS = 8000.0
RECON_NAMES = ["sweeps", "tiled", "columns"]
LAYOUT_NAMES = {0: "zone", 1: "split", 2: "split-2waves", 3: "zone-prescan", 4: "zone-2waves",
                5: "pair", 6: "pair-2waves", 7: "pair-2kernels"}
METRIC = "zone-updates/sec, 3D ADER-WENO3/4 Euler+MHD; mixed-prec batched vs FP64"


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
        else:
            ader.ader_autotune(ctx, 4)
            self.saved[key] = {"launch": ader.ader_get_launch(ctx),
                               "layout": ader.ader_get_layout(ctx),
                               "recon": ader.ader_get_recon(ctx)}

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


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` at 128^3 from the committed counter
    summary, if it was taken on these kernel sources; else None."""
    path = os.path.join(HERE, "profiles", "traffic_sedov128_o3.md")
    if not os.path.exists(path):
        return None
    value, digest = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_bytes_per_launch %s 128^3:" % kernel):
                value = float(line.rsplit(":", 1)[1])
            if line.startswith("kernel sources: sha256 "):
                digest = line.split()[-1]
    return value if value is not None and digest == kernel_source_hash() else None


def flop_counts():
    path = os.path.join(HERE, "paper_1006_2146_amd", "csrc", "generated", "flop_counts.json")
    with open(path) as fh:
        return json.load(fh)["counts"]


def run_variant(ader, torch, U0, precision, riemann, steps, warmup, order=3, B0=None, key="",
                form=None):
    """Autotune the launch shapes, time `steps` graph-replayed CFL steps
    (wall clock between synchronisations), then take a separate eager pass
    with per-stage HIP events for the stage breakdown."""
    nz, ny, nx = SHAPE
    N = nx * ny * nz
    stream = torch.cuda.Stream()
    mhd = B0 is not None
    s = ader.Solver(SHAPE, order=order, riemann=riemann, precision=precision,
                    stream=stream.cuda_stream, gamma=5.0 / 3.0 if mhd else 1.4,
                    system=ader.ADER_MHD if mhd else ader.ADER_EULER,
                    form=ader.ADER_MODAL if form is None else form)
    try:
        with torch.cuda.stream(stream):
            dU = torch.from_numpy(U0).to("cuda")            # resident state, 5 x N doubles
            dB = torch.from_numpy(B0).to("cuda") if mhd else None
        stream.synchronize()
        ader.ader_bind_device_state(s.ctx, dU.data_ptr(), dB.data_ptr() if mhd else None)
        TUNE.apply(ader, s.ctx, key)
        ader.ader_set_graph(s.ctx, True)
        for _ in range(warmup):
            s.step_cfl(CFL)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(CFL)
        s.synchronize()                                  # raises on an unphysical state
        t1 = time.perf_counter()
        # stage breakdown: eager steps with events around each stage
        ader.ader_set_timing(s.ctx, True)
        for _ in range(steps):
            s.step_cfl(CFL)
        stages = ader.ader_stage_times(s.ctx)
        ader.ader_set_timing(s.ctx, False)
        s.synchronize()
        finite = bool(torch.isfinite(dU).all().item())
        launch = ader.ader_get_launch(s.ctx)
        layout = LAYOUT_NAMES[ader.ader_get_layout(s.ctx)]
        recon_mode = RECON_NAMES[ader.ader_get_recon(s.ctx)]
    finally:
        s.close()
    wall = t1 - t0
    return {
        "zone_updates_per_s": N * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "launch": launch,
        "predict_layout": layout,
        "recon_mode": recon_mode,
        "finite": finite,
    }


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
        out = {"workload": "turbulent-mhd-384^3: 64-mode k^-5/3 velocity (rms Mach 1) and vector "
                           "potential, rho 1, P 0.6, rms |B| 1; order 4 modal, linearized, CT, "
                           "gamma 5/3, FP32 bulk / FP64 update",
               "zones": zones, "steps": steps,
               "zone_updates_per_s": zones * steps / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
               "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
               "device_gb": ader.ader_device_bytes(s.ctx) / 1e9,
               "predict_layout": LAYOUT_NAMES[ader.ader_get_layout(s.ctx)],
               "finite": bool(torch.isfinite(dU).all().item())}
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
    out = {"workload": WORKLOAD + " (Euler) and mhd-random-field-128^3 (MHD), HLL, CFL %.2f; "
           "SSP-RK2/RK3/SSP(5,4) at orders 2/3/4" % CFL,
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
                                system=ader.ADER_MHD if mhd else ader.ADER_EULER)
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
        ader.ader_set_graph(s.ctx, True)
        s.step_cfl(0.4)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(0.4)
        s.synchronize()
        t1 = time.perf_counter()
    finally:
        s.close()
    return {"workload": "density-wave-32^3, order 2 nodal, minmod, HLL, FP64, CFL 0.4",
            "steps": steps, "zone_updates_per_s": 32 ** 3 * steps / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / steps}


def run_host_roundtrip(ader, U0, steps):
    """The same 128^3 mixed HLL run through the host-buffer entry points:
    ader_set_state from host memory, `steps` CFL steps, ader_get_state back
    to host memory, all inside the timed region (the PCIe-inclusive rate; the
    headline value keeps the state resident)."""
    nz, ny, nx = SHAPE
    N = nx * ny * nz
    s = ader.Solver(SHAPE, order=3, riemann=ader.ADER_HLL, precision=ader.ADER_MIXED)
    try:
        cfg = TUNE.saved.get("mixed-hll")
        if cfg:
            ader.ader_set_launch(s.ctx, {k: tuple(v) for k, v in cfg["launch"].items()})
            ader.ader_set_layout(s.ctx, cfg["layout"])
            ader.ader_set_recon(s.ctx, cfg["recon"])
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


def run_ensemble(ader, torch, steps, warmup):
    """The batched ensemble: 64 uneven problems, order 3, HLL, mixed
    precision, one persistent launch per stage, graph-replayed, autotuned."""
    from paper_1006_2146_amd import workloads
    ens = workloads.ensemble()
    shapes = [s for s, _ in ens]
    zones = int(sum(np.prod(s) for s in shapes))
    out = {"workload": "64 problems, sides from {32,48,64,96} per axis (seed 4096), order 3 "
                       "modal, HLL, gamma 1.4, smooth random modes", "zones": zones}
    for name, prec in (("mixed", ader.ADER_MIXED), ("fp64", ader.ADER_FP64)):
        stream = torch.cuda.Stream()
        with ader.BatchSolver(shapes, order=3, precision=prec, stream=stream.cuda_stream) as b:
            for i, (_, U) in enumerate(ens):
                b.set_state(i, U)
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
            out[name] = {"zone_updates_per_s": zones * steps / (t1 - t0),
                         "ms_per_step": 1e3 * (t1 - t0) / steps,
                         "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
                         "launch": ader.ader_get_launch(b.ctx),
                         "predict_layout": LAYOUT_NAMES[ader.ader_get_layout(b.ctx)],
                         "recon_mode": RECON_NAMES[ader.ader_get_recon(b.ctx)]}
        log("ensemble", name, "%.3e zone-updates/s" % out[name]["zone_updates_per_s"])
    out["mixed_over_fp64"] = out["mixed"]["zone_updates_per_s"] / out["fp64"]["zone_updates_per_s"]
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
#   update U and the zone's own F read (40 + 120 B), U written (40 B).
def hbm_bytes_per_zone(b):
    return {"recon": 120 + 45 * b + 15 * b, "flux": 90 * b + 40 + 120, "update": 200}


def hbm_stages(pv, N, dtype, probes):
    b = 8 if dtype == "f64" else 4
    out = {}
    for stage, per_zone in hbm_bytes_per_zone(b).items():
        ms = pv["stage_ms_per_step"][stage]
        gbs = per_zone * N / (ms * 1e-3) / 1e9
        out[stage] = {"bytes_per_zone": per_zone, "ms": ms, "achieved_gbs": gbs,
                      "frac_of_8tbs": gbs / HBM_PEAK_GBS}
        if probes:
            out[stage]["frac_of_copy"] = gbs / probes["hbm_copy_gbs"]
    return out


def accuracy(ader, U0, order, riemann, steps, B0=None, trunc_order=None, form=None):
    """Untimed accuracy pass of the mixed path: the FP64 path takes `steps`
    CFL steps, the mixed path repeats them with the same dt sequence, and the
    relative L1 distance (largest over the variables) is reported.  With
    trunc_order, the FP64 result at that higher order on the same steps
    estimates the truncation error of the scheme at this resolution."""
    mhd = B0 is not None
    kw = dict(order=order, riemann=riemann, gamma=5.0 / 3.0 if mhd else 1.4,
              system=ader.ADER_MHD if mhd else ader.ADER_EULER,
              form=ader.ADER_MODAL if form is None else form)

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


def cpu_baseline(U0):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: one step of a 64^3 periodic sub-box (ghost zones included in
    the work, only the 64^3 interior counted)."""
    from oracle import OracleConfig, compute_dt, step_block
    cfg = OracleConfig(order=3, riemann="hll")
    dt = compute_dt(U0, cfg, CFL)
    box = (64, 64, 64)
    t0 = time.perf_counter()
    step_block(U0, dt, cfg, (32, 32, 32), box)
    el = time.perf_counter() - t0
    return {"value": float(np.prod(box) / el), "unit": "zone-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": "one order-3 HLL FP64 step of a 64^3 periodic sub-box of the "
                      "128^3 Sedov-mode workload (numpy, single thread), %.1f s" % el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants",
                    default="fp64-hll,fp64-lin,mixed-hll,mixed-lin,fp64-hll-nodal,mixed-hll-nodal",
                    help="order-3 Euler runs: {fp64,mixed}-{hll,lin}[-nodal]")
    ap.add_argument("--mhd-variants", default="fp64,mixed,mixed-lin",
                    help="order-4 MHD runs on the 128^3 random-field workload: fp64, mixed "
                         "(HLL), fp64-lin, mixed-lin (linearized); '' for none")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 64-problem batched ensemble")
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the ADER vs SSP-RK comparison (orders 2-4)")
    ap.add_argument("--no-turbulent", action="store_true",
                    help="skip the 384^3 turbulent MHD run (order 4, linearized, mixed)")
    ap.add_argument("--tune-file", default=None,
                    help="reuse the launch shapes and layouts in this file if it exists, "
                         "else autotune and write them there")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the FMA and HBM-copy peak probes")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the untimed mixed-vs-FP64 accuracy pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (a reference kernel "
                         "of known traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1006_2146_amd import ader, workloads

    global TUNE
    TUNE = Tuning(args.tune_file)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    ader.load()
    probes = None
    if not args.no_probes:
        log("peak probes")
        probes = {"fp32_fma_tflops": ader.ader_probe_peak(ader.ADER_PROBE_FP32_FMA),
                  "fp64_fma_tflops": ader.ader_probe_peak(ader.ADER_PROBE_FP64_FMA),
                  "hbm_copy_gbs": ader.ader_probe_peak(ader.ADER_PROBE_HBM_COPY)}
        log("probes", probes)
    log("building the workload", SHAPE)
    U0 = workloads.sedov_modes(SHAPE)
    N = int(np.prod(SHAPE))

    variants = {}
    table = {"fp64-hll": (ader.ADER_FP64, ader.ADER_HLL), "fp64-lin": (ader.ADER_FP64, ader.ADER_LINEARIZED),
             "mixed-hll": (ader.ADER_MIXED, ader.ADER_HLL), "mixed-lin": (ader.ADER_MIXED, ader.ADER_LINEARIZED)}
    for name in args.variants.split(","):
        # "-nodal": the nodal predictor of App. B instead of the modal one
        prec, rs = table[name.replace("-nodal", "")]
        form = ader.ADER_NODAL if name.endswith("-nodal") else ader.ADER_MODAL
        log("variant", name, "warmup", args.warmup, "steps", args.steps)
        variants[name] = run_variant(ader, torch, U0, prec, rs, args.steps, args.warmup, key=name,
                                     form=form)
        log("variant", name, "%.3e zone-updates/s" % variants[name]["zone_updates_per_s"])

    mhd_variants = {}
    if args.mhd_variants:
        log("building the MHD workload", SHAPE)
        Um, Bm = workloads.mhd_random_field(SHAPE)
        for name in args.mhd_variants.split(","):
            prec = ader.ADER_FP64 if name.startswith("fp64") else ader.ADER_MIXED
            rs = ader.ADER_LINEARIZED if name.endswith("-lin") else ader.ADER_HLL
            log("mhd variant", name)
            mhd_variants["mhd-o4-" + name] = run_variant(ader, torch, Um, prec, rs,
                                                         args.steps, args.warmup, order=4, B0=Bm,
                                                         key="mhd-o4-" + name)
            log("mhd variant", name, "%.3e zone-updates/s"
                % mhd_variants["mhd-o4-" + name]["zone_updates_per_s"])

    for name in ([] if args.no_accuracy else variants):
        if name.startswith("mixed"):
            log("accuracy", name)
            base = name.replace("-nodal", "")
            rs = ader.ADER_HLL if base.endswith("hll") else ader.ADER_LINEARIZED
            form = ader.ADER_NODAL if name.endswith("-nodal") else ader.ADER_MODAL
            variants[name]["accuracy"] = accuracy(ader, U0, 3, rs, 10, trunc_order=4, form=form)
    for name in ([] if args.no_accuracy else mhd_variants):
        if "mixed" in name:
            log("accuracy", name)
            rs = ader.ADER_LINEARIZED if name.endswith("-lin") else ader.ADER_HLL
            mhd_variants[name]["accuracy"] = accuracy(ader, Um, 4, rs, 3, B0=Bm)

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d bytes" % nbytes)

    log("density wave 32^3")
    small = run_density_wave(ader, torch)

    roundtrip = None
    if "mixed-hll" in variants:
        log("host round trip")
        roundtrip = run_host_roundtrip(ader, U0, args.steps)

    schemes = None
    if not args.no_schemes:
        log("ADER vs SSP-RK")
        schemes = run_schemes(ader, torch, U0, max(3, min(args.steps, 10)), 1,
                              *((Um, Bm) if args.mhd_variants else (None, None)))

    turbulent = None
    if not args.no_turbulent and args.mhd_variants:
        log("turbulent MHD 384^3")
        turbulent = run_turbulent(ader, torch, max(2, min(args.steps, 5)), 1)

    ensemble = None
    if not args.no_ensemble:
        log("batched ensemble")
        ensemble = run_ensemble(ader, torch, args.steps, args.warmup)

    primary = "mixed-hll" if "mixed-hll" in variants else next(iter(variants))
    pv = variants[primary]
    dtype = "f64" if primary.startswith("fp64") else "f32"
    flops_zone = flop_counts()["M3" if dtype == "f64" else "M3-dev"]["total"]
    pred_ms = pv["stage_ms_per_step"]["predict"]
    achieved = flops_zone * N / (pred_ms * 1e-3) / 1e12
    layout = pv.get("predict_layout")
    kernel = {("f32", "zone"): "k_predict<float,3,0,true,1>",
              ("f32", "zone-prescan"): "k_predict<float,3,0,false,1>",
              ("f32", "zone-2waves"): "k_predict<float,3,0,true,2>",
              ("f64", "zone"): "k_predict<double,3,0,true,1>",
              ("f64", "zone-prescan"): "k_predict<double,3,0,false,1>",
              ("f64", "zone-2waves"): "k_predict<double,3,0,true,2>"}.get((dtype, layout),
                                                                          "k_predict (%s)" % layout)
    roofline = {"bound": "alu", "kernel": kernel, "achieved": achieved,
                "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[dtype], "traffic": recorded_traffic(kernel),
                "traffic_unit": "HBM bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                "flops_per_zone": flops_zone, "launch_ms": pred_ms,
                "peak_basis": "256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz; FP32 without "
                              "packed instructions (disabled in this build)",
                "peak_published": PUBLISHED_TFLOPS[dtype],
                "frac_published": achieved / PUBLISHED_TFLOPS[dtype]}
    if probes:
        key = "fp64_fma_tflops" if dtype == "f64" else "fp32_fma_tflops"
        roofline["peak_measured"] = probes[key]
        roofline["frac_measured"] = achieved / probes[key]

    out = {
        "metric": METRIC,
        "value": pv["zone_updates_per_s"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": pv["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "system": "euler", "order": 3, "form": "modal",
                   "riemann": primary.split("-")[1], "precision": primary.split("-")[0],
                   "precision_detail": "FP32 bulk in deviation form; FP64 state, fluxes, "
                                       "update and dt" if dtype == "f32" else "FP64 throughout",
                   "zones": N, "cfl": CFL, "gamma": 1.4, "steps_replayed_as": "hipGraph",
                   "launch": "autotuned"},
        "roofline": roofline,
        "peak_probes": probes,
        "hbm_stages": hbm_stages(pv, N, dtype, probes),
        "variants": variants,
        "mhd_variants": {"workload": "mhd-random-field-128^3, order 4 modal, CT, gamma 5/3; "
                                     "HLL, or linearized (-lin)",
                         **mhd_variants},
        "ensemble": ensemble,
        "turbulent_mhd": turbulent,
        "ader_vs_ssprk": schemes,
        "host_roundtrip": roundtrip,
        "density_wave_32": small,
    }
    for prec in ("fp64", "mixed"):
        if prec + "-hll" in variants and prec + "-hll-nodal" in variants:
            out.setdefault("nodal_over_modal", {})[prec + "-hll"] = (
                variants[prec + "-hll-nodal"]["zone_updates_per_s"] /
                variants[prec + "-hll"]["zone_updates_per_s"])
    if "mixed-hll" in variants and "fp64-hll" in variants:
        out["mixed_over_fp64"] = (variants["mixed-hll"]["zone_updates_per_s"] /
                                  variants["fp64-hll"]["zone_updates_per_s"])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(U0)
    TUNE.write()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
