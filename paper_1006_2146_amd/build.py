"""Build libader_hip.so for gfx950 in-tree with hipcc.

The stage launches of every (system, precision, order, form) variant are
compiled from csrc/ader_stages.hip as separate objects, in parallel, next to
the host library csrc/ader_lib.hip, and linked into one shared library.
``python -m paper_1006_2146_amd.build`` (or ``build()``) always recompiles.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libader_hip.so")
PROBE_LIB = os.path.join(HERE, "libader_probe.so")
OBJ = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no hand-written or compiler-formed packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
]

VARIANTS = [(sys_, prec, order, form)
            for sys_ in ("euler", "mhd") for prec in ("fp64", "mixed")
            for order, form in ((2, 0), (2, 1), (3, 0), (3, 1), (4, 0), (4, 1))]
# linear advection (test system): FP64 only
VARIANTS += [("linadv", "fp64", order, form)
             for order, form in ((2, 0), (2, 1), (3, 0), (3, 1), (4, 0), (4, 1))]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _jobs():
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n or os.cpu_count() or 4))


def _compile(src, obj, defines, verbose):
    cmd = ([hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(HERE, "..", "include")] +
           ["-D%s=%s" % kv for kv in defines] + ["-c", "-o", obj, src])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed on %s %s:\n%s%s" % (os.path.basename(src), defines,
                                                             res.stdout, res.stderr))
    return obj


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    jobs = [(os.path.join(CSRC, "ader_lib.hip"), os.path.join(OBJ, "ader_lib.o"), []),
            (os.path.join(CSRC, "diagnostics.hip"), os.path.join(OBJ, "diagnostics.o"), []),
            (os.path.join(CSRC, "peak_probe.hip"), os.path.join(OBJ, "peak_probe.o"), [])]
    for sys_, prec, order, form in VARIANTS:
        obj = os.path.join(OBJ, "stages_%s_%s_o%d_f%d.o" % (sys_, prec, order, form))
        jobs.append((os.path.join(CSRC, "ader_stages.hip"), obj,
                     [("ADER_SYS", sys_), ("ADER_PREC", prec), ("ADER_ORDER", order),
                      ("ADER_FORM", form)]))
    with cf.ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], j[1], j[2], verbose), jobs))
    probe_obj = objs.pop(2)
    # the step library, and the measurement probes in a library of their own
    for lib, parts in ((LIB, objs), (PROBE_LIB, [probe_obj])):
        tmp = lib + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + parts
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking %s failed" % os.path.basename(lib))
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
