"""CPU checks of the C ABI: the built library loads and exports every symbol
that include/ader.h declares; argument validation that returns before any
device call."""

import ctypes
import os
import re

import pytest

from paper_1006_2146_amd import ader

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ader.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ader_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(ader.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ader.LIB_PATH):
        pytest.skip("libader_hip.so not built (run __graft_entry__.build())")
    return ader.load()


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert ader.strerror(code)
    assert ader.strerror(-99) == "unknown error"


def test_argument_validation_before_device(lib):
    out = ctypes.c_void_p()
    bad = ader.ader_mesh(0, 4, 4, 1.0, 1.0, 1.0)
    assert lib.ader_create(ctypes.byref(bad), 0, 0, None, ctypes.byref(out)) == ader.ADER_EINVAL
    neg = ader.ader_mesh(4, 4, 4, -1.0, 1.0, 1.0)
    assert lib.ader_create(ctypes.byref(neg), 0, 0, None, ctypes.byref(out)) == ader.ADER_EINVAL
    ok = ader.ader_mesh(4, 4, 4, 1.0, 1.0, 1.0)
    assert lib.ader_create(ctypes.byref(ok), 7, 0, None, ctypes.byref(out)) == ader.ADER_EINVAL
    assert lib.ader_create(None, 0, 0, None, ctypes.byref(out)) == ader.ADER_EINVAL
    assert lib.ader_set_gamma(None, 1.4) == ader.ADER_EINVAL
    assert lib.ader_step(None, 0.1) == ader.ADER_EINVAL
    assert lib.ader_set_order(None, 3, 0) == ader.ADER_EINVAL
    lib.ader_destroy(None)


def test_probe_library_apart_from_the_step_abi(lib):
    # the measurement probes live in their own library and header
    assert not hasattr(lib, "ader_probe_peak")
    probe = ader.load_probe()
    v = ctypes.c_double()
    assert probe.ader_probe_peak(0, 3, ctypes.byref(v)) == ader.ADER_EINVAL
    assert probe.ader_probe_peak(0, 0, None) == ader.ADER_EINVAL
    assert not hasattr(lib, "ader_probe_face_eval")
    out = (ctypes.c_double * 6)()
    assert probe.ader_probe_face_eval(0, 2, out) == ader.ADER_EINVAL
    assert probe.ader_probe_face_eval(0, 3, None) == ader.ADER_EINVAL


def test_product_path_has_no_oracle_dependency():
    # the HIP path's sources never name the oracle package
    pkg = os.path.join(ROOT, "paper_1006_2146_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
