"""The C-ABI library loads and exports every entry point declared in include/cq.h;
argument validation answers without touching a GPU (CPU only)."""
import ctypes
import os
import re

import pytest

import paper_2209_14487_amd as cq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cq.h")


def declared_names():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cq_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = cq.lib()
    names = declared_names()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # the binding declares exactly the header's entry points
    assert sorted(cq.exported_names()) == names


def test_invalid_arguments_are_rejected_before_any_device_work():
    L = cq.lib()
    h = ctypes.c_void_p()
    assert L.cq_system_create(0, 0, 1.0, ctypes.byref(h)) == cq.CQ_EINVAL
    assert b"n_up" in L.cq_last_error()
    assert L.cq_system_create(4, 8, 1.0, ctypes.byref(h)) == cq.CQ_EINVAL
    assert L.cq_system_create(6, 6, 1.0, ctypes.byref(h)) == cq.CQ_EINVAL   # not a multiple of 4
    assert L.cq_system_create(4, 4, -1.0, ctypes.byref(h)) == cq.CQ_EINVAL
    assert L.cq_system_create(4, 4, 5.0, None) == cq.CQ_EINVAL
    assert L.cq_system_create(4, 4, 5.0, ctypes.byref(h)) == cq.CQ_OK
    # bad table shapes are refused before any allocation
    assert L.cq_system_load_bspline(h, None, 4, 16, 16, 16, 4, 0) == cq.CQ_EINVAL
    buf = (ctypes.c_double * 8)()
    assert L.cq_system_load_bspline(h, buf, 2, 16, 16, 16, 4, 0) == cq.CQ_EINVAL
    assert L.cq_system_load_bspline(h, buf, 8, 16, 16, 8, 4, 0) == cq.CQ_EINVAL
    assert L.cq_system_load_bspline(h, buf, 8, 16, 16, 16, 5, 0) == cq.CQ_EINVAL
    assert L.cq_system_load_pade_j2(h, float("nan"), 0.5, 1.0) == cq.CQ_EINVAL
    assert L.cq_system_load_pade_j2(h, 0.25, 0.5, 1.0) == cq.CQ_OK
    # a crowd needs a table of its precision
    desc = cq.CrowdDesc(cq.CQ_FP64, 1, 0, 1, 0, None, 0, 0)
    systems = (ctypes.c_void_p * 1)(h.value)
    counts = (ctypes.c_int * 1)(16)
    c = ctypes.c_void_p()
    assert L.cq_crowd_create(systems, counts, 1, ctypes.byref(desc), ctypes.byref(c)) == cq.CQ_EINVAL
    assert b"no FP64 table" in L.cq_last_error()
    counts2 = (ctypes.c_int * 2)(16, 16)
    systems2 = (ctypes.c_void_p * 2)(h.value, h.value)
    assert L.cq_crowd_create(systems2, counts2, 2, ctypes.byref(desc), ctypes.byref(c)) == cq.CQ_EINVAL
    assert b"system 0 has no FP64 table" in L.cq_last_error()  # checked for every system, before any device call
    counts0 = (ctypes.c_int * 2)(16, 0)
    assert L.cq_crowd_create(systems2, counts0, 2, ctypes.byref(desc), ctypes.byref(c)) == cq.CQ_EINVAL
    L.cq_system_destroy(h)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(cq, "_lib", None)
    monkeypatch.setattr(cq, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        cq.lib()


def test_slater_inverse_arguments_are_checked():
    L = cq.lib()
    buf = (ctypes.c_double * 16)()
    ld = (ctypes.c_double * 1)()
    sg = (ctypes.c_int * 1)()
    assert L.cq_slater_inverse(None, 8, 4, 1, buf, ld, sg, None) == cq.CQ_EINVAL
    assert L.cq_slater_inverse(buf, 2, 4, 1, buf, ld, sg, None) == cq.CQ_EINVAL
    assert L.cq_slater_inverse(buf, 8, 0, 1, buf, ld, sg, None) == cq.CQ_EINVAL
    assert L.cq_slater_inverse(buf, 8, 4096, 1, buf, ld, sg, None) == cq.CQ_EINVAL
    assert L.cq_slater_inverse(buf, 8, 4, 0, buf, ld, sg, None) == cq.CQ_EINVAL
    assert b"nmat" in L.cq_last_error()
