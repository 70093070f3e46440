"""The C-ABI library loads and exports every declared symbol; host-side
error paths work without a GPU (no compute calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdhp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdhp_[a-z_]+)\s*\(", text)))


def test_header_lists_entry_points():
    names = _declared()
    for n in ("mdhp_plan_create", "mdhp_loglik", "mdhp_grad", "mdhp_fit_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2411_10258_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.EXPORTS)


def test_struct_layouts():
    from paper_2411_10258_amd import _lib
    import oracle
    assert ctypes.sizeof(_lib.MdhpFitOpts) == 80
    assert ctypes.sizeof(_lib.MdhpBatch) == 48
    assert len(oracle.FitOpts().pack()) == 72


def test_host_error_paths():
    from paper_2411_10258_amd import _lib
    lib = _lib.load()
    for s in range(-7, 1):
        assert lib.mdhp_status_string(s)
    out = ctypes.c_void_p()
    assert lib.mdhp_plan_create(None, 4, 0, None, ctypes.byref(out)) == -1
    buf = ctypes.create_string_buffer(256)
    assert lib.mdhp_last_error(buf, 256) == -1 and b"batch" in buf.value
    b = _lib.MdhpBatch(1, 0, None, None, None, None)
    assert lib.mdhp_plan_create(ctypes.byref(b), 0, 0, None, ctypes.byref(out)) == -1
    assert lib.mdhp_plan_create(ctypes.byref(b), 4, 7, None, ctypes.byref(out)) == -1
    assert lib.mdhp_loglik(None, None, None, None, None, None) == -1
    assert lib.mdhp_grad(None, None, None, None, None, None, None, None, None) == -1
    opts = _lib.MdhpFitOpts()
    assert lib.mdhp_fit_batch(None, ctypes.byref(opts), None, None, None, None, None, None,
                              None, None) == -1
    assert lib.mdhp_plan_windows(None) == 0
    lib.mdhp_plan_destroy(None)
    # allocation-free entry point: sizes beyond its workspace, partial
    # gradient outputs and empty batches are settled on the host
    dummy = ctypes.c_void_p(16)
    big = _lib.MdhpBatch(65537, 10, dummy, dummy, dummy, dummy)
    assert lib.mdhp_grad_static(ctypes.byref(big), 4, dummy, dummy, dummy, dummy, None, None,
                                None, None) == -1
    assert lib.mdhp_last_error(buf, 256) == -1 and b"static workspace" in buf.value
    big = _lib.MdhpBatch(1, 4194305, dummy, dummy, dummy, dummy)
    assert lib.mdhp_grad_static(ctypes.byref(big), 4, dummy, dummy, dummy, dummy, None, None,
                                None, None) == -1
    one = _lib.MdhpBatch(1, 10, dummy, dummy, dummy, dummy)
    assert lib.mdhp_grad_static(ctypes.byref(one), 4, dummy, dummy, dummy, dummy, dummy, None,
                                None, None) == -1
    assert lib.mdhp_grad_static(ctypes.byref(one), 65, dummy, dummy, dummy, dummy, None, None,
                                None, None) == -1
    empty = _lib.MdhpBatch(0, 0, None, None, None, None)
    assert lib.mdhp_grad_static(ctypes.byref(empty), 4, None, None, None, None, None, None,
                                None, None) == 0


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    from paper_2411_10258_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libmdhp.so"))
    with pytest.raises(ImportError):
        _lib.load()
