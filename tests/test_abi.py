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


def test_host_error_paths_of_the_simulator_and_the_lstm():
    """Argument checks that run before any device call."""
    from paper_2411_10258_amd import _lib
    lib = _lib.load()
    buf = ctypes.create_string_buffer(256)
    d = ctypes.c_void_p(16)
    # simulate: bad sizes, decay or simulation mode; per-pair decays above 32 dims
    assert lib.mdhp_simulate(-1, 4, 0, d, d, d, 1, None, d, 1, 0, d, d, d, d, None) == -1
    assert lib.mdhp_simulate(2, 65, 0, d, d, d, 1, None, d, 1, 0, d, d, d, d, None) == -1
    assert lib.mdhp_simulate(2, 33, 1, d, d, d, 1, None, d, 1, 0, d, d, d, d, None) == -1
    assert lib.mdhp_simulate(2, 4, 0, d, d, d, 5, None, d, 1, 0, d, d, d, d, None) == -1
    assert lib.mdhp_simulate(2, 4, 0, d, d, d, 0, None, d, 1, 0, d, d, d, d, None) == -1
    assert lib.mdhp_last_error(buf, 256) == -1 and b"null pointer" in buf.value
    assert lib.mdhp_simulate(0, 4, 0, None, None, None, 1, None, None, 1, 0, None, None, None,
                             None, None) == 0
    assert lib.mdhp_attack_times(-1, d, d, d, d, d, 1, 0, d, d, None) == -1
    assert lib.mdhp_attack_times(3, None, d, d, d, d, 1, 0, d, d, None) == -1
    assert lib.mdhp_attack_times(0, None, None, None, None, None, 1, 0, None, None, None) == 0
    assert lib.mdhp_plan_dim_counts(None, d, None) == -1
    # MDHP-LSTM: dimensions, null pointers, the empty forward pass
    saved, work = ctypes.c_int64(), ctypes.c_int64()
    for B, L, D, H, M, mode in ((4, 3, 5, 96, 2, 0), (4, 0, 5, 64, 2, 0), (-1, 3, 5, 64, 2, 0),
                                (4, 3, 5, 64, 65, 0), (4, 3, 5, 64, 2, 3), (4, 3, 0, 64, 2, 0)):
        dims = _lib.MdhpLstmDims(B, L, D, H, M, mode)
        assert lib.mdhp_lstm_sizes(ctypes.byref(dims), ctypes.byref(saved),
                                   ctypes.byref(work)) == -1
    dims = _lib.MdhpLstmDims(4096, 128, 256, 256, 16, 0)
    assert lib.mdhp_lstm_sizes(ctypes.byref(dims), ctypes.byref(saved), ctypes.byref(work)) == 0
    Kf = 16 * 16 + 1 + 16
    assert saved.value == 4096 * 128 * 5 * 256 + 4096 * 256 + 4096 * Kf
    pair = _lib.MdhpLstmDims(8, 2, 3, 64, 4, 1)
    s_pair = ctypes.c_int64()
    assert lib.mdhp_lstm_sizes(ctypes.byref(pair), ctypes.byref(s_pair), ctypes.byref(work)) == 0
    assert s_pair.value == 8 * 2 * 5 * 64 + 8 * 64 + 8 * (16 + 16 + 4)
    assert lib.mdhp_lstm_sizes(None, ctypes.byref(saved), ctypes.byref(work)) == -1
    args = [d] * 12
    assert lib.mdhp_lstm_forward(ctypes.byref(dims), *([None] + args[1:]), None) == -1
    assert lib.mdhp_last_error(buf, 256) == -1 and b"null pointer" in buf.value
    empty = _lib.MdhpLstmDims(0, 3, 5, 64, 2, 0)
    assert lib.mdhp_lstm_forward(ctypes.byref(empty), *([None] * 12), None) == 0
    assert lib.mdhp_lstm_backward(ctypes.byref(dims), *([None] * 14), None) == -1
    # with B = 0 the weight arrays are still required
    assert lib.mdhp_lstm_backward(ctypes.byref(empty), *([None] * 14), None) == -1


def test_first_slots_compaction():
    """The binding's compaction of per-window rooms to the events drawn."""
    import torch
    from paper_2411_10258_amd.api import _first_slots
    off = torch.tensor([0, 5, 5, 12, 20])
    n = torch.tensor([3, 0, 7, 2])
    assert _first_slots(off, n).tolist() == [0, 1, 2, 5, 6, 7, 8, 9, 10, 11, 12, 13]
    assert _first_slots(torch.tensor([0]), torch.zeros(0, dtype=torch.int64)).numel() == 0
    assert _first_slots(torch.tensor([0, 4]), torch.tensor([4])).tolist() == [0, 1, 2, 3]
