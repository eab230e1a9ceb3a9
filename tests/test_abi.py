"""The C-ABI library loads and exports every symbol include/rsk.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2203_10838_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rsk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rsk_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    assert "rsk_avg_solve_dense" in names and "rsk_rownorm2_dense" in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("librsk.so not built (python -m paper_2203_10838_amd.build)")
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(_declared()) <= set(_abi.SIGNATURES), set(_declared()) - set(_abi.SIGNATURES)


def test_host_only_calls():
    lib = _abi.load()
    assert lib.rsk_abi_version() == 6
    assert lib.rsk_status_string(7) == b"RSK_ERR_NONFINITE"
    assert lib.rsk_status_string(99) == b"RSK_ERR_UNKNOWN"


def test_host_validation_rejects_bad_arguments():
    """Validation runs before any device work, so these need no GPU."""
    lib = _abi.load()
    d = _abi.RskDense(10, 5, 5, 0, 0x1000)
    p = _abi.RskParams(1.0, 2, 1.0, None, 3, 0x2000, 0, 0x3000, 0, None, 0, 0.0, None, None, 0x4000, 0)
    nb = ctypes.c_size_t(0)
    call = lambda: lib.rsk_avg_solve_dense(ctypes.byref(d), 0x5000, ctypes.byref(p), 0x6000, 0x7000, 0x8000,
                                           1 << 20, None)
    bad = []
    for field, val in [("eta", 0), ("K", -1), ("lambda_", -1.0), ("alpha", 0.0), ("alpha", float("nan")),
                       ("index_stream", None), ("rownorm2", None), ("status_dev", None), ("stream_offset", -3)]:
        old = getattr(p, field)
        setattr(p, field, val)
        bad.append((field, call()))
        setattr(p, field, old)
    assert all(code == 1 for _, code in bad), bad
    for field, val in [("m", 0), ("n", -1), ("ld", 4)]:
        old = getattr(d, field)
        setattr(d, field, val)
        assert call() == 1, field
        setattr(d, field, old)
    d.dtype = 3
    assert call() == 2
    assert lib.rsk_workspace_size_dense(ctypes.byref(d), ctypes.byref(p), ctypes.byref(nb)) == 2
    d.dtype = 0
    assert lib.rsk_avg_solve_dense(None, 0x5000, ctypes.byref(p), 0x6000, 0x7000, 0x8000, 1 << 20, None) == 1
    assert lib.rsk_avg_solve_dense(ctypes.byref(d), None, ctypes.byref(p), 0x6000, 0x7000, 0x8000, 1 << 20,
                                   None) == 1


def test_batched_launch_choice_host_only():
    """rsk_plan_batched (host only): the register tile for a float32 batch whose systems all fit it
    (rows 16-byte aligned, ld % 4 == 0, eta <= 512), else the general kernel; kernel = 2 on a batch
    that does not fit is refused."""
    lib = _abi.load()

    def items(specs):
        arr = (_abi.RskBatchItem * len(specs))()
        for i, (m, n, ld, eta, base) in enumerate(specs):
            arr[i] = _abi.RskBatchItem(base, m, n, ld, 0x2000, 0x3000, 0x4000, 10, eta, 0, 1.0, 0.5, 0x5000, 0x6000,
                                       None, 0, 0.0, None, 0x7000)
        return arr

    def plan(specs, dtype=0, wg=0, kernel=0):
        arr = items(specs)
        k = ctypes.c_int32(-1)
        g = (ctypes.c_int32 * len(specs))()
        st = lib.rsk_plan_batched(len(specs), dtype, ctypes.addressof(arr), wg, kernel, ctypes.byref(k), g)
        return st, k.value, list(g)

    fits = [(4000, 2000, 2000, 201, 0x10000), (1000, 301, 304, 31, 0x20000), (600, 200, 200, 21, 0x30000)]
    st, k, g = plan(fits)
    assert st == 0 and k == 2, (st, k)
    # 2000 columns: 125 units of 16 floats, at most 10 a lane -> at least 13 slices; 201 rows of
    # 8000 bytes at 128 KiB a workgroup -> 13 workgroups
    assert g[0] == 13 and g[1] >= 2 and g[2] >= 2, g
    st, k, g = plan(fits, wg=16 << 10)
    assert st == 0 and k == 2 and g[0] == 99, g
    assert plan(fits, kernel=1)[:2] == (0, 1)
    for bad in [(4000, 2000, 2000, 600, 0x10000),  # eta > 512
                (1000, 301, 301, 31, 0x20000),      # ld % 4 != 0
                (1000, 300, 300, 31, 0x20004)]:     # rows not 16-byte aligned
        assert plan(fits + [bad])[:2] == (0, 1), bad
        assert plan(fits + [bad], kernel=2)[0] == 2, bad  # RSK_ERR_UNSUPPORTED
    assert plan(fits, dtype=1)[:2] == (0, 1)  # float64: general kernel
    assert plan(fits, dtype=1, kernel=2)[0] == 2
