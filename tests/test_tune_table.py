"""The library's tuning table on the host (no GPU needed): entries replace by key, erase and
clear, the text cache file round-trips, malformed lines are skipped, and RSK_TUNE_CACHE is read
at the first lookup of a fresh process."""
import ctypes
import os
import subprocess
import sys

from paper_2203_10838_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _e(path, dtype, m, n, eta, R, v0, v1, us=0.0, v2=0):
    return _abi.RskTuneEntry(path, dtype, m, n, eta, R, v0, v1, v2, us)


def _get(lib, key):
    out = _abi.RskTuneEntry()
    found = ctypes.c_int32(0)
    assert lib.rsk_tune_get(ctypes.byref(key), ctypes.byref(out), ctypes.byref(found)) == 0
    return out if found.value else None


def test_set_get_erase_clear_and_file_roundtrip(tmp_path):
    lib = _abi.load()
    lib.rsk_tune_clear(-1)
    try:
        d = _e(_abi.RSK_TUNE_DENSE, 0, 100000, 20000, 1024, 0, 2, 256, 20.5)
        assert lib.rsk_tune_set(ctypes.byref(d)) == 0
        assert lib.rsk_tune_set(ctypes.byref(_e(_abi.RSK_TUNE_DENSE, 0, 100000, 20000, 1024, 0, 3, 128, 19.0))) == 0
        got = _get(lib, d)
        assert (got.v0, got.v1, got.us) == (3, 128, 19.0)   # same key: replaced
        mr = _e(_abi.RSK_TUNE_MULTIRHS, 0, 32768, 8192, 820, 256, 24, 1, 101.0, v2=2)
        assert lib.rsk_tune_set(ctypes.byref(mr)) == 0
        for hi, wg in ((32 << 10, 16 << 10), (1 << 62, 64 << 10)):
            assert lib.rsk_tune_set(ctypes.byref(_e(_abi.RSK_TUNE_BATCHED, 0, hi, 0, 0, 0, wg, 0))) == 0
        # invalid entries are refused
        assert lib.rsk_tune_set(ctypes.byref(_e(7, 0, 1, 1, 1, 0, 1, 1))) == 1
        assert lib.rsk_tune_set(ctypes.byref(_e(_abi.RSK_TUNE_BATCHED, 0, 0, 0, 0, 0, 4096, 0))) == 1
        f = str(tmp_path / "tune.txt")
        assert lib.rsk_tune_save(f.encode()) == 0
        assert lib.rsk_tune_clear(-1) == 0 and _get(lib, d) is None
        with open(f, "a") as fh:
            fh.write("garbage line\n1 0 5 5\n# comment\n")
        assert lib.rsk_tune_load(f.encode()) == 0
        got = _get(lib, mr)
        assert (got.v0, got.v1, got.v2, got.us) == (24, 1, 2, 101.0)
        assert _get(lib, _e(_abi.RSK_TUNE_BATCHED, 0, 32 << 10, 0, 0, 0, 0, 0)).v0 == 16 << 10
        assert lib.rsk_tune_erase(ctypes.byref(mr)) == 0 and _get(lib, mr) is None
        assert _get(lib, d).v0 == 3
        assert lib.rsk_tune_clear(_abi.RSK_TUNE_DENSE) == 0 and _get(lib, d) is None
        assert _get(lib, _e(_abi.RSK_TUNE_BATCHED, 0, 1 << 62, 0, 0, 0, 0, 0)).v0 == 64 << 10
        assert lib.rsk_tune_load(str(tmp_path / "missing.txt").encode()) == 1
    finally:
        lib.rsk_tune_clear(-1)


def test_cache_named_by_the_environment_is_read_at_first_lookup(tmp_path):
    f = tmp_path / "env_tune.txt"
    f.write_text("# librsk tuning cache: path dtype m n eta R v0 v1 v2 us\n0 1 1000 500 10 0 1 4 0 12.5\n")
    code = (
        "import ctypes, sys; sys.path.insert(0, %r)\n"
        "from paper_2203_10838_amd import _abi\n"
        "lib = _abi.load()\n"
        "out = _abi.RskTuneEntry(); found = ctypes.c_int32(0)\n"
        "key = _abi.RskTuneEntry(0, 1, 1000, 500, 10, 0, 0, 0, 0, 0.0)\n"
        "assert lib.rsk_tune_get(ctypes.byref(key), ctypes.byref(out), ctypes.byref(found)) == 0\n"
        "print(found.value, out.v0, out.v1)\n" % ROOT)
    env = dict(os.environ, RSK_TUNE_CACHE=str(f))
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert res.stdout.split() == ["1", "1", "4"]
