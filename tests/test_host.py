"""Host-side behaviour that needs no GPU: the benchmark's one-GPU contract and the binding's
refusal to run without the HIP library (there is no CPU fallback)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd="/tmp")
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert '"metric"' not in r.stdout  # no benchmark line for a configuration it does not run


def test_binding_without_library_fails_loudly(monkeypatch):
    from paper_2203_10838_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _abi.load(os.path.join(ROOT, "no_such_dir", "librsk.so"))


def test_solver_entry_needs_the_library(monkeypatch):
    """The Python solve functions reach the kernels only through the C ABI: with no library they
    raise instead of computing anything on the host."""
    from paper_2203_10838_amd import _abi, rsk
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "librsk.so"))
    load = _abi.load
    monkeypatch.setattr(_abi, "load", lambda path=_abi.LIB_PATH: load(path))
    with pytest.raises(RuntimeError, match="not built"):
        rsk._lib()
