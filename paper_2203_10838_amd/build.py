"""Build librsk.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2203_10838_amd.build  (or call ``build()``).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librsk.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # never let the compiler form packed fp32 arithmetic (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _filter(stderr: str) -> str:
    return "\n".join(l for l in (stderr or "").splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object in parallel (each translation unit holds its own
    kernels and device code), then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile

    srcs = sources()
    tmp = LIB + f".tmp{os.getpid()}"
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="rsk_build_") as objdir:
        def compile_one(src):
            obj = os.path.join(objdir, os.path.basename(src) + ".o")
            cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            return obj, subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(compile_one, srcs))
        for obj, res in results:
            err = _filter(res.stderr)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed ({res.returncode}) on {os.path.basename(obj)}:\n{err}")
            if verbose and err.strip():
                print(err, file=sys.stderr)
        cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *[o for o, _ in results], "-o", tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{_filter(res.stderr)}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
