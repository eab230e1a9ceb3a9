"""The library's host code (validation, planners, workspace queries, tuning table and its cache
file) under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

Every source of the library is compiled with the sanitizers on its host part only (the device
code is built as usual and never runs), linked with `host_sanitizer/rsk_host_check.c`, and that
program is run: it makes several thousand host-only calls, each checked against its documented
status code, and any sanitizer finding ends it with a non-zero status.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_10838_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "host_sanitizer", "rsk_host_check.c")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
# sanitizer flags for the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run_all(cmds, jobs=8):
    procs, fails = [], []
    for cmd in cmds:
        while len(procs) >= jobs:
            p = procs.pop(0)
            if p.wait() != 0:
                fails.append((p.args, p.stderr.read()))
        procs.append(subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True))
    for p in procs:
        if p.wait() != 0:
            fails.append((p.args, p.stderr.read()))
    return fails


@pytest.mark.timeout(900)
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not installed")
    objs, cmds = [], []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        objs.append(obj)
        cmds.append([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
                     f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj])
    drv = str(tmp_path / "rsk_host_check.o")
    cmds.append([CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=all", f"-I{INCLUDE}", "-c", DRIVER, "-o", drv])
    fails = _run_all(cmds, jobs=min(8, os.cpu_count() or 1))
    assert not fails, fails[0]
    # the library's host code really carries both sanitizers' checks
    nm_tool = shutil.which("nm") or "/usr/bin/nm"
    nm = subprocess.run([nm_tool, str(tmp_path / "rsk_api.o")], capture_output=True, text=True)
    assert "__asan_report" in nm.stdout and "__ubsan_handle" in nm.stdout
    exe = str(tmp_path / "rsk_host_check")
    link = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", drv, *objs, "-o", exe], capture_output=True, text=True)
    assert link.returncode == 0, link.stderr
    run_dir = tmp_path / "run"
    run_dir.mkdir()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("RSK_TUNE_CACHE", None)
    res = subprocess.run([exe, str(run_dir)], capture_output=True, text=True, timeout=600, env=env, cwd=str(tmp_path))
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 failed" in res.stdout, out[-4000:]
