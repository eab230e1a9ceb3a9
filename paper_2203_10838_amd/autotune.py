"""Autotuner: times candidate launches on the device and installs the winners in the library's
tuning table (rsk_tune_set), which the solves read whenever the caller leaves a choice to the
library (kernel = 0 / grid = 0 dense solves, the multi-RHS and adjoint product splits, the
batched per-system workgroup targets with wg_bytes = 0). ``save``/``load`` keep the table in a
text cache file; the library also loads the file named by RSK_TUNE_CACHE at its first lookup.

What is tuned, per key:
* dense (dtype, m, n, eta): the kernel (general; register tile with one or two row groups; one
  workgroup with the step in registers) and its workgroup count, among the launches rsk_plan_dense
  accepts;
* multi-RHS (dtype, m, n, eta, R): S, the column splits of A_tau X, and S2, the row splits of
  A_tau^T C;
* batched (dtype, size class of a system's step bytes eta*n*s, launch: general kernel or register
  tile): the row bytes per workgroup that set a system's workgroup count.

A candidate's time is the median of ``reps`` timed calls (HIP events on the current stream)
after one untimed call. Every candidate computes the same iteration: a tuned choice changes
speed, never the method (results equal the explicit choice's, bit for bit).
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional

import numpy as np
import torch

from . import _abi, rsk


def _entry(path, dtype, m=0, n=0, eta=0, R=0, v0=0, v1=0, v2=0, us=0.0) -> _abi.RskTuneEntry:
    return _abi.RskTuneEntry(int(path), int(dtype), int(m), int(n), int(eta), int(R), int(v0), int(v1), int(v2),
                             float(us))


def set_entry(path, dtype, *, m=0, n=0, eta=0, R=0, v0, v1=0, v2=0, us=0.0) -> None:
    st = rsk._lib().rsk_tune_set(ctypes.byref(_entry(path, dtype, m, n, eta, R, v0, v1, v2, us)))
    if st:
        raise rsk.RskError(st, "rsk_tune_set")


def get_entry(path, dtype, *, m=0, n=0, eta=0, R=0) -> Optional[dict]:
    key = _entry(path, dtype, m, n, eta, R)
    out = _abi.RskTuneEntry()
    found = ctypes.c_int32(0)
    st = rsk._lib().rsk_tune_get(ctypes.byref(key), ctypes.byref(out), ctypes.byref(found))
    if st:
        raise rsk.RskError(st, "rsk_tune_get")
    if not found.value:
        return None
    return {f: getattr(out, f) for f, _ in _abi.RskTuneEntry._fields_}


def erase(path, dtype, *, m=0, n=0, eta=0, R=0) -> None:
    """Remove the entry of one key (if any)."""
    st = rsk._lib().rsk_tune_erase(ctypes.byref(_entry(path, dtype, m, n, eta, R)))
    if st:
        raise rsk.RskError(st, "rsk_tune_erase")


def clear(path: int = -1) -> None:
    rsk._lib().rsk_tune_clear(int(path))


def save(path: str) -> None:
    st = rsk._lib().rsk_tune_save(str(path).encode())
    if st:
        raise rsk.RskError(st, "rsk_tune_save")


def load(path: str) -> None:
    st = rsk._lib().rsk_tune_load(str(path).encode())
    if st:
        raise rsk.RskError(st, "rsk_tune_load")


def _time_ms(fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    fn()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def dense_candidates(A: torch.Tensor, eta: int) -> list:
    """(kernel, grid) pairs the library accepts for A and eta (rsk_plan_dense), duplicates removed."""
    cus = torch.cuda.get_device_properties(A.device).multi_processor_count
    grids = sorted({g for g in (1, 2, 4, 8, 16, 24, 32, 48, 64, 96, 128, 160, 192, 224, 256, cus) if 1 <= g <= cus})
    seen, out = set(), []
    for kernel in (2, 3, 1, 4):
        for g in (grids if kernel != 4 else [1]):
            try:
                plan = rsk.plan_dense(A, eta=eta, grid=g, kernel=kernel)
            except rsk.RskError:
                continue
            sig = tuple(plan.values())
            if sig in seen:
                continue
            seen.add(sig)
            out.append((kernel, plan["G"]))
    return out


def tune_dense(A: torch.Tensor, b: torch.Tensor, *, eta: int, lam: float, alpha: float, index_stream: torch.Tensor,
               steps: int = 20, reps: int = 3, candidates: Optional[Iterable] = None, install: bool = True,
               rownorm2_t: Optional[torch.Tensor] = None) -> dict:
    """Time every (kernel, grid) candidate on ``steps`` steps of the given stream; install the fastest
    for (dtype, m, n, eta). Returns {"choice": (kernel, grid), "us_per_step", "default", "table"}."""
    m, n = A.shape
    dtype = rsk._dtype_code(A)
    r2 = rownorm2_t if rownorm2_t is not None else rsk.rownorm2(A)
    cands = list(candidates) if candidates is not None else dense_candidates(A, eta)
    x_star = torch.empty(n, dtype=A.dtype, device=A.device)

    def run(kernel, grid):
        return rsk.solve_dense(A, b, lam=lam, eta=eta, alpha=alpha, K=steps, index_stream=index_stream,
                               rownorm2_t=r2, kernel=kernel, grid=grid, x_star=x_star, check=False)

    prev = get_entry(_abi.RSK_TUNE_DENSE, dtype, m=m, n=n, eta=eta)
    erase(_abi.RSK_TUNE_DENSE, dtype, m=m, n=n, eta=eta)   # the built-in choice, timed without an entry
    default_plan = rsk.plan_dense(A, eta=eta)
    default_ms = _time_ms(lambda: run(0, 0), reps)
    table = []
    for kernel, grid in cands:
        ms = _time_ms(lambda: run(kernel, grid), reps)
        table.append({"kernel": kernel, "grid": grid, "us_per_step": ms * 1e3 / steps})
    best = min(table, key=lambda r: r["us_per_step"])
    if install:
        set_entry(_abi.RSK_TUNE_DENSE, dtype, m=m, n=n, eta=eta, v0=best["kernel"], v1=best["grid"],
                  us=best["us_per_step"])
    elif prev is not None:
        set_entry(_abi.RSK_TUNE_DENSE, dtype, m=m, n=n, eta=eta, v0=prev["v0"], v1=prev["v1"], us=prev["us"])
    return {"choice": (best["kernel"], best["grid"]), "us_per_step": best["us_per_step"],
            "default": {"plan": default_plan, "us_per_step": default_ms * 1e3 / steps}, "table": table}


def multirhs_candidates(A: torch.Tensor, R: int, eta: int) -> list:
    """(S, S2) pairs: column splits of A_tau X (at least 64 columns a split) and row splits of A_tau^T C.
    Besides powers of two and whole XCD rounds, the splits that put one wide-tile workgroup on each CU
    (CUs / tiles and one less)."""
    n = A.shape[1]
    max_s = max(1, (n + 63) // 64)        # a tuned split keeps at least 64 columns (one stage)
    cus = torch.cuda.get_device_properties(A.device).multi_processor_count if A.is_cuda else 256
    tiles = -(-eta // 128) * (-(-R // 128) if R > 64 else 1)
    fill = cus // tiles
    svals = sorted({s for s in (1, 2, 4, 8, 16, 24, 32, 48, 64, 96, 128, fill, fill - 1) if 1 <= s <= max_s})
    s2vals = [s2 for s2 in (1, 2, 4, 8) if s2 <= max(1, (eta + 15) // 16)]
    return [(s, s2, kernel) for kernel in (1, 2, 3) for s in svals for s2 in s2vals]


def tune_multirhs(A: torch.Tensor, B: torch.Tensor, *, eta: int, lam: float, alpha: float,
                  index_stream: torch.Tensor, steps: int = 4, reps: int = 3, candidates: Optional[Iterable] = None,
                  install: bool = True, rownorm2_t: Optional[torch.Tensor] = None) -> dict:
    """Time (S, S2, kernel) candidates of the multi-RHS forward (kernel 1: step kernels, 2: one persistent
    launch, 3: step kernels with wide product tiles); install the fastest for (dtype, m, n, eta, R)."""
    m, n = A.shape
    R = B.shape[1]
    dtype = rsk._dtype_code(A)
    r2 = rownorm2_t if rownorm2_t is not None else rsk.rownorm2(A)
    prev = get_entry(_abi.RSK_TUNE_MULTIRHS, dtype, m=m, n=n, eta=eta, R=R)
    X_star = torch.empty((n, R), dtype=A.dtype, device=A.device)

    def run():
        return rsk.solve_multirhs(A, B, lam=lam, eta=eta, alpha=alpha, K=steps, index_stream=index_stream,
                                  rownorm2_t=r2, X_star=X_star, check=False)

    erase(_abi.RSK_TUNE_MULTIRHS, dtype, m=m, n=n, eta=eta, R=R)   # the built-in split, without an entry
    default_plan = rsk.plan_multirhs(A, R, eta=eta, K=steps)
    default_ms = _time_ms(run, reps)
    table = []
    seen = set()
    for cand in (list(candidates) if candidates is not None else multirhs_candidates(A, R, eta)):
        S, S2, kernel = (tuple(cand) + (1,))[:3]
        set_entry(_abi.RSK_TUNE_MULTIRHS, dtype, m=m, n=n, eta=eta, R=R, v0=S, v1=S2, v2=kernel)
        plan = rsk.plan_multirhs(A, R, eta=eta, K=steps)
        sig = (plan["S"], plan["S2"], plan["kernel"])
        if sig in seen:
            continue
        seen.add(sig)
        try:
            ms = _time_ms(run, reps)
        except rsk.RskError:
            continue
        table.append({"S": S, "S2": plan["S2"], "kernel": plan["kernel"], "us_per_step": ms * 1e3 / steps})
    best = min(table, key=lambda r: r["us_per_step"])
    if install:
        set_entry(_abi.RSK_TUNE_MULTIRHS, dtype, m=m, n=n, eta=eta, R=R, v0=best["S"], v1=best["S2"],
                  v2=best["kernel"], us=best["us_per_step"])
    elif prev is not None:
        set_entry(_abi.RSK_TUNE_MULTIRHS, dtype, m=m, n=n, eta=eta, R=R, v0=prev["v0"], v1=prev["v1"], v2=prev["v2"],
                  us=prev["us"])
    else:
        erase(_abi.RSK_TUNE_MULTIRHS, dtype, m=m, n=n, eta=eta, R=R)
    return {"choice": (best["S"], best["S2"], best["kernel"]), "us_per_step": best["us_per_step"],
            "default": {"plan": default_plan, "us_per_step": default_ms * 1e3 / steps}, "table": table}


BATCH_CLASS_BOUNDS = (32 << 10, 128 << 10, 512 << 10, 2 << 20, 8 << 20, 1 << 62)
BATCH_CANDIDATES_KIB = (8, 16, 24, 32, 48, 64, 96, 128)
BATCH_RT_CANDIDATES_KIB = (16, 32, 64, 128, 256)


def tune_batched(systems, *, bounds=BATCH_CLASS_BOUNDS, candidates_kib=None, reps: int = 2, kernel: int = 0,
                 install: bool = True) -> dict:
    """Per size class of a system's step bytes (eta * n * element bytes, classes ending at ``bounds``):
    the systems of that class run as one batch for each candidate target of row bytes per
    workgroup; the fastest target is installed for the class and the launch (``kernel`` 1 general,
    2 register tile, 0 the launch the library picks for the whole batch). Systems of other classes
    are not in the timed batch (a class is tuned on its own). Returns the per-class table."""
    if not systems:
        raise ValueError("empty batch")
    dtype = rsk._dtype_code(systems[0].A)
    es = systems[0].A.element_size()
    if kernel == 0:
        kernel = rsk.plan_batched(systems)["kernel"]
    if candidates_kib is None:
        candidates_kib = BATCH_RT_CANDIDATES_KIB if kernel == 2 else BATCH_CANDIDATES_KIB
    step = [s.eta * s.A.shape[1] * es for s in systems]
    out, lo = [], 0
    for hi in bounds:
        members = [s for s, b in zip(systems, step) if lo < b <= hi]
        lo = hi
        if not members:
            continue
        rows = []
        for kib in candidates_kib:
            try:
                rsk.solve_batched(members, wg_bytes=kib << 10, kernel=kernel, check=False)
            except rsk.RskError:
                continue
            ms = _time_ms(lambda: rsk.solve_batched(members, wg_bytes=kib << 10, kernel=kernel, check=False), reps)
            rows.append({"wg_kib": kib, "ms": ms})
        if not rows:
            continue
        best = min(rows, key=lambda r: r["ms"])
        out.append({"step_bytes_hi": hi, "systems": len(members), "wg_kib": best["wg_kib"], "ms": best["ms"],
                    "table": rows})
        if install:
            set_entry(_abi.RSK_TUNE_BATCHED, dtype, m=hi, R=2 if kernel == 2 else 0, v0=best["wg_kib"] << 10,
                      us=best["ms"] * 1e3)
    return {"kernel": kernel, "classes": out}
