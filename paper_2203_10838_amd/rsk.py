"""Python binding of librsk over torch device tensors.

Argument marshalling only: every step of the method runs in the HIP library.
Tensors must live on the GPU; there is no CPU path. Names follow include/rsk.h
and the paper's notation (lambda -> ``lam``, eta, alpha, K, tau -> ``index_stream``).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _abi


class RskError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = int(code)
        self.name = _abi.STATUS_NAMES.get(self.code, f"code {code}")
        super().__init__(f"{where}: {self.name}")


def _lib():
    return _abi.load()


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return _abi.RSK_F32
    if t.dtype == torch.float64:
        return _abi.RSK_F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _dev(t: Optional[torch.Tensor], name: str, dtype=None, numel=None) -> int:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def dense_desc(A: torch.Tensor) -> _abi.RskDense:
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    if not A.is_cuda:
        raise TypeError("A must be a GPU tensor")
    if A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise ValueError("A must be row-major with leading dimension >= n")
    return _abi.RskDense(A.shape[0], A.shape[1], A.stride(0), _dtype_code(A), A.data_ptr())


def rownorm2(A: torch.Tensor) -> torch.Tensor:
    """||a_i||^2 of every row of a dense A (Definition 1's D, squared)."""
    d = dense_desc(A)
    out = torch.empty(A.shape[0], dtype=A.dtype, device=A.device)
    st = _lib().rsk_rownorm2_dense(ctypes.byref(d), out.data_ptr(), _stream())
    if st:
        raise RskError(st, "rsk_rownorm2_dense")
    return out


@dataclass
class SolveResult:
    x_star: torch.Tensor
    x: torch.Tensor
    status: Optional[int]
    k_done: Optional[int]
    err_hist: Optional[torch.Tensor]
    status_dev: torch.Tensor


def make_params(*, lam, eta, alpha, K, index_stream, rownorm2_t, status_dev, stream_offset=0, alpha_k=None,
                warm_start=False, x_ref=None, check_every=0, tol=0.0, err_hist=None, y_out=None, grid=0,
                kernel=0, dtype=None, row_w=None) -> _abi.RskParams:
    if K > 0:
        _dev(index_stream, "index_stream", torch.int32, stream_offset + K * eta)
    return _abi.RskParams(
        float(lam), int(eta), float(alpha),
        _dev(alpha_k, "alpha_k", dtype, K if K > 0 else None),
        int(K), _dev(index_stream, "index_stream") if index_stream is not None else None, int(stream_offset),
        _dev(rownorm2_t, "rownorm2", dtype), 1 if warm_start else 0,
        _dev(x_ref, "x_ref", dtype), int(check_every), float(tol),
        _dev(err_hist, "err_hist", torch.float64), _dev(y_out, "y_out", dtype),
        _dev(status_dev, "status_dev", torch.int32, 2), int(grid), int(kernel), _dev(row_w, "row_w", dtype))


def workspace_size_dense(A: torch.Tensor, params: _abi.RskParams) -> int:
    d = dense_desc(A)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_dense(ctypes.byref(d), ctypes.byref(params), ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_dense")
    return int(nbytes.value)


PLAN_FIELDS = ("kernel", "G", "threads", "row_passes", "chunks_per_lane", "row_groups", "hops", "vec", "row_tile")


def plan_dense(A: torch.Tensor, *, eta: int, K: int = 1, grid: int = 0, kernel: int = 0, lam: float = 0.0,
               alpha: float = 1.0) -> dict:
    """The launch rsk_avg_solve_dense would make for A, eta, grid and kernel (nothing is queued):
    the kernel (1 general, 2 register tile, 3 register tile over two row groups), its workgroups,
    threads, row passes and chunks per lane, row groups, exchange hops, vector width and the
    general kernel's row tile (0 none, 1 in LDS, 2 two LDS tiles loaded a step ahead)."""
    d = dense_desc(A)
    dummy = torch.empty(2, dtype=torch.int32, device=A.device)
    params = _abi.RskParams(float(lam), int(eta), float(alpha), None, int(K), dummy.data_ptr(), 0,
                            A.data_ptr(), 0, None, 0, 0.0, None, None, dummy.data_ptr(), int(grid), int(kernel), None)
    out = (ctypes.c_int32 * 9)()
    st = _lib().rsk_plan_dense(ctypes.byref(d), ctypes.byref(params), out)
    if st:
        raise RskError(st, "rsk_plan_dense")
    return dict(zip(PLAN_FIELDS, [int(v) for v in out]))


def gather_rate(A: torch.Tensor, index_stream: torch.Tensor, *, eta: int, K: int, grid: int = 256,
                row_groups: int = 1, layout: int = 0, stream_offset: int = 0) -> torch.Tensor:
    """Queue the gather of a float32 register-tile solve alone (rsk_gather_rate_dense): K steps of
    the sampled rows' column slices that ``grid`` workgroups in ``row_groups`` row groups would
    read, no exchange, no update; ``layout`` 0 reads whole pieces per instruction, 1 the register
    tile's lanes. Returns the sink (grid * 512 floats); time the call with events."""
    d = dense_desc(A)
    _dev(index_stream, "index_stream", torch.int32, stream_offset + K * eta)
    sink = torch.empty(grid * 512, dtype=torch.float32, device=A.device)
    st = _lib().rsk_gather_rate_dense(ctypes.byref(d), index_stream.data_ptr() + 4 * stream_offset, int(eta), int(K),
                                      int(grid), int(row_groups), int(layout), sink.data_ptr(), _stream())
    if st:
        raise RskError(st, "rsk_gather_rate_dense")
    return sink


def plan_multirhs(A: torch.Tensor, R: int, *, eta: int, K: int = 1, kernel: int = 0) -> dict:
    """The split rsk_avg_solve_multirhs would use (nothing is queued): S column splits of A_tau X
    (and the columns per split), S2 row splits of A_tau^T C, eta padded to a multiple of the
    product tile edge (64, or 128 for kernel 3), the kernel."""
    d = dense_desc(A)
    dummy = torch.empty(2, dtype=torch.int32, device=A.device)
    params = _abi.RskParams(0.0, int(eta), 1.0, None, int(K), dummy.data_ptr(), 0, A.data_ptr(), 0, None, 0, 0.0,
                            None, None, dummy.data_ptr(), 0, int(kernel), None)
    out = (ctypes.c_int32 * 5)()
    st = _lib().rsk_plan_multirhs(ctypes.byref(d), int(R), ctypes.byref(params), out)
    if st:
        raise RskError(st, "rsk_plan_multirhs")
    return dict(zip(("S", "kspan", "S2", "eta_pad", "kernel"), [int(v) for v in out]))


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def solve_dense(A: torch.Tensor, b: torch.Tensor, *, lam: float, eta: int, alpha: float, K: int,
                index_stream: torch.Tensor, stream_offset: int = 0, alpha_k: Optional[torch.Tensor] = None,
                rownorm2_t: Optional[torch.Tensor] = None, x_star: Optional[torch.Tensor] = None,
                warm_start: bool = False, x_ref: Optional[torch.Tensor] = None, check_every: int = 0,
                tol: float = 0.0, y_out: Optional[torch.Tensor] = None, grid: int = 0, kernel: int = 0,
                row_w: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                check: bool = True, noalloc: bool = False) -> SolveResult:
    """K steps of RSKA (eq. (rska), Algorithm 1) on a dense system, one persistent launch.

    ``noalloc``: call rsk_avg_solve_dense_noalloc, whose exchange scratch is the library's static
    per-GPU array (no workspace; calls that overlap on one GPU race).

    ``row_w`` (m, optional): per-row weights w_i of Definition 1 (variants v3/v4 of Sec. 5);
    row i is then relaxed by alpha (or alpha_k[k]) times w_i.

    ``kernel``: 0 library's choice, 1 general, 2 float32 register tile, 3 register tile over two
    row groups (half of a step's rows per workgroup over slices twice as wide).

    ``x_star`` (optional, in/out) receives x*_K; with ``warm_start`` it is also x*_0.
    With ``check`` the call synchronises, reads the device status and raises
    ``RskError`` on a device-side fault.
    """
    m, n = A.shape
    dt = A.dtype
    _dev(b, "b", dt, m)
    if rownorm2_t is None:
        rownorm2_t = rownorm2(A)
    if x_star is None:
        if warm_start:
            raise ValueError("warm_start needs x_star")
        x_star = torch.empty(n, dtype=dt, device=A.device)
    _dev(x_star, "x_star", dt, n)
    x = torch.empty(n, dtype=dt, device=A.device)
    status_dev = torch.empty(2, dtype=torch.int32, device=A.device)
    nh = (K // check_every) if (x_ref is not None and check_every > 0) else 0
    err_hist = torch.full((max(nh, 1),), float("nan"), dtype=torch.float64, device=A.device) if nh else None
    params = make_params(lam=lam, eta=eta, alpha=alpha, K=K, index_stream=index_stream, rownorm2_t=rownorm2_t,
                         status_dev=status_dev, stream_offset=stream_offset, alpha_k=alpha_k,
                         warm_start=warm_start, x_ref=x_ref, check_every=check_every, tol=tol, err_hist=err_hist,
                         y_out=y_out, grid=grid, kernel=kernel, dtype=dt, row_w=row_w)
    if row_w is not None:
        _dev(row_w, "row_w", dt, m)
    if y_out is not None:
        _dev(y_out, "y_out", dt, m)
    d = dense_desc(A)
    if noalloc:
        st = _lib().rsk_avg_solve_dense_noalloc(ctypes.byref(d), b.data_ptr(), ctypes.byref(params),
                                                x_star.data_ptr(), x.data_ptr(), _stream())
        if st:
            raise RskError(st, "rsk_avg_solve_dense_noalloc")
    else:
        need = workspace_size_dense(A, params)
        if workspace is None or workspace.numel() < need:
            workspace = _workspace(need, A.device)
        st = _lib().rsk_avg_solve_dense(ctypes.byref(d), b.data_ptr(), ctypes.byref(params), x_star.data_ptr(),
                                        x.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream())
        if st:
            raise RskError(st, "rsk_avg_solve_dense")
    status = k_done = None
    if check:
        s = status_dev.cpu().tolist()
        status, k_done = int(s[0]), int(s[1])
        if status:
            raise RskError(status, "rsk_avg_solve_dense (device)")
    return SolveResult(x_star, x, status, k_done, err_hist, status_dev)


# ---------------------------------------------------------------------------
# CSR
# ---------------------------------------------------------------------------

def csr_desc(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n: int) -> _abi.RskCsr:
    _dev(row_ptr, "row_ptr", torch.int64)
    _dev(col, "col", torch.int32)
    _dev(val, "val")
    m = row_ptr.numel() - 1
    return _abi.RskCsr(m, int(n), col.numel(), _dtype_code(val), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())


def rownorm2_csr(row_ptr, col, val, n) -> torch.Tensor:
    """||a_i||^2 of every CSR row."""
    d = csr_desc(row_ptr, col, val, n)
    out = torch.empty(d.m, dtype=val.dtype, device=val.device)
    st = _lib().rsk_rownorm2_csr(ctypes.byref(d), out.data_ptr(), _stream())
    if st:
        raise RskError(st, "rsk_rownorm2_csr")
    return out


def solve_csr(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n: int, b: torch.Tensor, *, lam: float,
              eta: int, alpha: float, K: int, index_stream: torch.Tensor, stream_offset: int = 0,
              alpha_k: Optional[torch.Tensor] = None, rownorm2_t: Optional[torch.Tensor] = None,
              x_star: Optional[torch.Tensor] = None, warm_start: bool = False, x_ref: Optional[torch.Tensor] = None,
              check_every: int = 0, tol: float = 0.0, y_out: Optional[torch.Tensor] = None,
              grid: int = 0, kernel: int = 0, row_w: Optional[torch.Tensor] = None,
              workspace: Optional[torch.Tensor] = None, check: bool = True) -> SolveResult:
    """K steps of RSKA on a CSR system (kernel 1: one workgroup, 2: multi-workgroup, 0: by eta)."""
    d = csr_desc(row_ptr, col, val, n)
    dt = val.dtype
    dev = val.device
    _dev(b, "b", dt, d.m)
    if rownorm2_t is None:
        rownorm2_t = rownorm2_csr(row_ptr, col, val, n)
    if x_star is None:
        if warm_start:
            raise ValueError("warm_start needs x_star")
        x_star = torch.empty(n, dtype=dt, device=dev)
    _dev(x_star, "x_star", dt, n)
    x = torch.empty(n, dtype=dt, device=dev)
    status_dev = torch.empty(2, dtype=torch.int32, device=dev)
    nh = (K // check_every) if (x_ref is not None and check_every > 0) else 0
    err_hist = torch.full((max(nh, 1),), float("nan"), dtype=torch.float64, device=dev) if nh else None
    params = make_params(lam=lam, eta=eta, alpha=alpha, K=K, index_stream=index_stream, rownorm2_t=rownorm2_t,
                         status_dev=status_dev, stream_offset=stream_offset, alpha_k=alpha_k, warm_start=warm_start,
                         x_ref=x_ref, check_every=check_every, tol=tol, err_hist=err_hist, y_out=y_out, grid=grid,
                         kernel=kernel, dtype=dt, row_w=row_w)
    if row_w is not None:
        _dev(row_w, "row_w", dt, d.m)
    if y_out is not None:
        _dev(y_out, "y_out", dt, d.m)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_csr(ctypes.byref(d), ctypes.byref(params), ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_csr")
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = _workspace(nbytes.value, dev)
    st = _lib().rsk_avg_solve_csr(ctypes.byref(d), b.data_ptr(), ctypes.byref(params), x_star.data_ptr(),
                                  x.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream())
    if st:
        raise RskError(st, "rsk_avg_solve_csr")
    status = k_done = None
    if check:
        s = status_dev.cpu().tolist()
        status, k_done = int(s[0]), int(s[1])
        if status:
            raise RskError(status, "rsk_avg_solve_csr (device)")
    return SolveResult(x_star, x, status, k_done, err_hist, status_dev)


# ---------------------------------------------------------------------------
# Many right-hand sides sharing A and the stream (matrix cores)
# ---------------------------------------------------------------------------

def solve_multirhs(A: torch.Tensor, B: torch.Tensor, *, lam: float, eta: int, alpha: float, K: int,
                   index_stream: torch.Tensor, stream_offset: int = 0, alpha_k: Optional[torch.Tensor] = None,
                   rownorm2_t: Optional[torch.Tensor] = None, X_star: Optional[torch.Tensor] = None,
                   warm_start: bool = False, workspace: Optional[torch.Tensor] = None,
                   ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                   row_w: Optional[torch.Tensor] = None, kernel: int = 0, check: bool = True) -> SolveResult:
    """K RSKA steps for the R columns of B (m x R) at once; X*, X are n x R (row-major).

    ``kernel``: 1 the step kernels, 2 one persistent launch for all K steps, 3 the step kernels with
    wide product tiles, 0 the library's choice (a tuned one, else 3 when R > 64 and eta >= 128, else 1).

    With ``ckpt`` (ceil(K/ckpt_every) x n x R float32) the x* checkpoints the
    adjoint recomputes from are written as well.
    """
    m, n = A.shape
    if B.dim() != 2 or B.shape[0] != m:
        raise ValueError("B must be m x R")
    R = B.shape[1]
    dt = A.dtype
    _dev(B, "B", dt)
    if rownorm2_t is None:
        rownorm2_t = rownorm2(A)
    if X_star is None:
        if warm_start:
            raise ValueError("warm_start needs X_star")
        X_star = torch.empty((n, R), dtype=dt, device=A.device)
    _dev(X_star, "X_star", dt, n * R)
    X = torch.empty((n, R), dtype=dt, device=A.device)
    status_dev = torch.empty(2, dtype=torch.int32, device=A.device)
    params = make_params(lam=lam, eta=eta, alpha=alpha, K=K, index_stream=index_stream, rownorm2_t=rownorm2_t,
                         status_dev=status_dev, stream_offset=stream_offset, alpha_k=alpha_k, warm_start=warm_start,
                         dtype=dt, row_w=row_w, kernel=kernel)
    if row_w is not None:
        _dev(row_w, "row_w", dt, m)
    d = dense_desc(A)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_multirhs(ctypes.byref(d), R, ctypes.byref(params), ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_multirhs")
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = _workspace(nbytes.value, A.device)
    if ckpt is not None:
        if ckpt_every < 1:
            raise ValueError("ckpt needs ckpt_every >= 1")
        _dev(ckpt, "ckpt", dt, max(1, -(-K // ckpt_every)) * n * R)
        st = _lib().rsk_avg_solve_multirhs_ckpt(ctypes.byref(d), B.data_ptr(), R, ctypes.byref(params),
                                                int(ckpt_every), X_star.data_ptr(), X.data_ptr(), ckpt.data_ptr(),
                                                workspace.data_ptr(), workspace.numel(), _stream())
    else:
        st = _lib().rsk_avg_solve_multirhs(ctypes.byref(d), B.data_ptr(), R, ctypes.byref(params),
                                           X_star.data_ptr(), X.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                           _stream())
    if st:
        raise RskError(st, "rsk_avg_solve_multirhs")
    status = k_done = None
    if check:
        s = status_dev.cpu().tolist()
        status, k_done = int(s[0]), int(s[1])
        if status:
            raise RskError(status, "rsk_avg_solve_multirhs (device)")
    return SolveResult(X_star, X, status, k_done, None, status_dev)


@dataclass
class AdjointResult:
    Bbar: torch.Tensor
    lambda_bar: torch.Tensor
    alpha_bar: torch.Tensor
    status_dev: torch.Tensor


def adjoint_multirhs(A: torch.Tensor, B: torch.Tensor, *, lam: float, eta: int, alpha_k: torch.Tensor, K: int,
                     index_stream: torch.Tensor, ckpt: torch.Tensor, ckpt_every: int, X_star_K: torch.Tensor,
                     Xbar_K: torch.Tensor, stream_offset: int = 0, rownorm2_t: Optional[torch.Tensor] = None,
                     workspace: Optional[torch.Tensor] = None, check: bool = True) -> AdjointResult:
    """dL/dB, dL/dlambda, dL/dalpha_k of K unrolled multi-RHS steps, given Xbar_K = dL/dx_K."""
    m, n = A.shape
    R = B.shape[1]
    dt = A.dtype
    _dev(B, "B", dt, m * R)
    _dev(X_star_K, "X_star_K", dt, n * R)
    _dev(Xbar_K, "Xbar_K", dt, n * R)
    _dev(alpha_k, "alpha_k", dt, K)
    if rownorm2_t is None:
        rownorm2_t = rownorm2(A)
    status_dev = torch.empty(2, dtype=torch.int32, device=A.device)
    params = make_params(lam=lam, eta=eta, alpha=1.0, K=K, index_stream=index_stream, rownorm2_t=rownorm2_t,
                         status_dev=status_dev, stream_offset=stream_offset, alpha_k=alpha_k, dtype=dt)
    d = dense_desc(A)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_adjoint(ctypes.byref(d), R, ctypes.byref(params), int(ckpt_every),
                                           ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_adjoint")
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = _workspace(nbytes.value, A.device)
    Bbar = torch.empty((m, R), dtype=dt, device=A.device)
    lbar = torch.zeros(1, dtype=torch.float64, device=A.device)
    abar = torch.zeros(max(K, 1), dtype=dt, device=A.device)
    st = _lib().rsk_avg_adjoint(ctypes.byref(d), B.data_ptr(), R, ctypes.byref(params), int(ckpt_every),
                                ckpt.data_ptr(), X_star_K.data_ptr(), Xbar_K.data_ptr(), Bbar.data_ptr(),
                                lbar.data_ptr(), abar.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream())
    if st:
        raise RskError(st, "rsk_avg_adjoint")
    if check:
        s = int(status_dev[0].item())
        if s:
            raise RskError(s, "rsk_avg_adjoint (device)")
    return AdjointResult(Bbar, lbar, abar[:K], status_dev)


# ---------------------------------------------------------------------------
# Row sampler
# ---------------------------------------------------------------------------

def _cdf_workspace(m: int, device) -> torch.Tensor:
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_sampling_cdf(int(m), ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_sampling_cdf")
    return _workspace(nbytes.value, device)


def sampling_cdf(A: torch.Tensor, row_w: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Running sums of the FP64 row norms ||a_i||^2 on the device (m doubles); with ``row_w``
    the sums of ||a_i||^2 / w_i (variant v4's probabilities, Sec. 5)."""
    d = dense_desc(A)
    ws = _cdf_workspace(d.m, A.device)
    cdf = torch.empty(A.shape[0], dtype=torch.float64, device=A.device)
    if row_w is None:
        st = _lib().rsk_sampling_cdf_dense(ctypes.byref(d), cdf.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    else:
        _dev(row_w, "row_w", A.dtype, A.shape[0])
        st = _lib().rsk_sampling_cdf_dense_weighted(ctypes.byref(d), row_w.data_ptr(), cdf.data_ptr(), ws.data_ptr(),
                                                    ws.numel(), _stream())
    if st:
        raise RskError(st, "rsk_sampling_cdf_dense")
    return cdf


def sampling_cdf_weights(weights: torch.Tensor) -> torch.Tensor:
    """Running sums of arbitrary non-negative FP64 weights on the device (m doubles)."""
    _dev(weights, "weights", torch.float64)
    ws = _cdf_workspace(weights.numel(), weights.device)
    cdf = torch.empty(weights.numel(), dtype=torch.float64, device=weights.device)
    st = _lib().rsk_sampling_cdf_weights(weights.data_ptr(), weights.numel(), cdf.data_ptr(), ws.data_ptr(),
                                         ws.numel(), _stream())
    if st:
        raise RskError(st, "rsk_sampling_cdf_weights")
    return cdf


def sample_stream(cdf: torch.Tensor, *, seed: int, K: int, eta: int, k0: int = 0,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K*eta row indices (steps k0 .. k0+K-1) from Philox4x32-10 and the inverse CDF, on the device."""
    _dev(cdf, "cdf", torch.float64)
    m = cdf.numel()
    if out is None:
        out = torch.empty(max(K * eta, 1), dtype=torch.int32, device=cdf.device)
    _dev(out, "out", torch.int32, K * eta)
    st = _lib().rsk_sample_stream(cdf.data_ptr(), m, int(seed) & ((1 << 64) - 1), int(k0), int(K), int(eta),
                                  out.data_ptr(), _stream())
    if st:
        raise RskError(st, "rsk_sample_stream")
    return out[:K * eta]


# ---------------------------------------------------------------------------
# Linearized Bregman (full-batch comparator) and sigma_max(A)^2
# ---------------------------------------------------------------------------

def _lb_workspace(A: torch.Tensor, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    d = dense_desc(A)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_lb_dense(ctypes.byref(d), ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_lb_dense")
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = _workspace(nbytes.value, A.device)
    return workspace


def spectral_norm2(A: torch.Tensor, iters: int = 100, *, v: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None) -> float:
    """sigma_max(A)^2 by power iteration on A^T A (on the device); ``v`` receives the last unit vector."""
    d = dense_desc(A)
    ws = _lb_workspace(A, workspace)
    if v is None:
        v = torch.empty(A.shape[1], dtype=A.dtype, device=A.device)
    _dev(v, "v", A.dtype, A.shape[1])
    est = torch.empty(1, dtype=torch.float64, device=A.device)
    st = _lib().rsk_spectral_norm2_dense(ctypes.byref(d), int(iters), v.data_ptr(), est.data_ptr(), ws.data_ptr(),
                                         ws.numel(), _stream())
    if st:
        raise RskError(st, "rsk_spectral_norm2_dense")
    return float(est.item())


@dataclass
class LbResult:
    x_star: torch.Tensor
    x: torch.Tensor
    status: Optional[int]
    k_done: Optional[int]
    err_hist: Optional[torch.Tensor]
    res_hist: Optional[torch.Tensor]


def lb_solve(A: torch.Tensor, b: torch.Tensor, *, lam: float, step: float, K: int,
             x_star: Optional[torch.Tensor] = None, warm_start: bool = False, x_ref: Optional[torch.Tensor] = None,
             check_every: int = 0, residuals: bool = False, workspace: Optional[torch.Tensor] = None,
             check: bool = True) -> LbResult:
    """K linearized Bregman iterations x* -= step A^T(Ax - b), x = S_lambda(x*), each reading A once."""
    m, n = A.shape
    dt = A.dtype
    _dev(b, "b", dt, m)
    if x_star is None:
        if warm_start:
            raise ValueError("warm_start needs x_star")
        x_star = torch.empty(n, dtype=dt, device=A.device)
    _dev(x_star, "x_star", dt, n)
    x = torch.empty(n, dtype=dt, device=A.device)
    status_dev = torch.empty(2, dtype=torch.int32, device=A.device)
    nh = (K // check_every) if (x_ref is not None and check_every > 0) else 0
    err_hist = torch.full((max(nh, 1),), float("nan"), dtype=torch.float64, device=A.device) if nh else None
    res_hist = torch.full((max(K, 1),), float("nan"), dtype=torch.float64, device=A.device) if residuals else None
    p = _abi.RskLbParams(float(lam), float(step), int(K), 1 if warm_start else 0, _dev(x_ref, "x_ref", dt, n),
                         int(check_every), _dev(err_hist, "err_hist"), _dev(res_hist, "res_hist"),
                         status_dev.data_ptr())
    d = dense_desc(A)
    ws = _lb_workspace(A, workspace)
    st = _lib().rsk_lb_solve_dense(ctypes.byref(d), b.data_ptr(), ctypes.byref(p), x_star.data_ptr(), x.data_ptr(),
                                   ws.data_ptr(), ws.numel(), _stream())
    if st:
        raise RskError(st, "rsk_lb_solve_dense")
    status = k_done = None
    if check:
        s = status_dev.cpu().tolist()
        status, k_done = int(s[0]), int(s[1])
        if status:
            raise RskError(status, "rsk_lb_solve_dense (device)")
    return LbResult(x_star, x, status, k_done, err_hist, None if res_hist is None else res_hist[:K])


@dataclass
class BskResult:
    x_star: torch.Tensor
    x: torch.Tensor
    status: Optional[int]
    k_done: Optional[int]
    err_hist: Optional[torch.Tensor]
    block_norm2: Optional[torch.Tensor]


def bsk_solve(A: torch.Tensor, b: torch.Tensor, *, lam: float, eta: int, w: float, K: int,
              index_stream: torch.Tensor, stream_offset: int = 0, x_star: Optional[torch.Tensor] = None,
              warm_start: bool = False, x_ref: Optional[torch.Tensor] = None, check_every: int = 0,
              block_norms: bool = False, grid: int = 0, kernel: int = 0,
              workspace: Optional[torch.Tensor] = None, check: bool = True) -> BskResult:
    """K block sparse Kaczmarz steps, eq. (bsk): x* -= w A_tau^T(A_tau x - b_tau)/||A_tau||_2^2, x = S_lambda(x*).

    ``grid`` and ``kernel`` select the dense kernel of the steps as in ``solve_dense``."""
    m, n = A.shape
    dt = A.dtype
    _dev(b, "b", dt, m)
    if x_star is None:
        if warm_start:
            raise ValueError("warm_start needs x_star")
        x_star = torch.empty(n, dtype=dt, device=A.device)
    _dev(x_star, "x_star", dt, n)
    x = torch.empty(n, dtype=dt, device=A.device)
    status_dev = torch.empty(2, dtype=torch.int32, device=A.device)
    nh = (K // check_every) if (x_ref is not None and check_every > 0) else 0
    err_hist = torch.full((max(nh, 1),), float("nan"), dtype=torch.float64, device=A.device) if nh else None
    norms = torch.full((max(K, 1),), float("nan"), dtype=torch.float64, device=A.device) if block_norms else None
    if K > 0:
        _dev(index_stream, "index_stream", torch.int32, stream_offset + K * eta)
    p = _abi.RskParams(float(lam), int(eta), float(w), None, int(K),
                       _dev(index_stream, "index_stream") if index_stream is not None else None, int(stream_offset),
                       None, 1 if warm_start else 0, _dev(x_ref, "x_ref", dt, n), int(check_every), 0.0,
                       _dev(err_hist, "err_hist"), None, status_dev.data_ptr(), int(grid), int(kernel))
    d = dense_desc(A)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_bsk_dense(ctypes.byref(d), ctypes.byref(p), ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_bsk_dense")
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = _workspace(nbytes.value, A.device)
    st = _lib().rsk_bsk_solve_dense(ctypes.byref(d), b.data_ptr(), ctypes.byref(p), x_star.data_ptr(), x.data_ptr(),
                                    _dev(norms, "block_norm2"), workspace.data_ptr(), workspace.numel(), _stream())
    if st:
        raise RskError(st, "rsk_bsk_solve_dense")
    status = k_done = None
    if check:
        s_ = status_dev.cpu().tolist()
        status, k_done = int(s_[0]), int(s_[1])
        if status:
            raise RskError(status, "rsk_bsk_solve_dense (device)")
    return BskResult(x_star, x, status, k_done, err_hist, None if norms is None else norms[:K])


# ---------------------------------------------------------------------------
# Batched independent systems
# ---------------------------------------------------------------------------

@dataclass
class BatchSystem:
    """One system of a batch: device tensors plus its own parameters."""
    A: torch.Tensor
    b: torch.Tensor
    index_stream: torch.Tensor
    eta: int
    K: int
    alpha: float
    lam: float
    rownorm2_t: Optional[torch.Tensor] = None
    x_star: Optional[torch.Tensor] = None
    warm_start: bool = False
    x_ref: Optional[torch.Tensor] = None
    check_every: int = 0
    tol: float = 0.0


@dataclass
class BatchResult:
    x_star: list
    x: list
    status: Optional[list]
    k_done: Optional[list]
    err_hist: list
    status_dev: torch.Tensor
    items_dev: torch.Tensor
    keep: list


def _batch_items(systems):
    """Host descriptors of a batch and the tensors they point to (outputs, row norms kept alive)."""
    dev = systems[0].A.device
    dt = systems[0].A.dtype
    nsys = len(systems)
    status_dev = torch.zeros((nsys, 2), dtype=torch.int32, device=dev)
    items = (_abi.RskBatchItem * nsys)()
    xs_out, x_out, hist_out, keep = [], [], [], []
    for i, sy in enumerate(systems):
        A = sy.A
        if A.dtype != dt:
            raise TypeError("every system of a batch has the same dtype")
        d = dense_desc(A)
        m, n = A.shape
        _dev(sy.b, "b", dt, m)
        _dev(sy.index_stream, "index_stream", torch.int32, sy.K * sy.eta)
        r2 = sy.rownorm2_t if sy.rownorm2_t is not None else rownorm2(A)
        keep.append(r2)  # must outlive the launch: the kernel reads it through the descriptor
        xs = sy.x_star if sy.x_star is not None else torch.empty(n, dtype=dt, device=dev)
        x = torch.empty(n, dtype=dt, device=dev)
        nh = (sy.K // sy.check_every) if (sy.x_ref is not None and sy.check_every > 0) else 0
        eh = torch.full((max(nh, 1),), float("nan"), dtype=torch.float64, device=dev) if nh else None
        items[i] = _abi.RskBatchItem(A.data_ptr(), m, n, d.ld, sy.b.data_ptr(), r2.data_ptr(),
                                     sy.index_stream.data_ptr(), sy.K, sy.eta, 1 if sy.warm_start else 0,
                                     float(sy.alpha), float(sy.lam), xs.data_ptr(), x.data_ptr(),
                                     _dev(sy.x_ref, "x_ref", dt, n), int(sy.check_every), float(sy.tol),
                                     None if eh is None else eh.data_ptr(), status_dev[i].data_ptr())
        xs_out.append(xs)
        x_out.append(x)
        hist_out.append(eh)
    return items, status_dev, xs_out, x_out, hist_out, keep


def plan_batched(systems, *, wg_bytes: int = 0, kernel: int = 0) -> dict:
    """The launch rsk_avg_solve_batched would make (nothing is queued): the kernel (1 general,
    2 register tile) and each system's workgroups."""
    if not systems:
        raise ValueError("empty batch")
    items, _, _, _, _, _ = _batch_items(systems)
    kout = ctypes.c_int32(0)
    groups = (ctypes.c_int32 * len(systems))()
    st = _lib().rsk_plan_batched(len(systems), _dtype_code(systems[0].A), ctypes.addressof(items), int(wg_bytes),
                                 int(kernel), ctypes.byref(kout), groups)
    if st:
        raise RskError(st, "rsk_plan_batched")
    return {"kernel": int(kout.value), "groups": [int(g) for g in groups]}


def solve_batched(systems, *, order=None, wg_bytes: int = 0, kernel: int = 0,
                  workspace: Optional[torch.Tensor] = None, check: bool = True) -> BatchResult:
    """All systems in one launch; system i on G_i workgroups (most steps first by default).
    ``kernel``: 0 library's choice, 1 general kernel, 2 float32 register tile."""
    if not systems:
        raise ValueError("empty batch")
    dev = systems[0].A.device
    nsys = len(systems)
    items, status_dev, xs_out, x_out, hist_out, keep = _batch_items(systems)
    items_dev = torch.frombuffer(bytearray(bytes(items)), dtype=torch.uint8).to(dev)
    if order is None:
        # longest first: a system's steps take about the same time whatever its size (each step is
        # bound by the exchange latency), so the systems with the most steps go first, larger work
        # first among equal step counts, and the launch does not end on a long system started late
        work = [sy.K * sy.eta * sy.A.shape[1] for sy in systems]
        order = sorted(range(nsys), key=lambda i: (-systems[i].K, -work[i]))
    order_dev = torch.tensor(list(order), dtype=torch.int32, device=dev)
    code = _dtype_code(systems[0].A)
    nbytes = ctypes.c_size_t(0)
    st = _lib().rsk_workspace_size_batched(nsys, code, ctypes.addressof(items), int(wg_bytes), int(kernel),
                                           ctypes.byref(nbytes))
    if st:
        raise RskError(st, "rsk_workspace_size_batched")
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = _workspace(nbytes.value, dev)
    st = _lib().rsk_avg_solve_batched(nsys, code, ctypes.addressof(items), items_dev.data_ptr(), order_dev.data_ptr(),
                                      int(wg_bytes), int(kernel), workspace.data_ptr(), workspace.numel(), _stream())
    if st:
        raise RskError(st, "rsk_avg_solve_batched")
    status = k_done = None
    if check:
        s = status_dev.cpu().tolist()
        status = [int(v[0]) for v in s]
        k_done = [int(v[1]) for v in s]
        bad = [(i, c) for i, c in enumerate(status) if c]
        if bad:
            raise RskError(bad[0][1], f"rsk_avg_solve_batched (device, system {bad[0][0]})")
    return BatchResult(xs_out, x_out, status, k_done, hist_out, status_dev, items_dev, keep + [order_dev, workspace])
