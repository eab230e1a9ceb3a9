"""rsk_avg_solve_dense_noalloc (the entry point for callers that cannot allocate) against
rsk_avg_solve_dense, both called through the C ABI with caller-owned outputs: the same plan and
kernels, so the results must be the same bits. Two calls in a row on one stream (the second
smaller, so a stale scratch from the first would show), float32 and FP64, and the refusal of a
plan whose exchange exceeds the static scratch."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import alpha_star, check_iterate

pytestmark = pytest.mark.gpu


def _call(A, b, idx, *, lam, eta, alpha, K, noalloc, grid=0, kernel=0):
    """One solve through the C ABI; returns (status code, x*, x, device status)."""
    import torch
    from paper_2203_10838_amd import _abi, rsk
    lib = _abi.load()
    m, n = A.shape
    r2 = rsk.rownorm2(A)
    xs = torch.full((n,), float("nan"), dtype=A.dtype, device=A.device)
    x = torch.full((n,), float("nan"), dtype=A.dtype, device=A.device)
    st_dev = torch.full((2,), -1, dtype=torch.int32, device=A.device)
    p = rsk.make_params(lam=lam, eta=eta, alpha=alpha, K=K, index_stream=idx, rownorm2_t=r2, status_dev=st_dev,
                        grid=grid, kernel=kernel, dtype=A.dtype)
    d = rsk.dense_desc(A)
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        code = lib.rsk_avg_solve_dense_noalloc(ctypes.byref(d), b.data_ptr(), ctypes.byref(p), xs.data_ptr(),
                                               x.data_ptr(), stream)
    else:
        nbytes = ctypes.c_size_t(0)
        assert lib.rsk_workspace_size_dense(ctypes.byref(d), ctypes.byref(p), ctypes.byref(nbytes)) == 0
        ws = torch.empty(max(256, nbytes.value), dtype=torch.uint8, device=A.device)
        code = lib.rsk_avg_solve_dense(ctypes.byref(d), b.data_ptr(), ctypes.byref(p), xs.data_ptr(), x.data_ptr(),
                                       ws.data_ptr(), ws.numel(), stream)
    torch.cuda.synchronize()
    return code, xs, x, st_dev.cpu().tolist()


def _system(m, n, dtype, eta, K, seed):
    sysd = inputs.dense_system(m, n, max(1, n // 25), dtype=dtype, seed=seed)
    idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, seed + 1)
    return sysd, idx


@pytest.mark.parametrize("dtype,tol,shapes", [
    ("f32", 1e-4, [(4000, 2560, 1000, 30, 32, 0), (1500, 640, 96, 40, 0, 0)]),   # register tile; the second smaller
    ("f64", 1e-10, [(1000, 500, 10, 300, 0, 0), (300, 97, 7, 100, 5, 1)]),       # general kernel; the second smaller
])
def test_noalloc_equals_workspace_entry_point(cuda, rsk_lib, dtype, tol, shapes):
    import torch
    for m, n, eta, K, grid, kernel in shapes:
        sysd, idx = _system(m, n, dtype, eta, K, 900 + m)
        A = torch.from_numpy(sysd["A"]).to(cuda)
        b = torch.from_numpy(sysd["b"]).to(cuda)
        ix = torch.from_numpy(idx).to(cuda)
        alpha = alpha_star(sysd["A"], eta)
        kw = dict(lam=0.5, eta=eta, alpha=alpha, K=K, grid=grid, kernel=kernel)
        c0, xs0, x0, s0 = _call(A, b, ix, noalloc=False, **kw)
        c1, xs1, x1, s1 = _call(A, b, ix, noalloc=True, **kw)
        assert c0 == 0 and c1 == 0 and s0 == [0, K] and s1 == [0, K], (c0, c1, s0, s1)
        assert torch.equal(xs1, xs0) and torch.equal(x1, x0), (m, n, eta)
        ref = oracle.rska_dense(sysd["A"], sysd["b"], 0.5, eta, alpha, K, idx)
        check_iterate(xs1, x1, ref, 0.5, tol, min_support=1, what=f"noalloc {m}x{n} eta={eta}")


def test_noalloc_refuses_a_plan_beyond_its_scratch(cuda, rsk_lib):
    """The general float32 kernel at eta = 4096 on 256 workgroups exchanges 2 x 256 x 4096 words a
    step (16.8 MB of workspace): more than the 8 MiB static array, so the call is refused before
    anything is queued (the workspace entry point takes the same plan)."""
    import torch
    from paper_2203_10838_amd import _abi, rsk
    sysd, idx = _system(600, 2048, "f32", 4096, 1, 31)
    A = torch.from_numpy(sysd["A"]).to(cuda)
    b = torch.from_numpy(sysd["b"]).to(cuda)
    ix = torch.from_numpy(idx).to(cuda)
    st_dev = torch.zeros(2, dtype=torch.int32, device=cuda)
    p = rsk.make_params(lam=0.5, eta=4096, alpha=1.0, K=1, index_stream=ix, rownorm2_t=rsk.rownorm2(A),
                        status_dev=st_dev, grid=256, kernel=1, dtype=A.dtype)
    need = rsk.workspace_size_dense(A, p)
    assert need > _abi.NOALLOC_SCRATCH_BYTES
    code, xs, x, st = _call(A, b, ix, lam=0.5, eta=4096, alpha=1.0, K=1, noalloc=True, grid=256, kernel=1)
    assert _abi.STATUS_NAMES[code] == "RSK_ERR_WORKSPACE"
    assert st == [-1, -1] and torch.isnan(xs).all()
    # the workspace entry point runs the same plan
    c0, xs0, x0, s0 = _call(A, b, ix, lam=0.5, eta=4096, alpha=1.0, K=1, noalloc=False, grid=256, kernel=1)
    assert c0 == 0 and s0 == [0, 1]
