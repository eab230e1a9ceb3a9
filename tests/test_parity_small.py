"""GPU parity of the one-workgroup dense kernel (kernel 4: the step in registers, no exchange between
workgroups) against the FP64 oracle on the same index stream, element by element (tests/parity.py):
every column count it takes (1, 2, 4 or 8 columns a thread, ragged n), the largest eta of each,
per-row weights and per-step alpha, the dual y with rows repeated within a step, the monitor and
its early stop, resume, determinism and the device errors."""
import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import alpha_star, check_iterate, check_vec, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def _case(m, n, s, dtype, seed, eta, K):
    sysd = inputs.dense_system(m, n, s, dtype=dtype, seed=seed)
    idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, seed + 1)
    return sysd, idx


def _solve(sysd, idx, dev, **kw):
    from paper_2203_10838_amd import rsk
    return rsk.solve_dense(to_dev(sysd["A"], dev), to_dev(sysd["b"], dev), index_stream=to_dev(idx, dev), **kw)


@pytest.mark.parametrize("dtype,m,n,eta,K,lam,cpt", [
    ("f64", 1000, 500, 10, 3000, 1.0, 2),   # the plain FP64 workload at full size
    ("f64", 300, 97, 7, 400, 0.5, 1),       # odd n: most threads own no column
    ("f32", 700, 256, 32, 300, 1.0, 1),     # one column a thread, the largest eta (32)
    ("f32", 500, 257, 16, 400, 0.5, 2),     # one column past a thread each: two a thread, eta 16
    ("f32", 900, 1000, 8, 300, 0.3, 4),     # four a thread, eta 8
    ("f64", 3000, 2048, 4, 400, 1.0, 8),    # eight a thread (n = 2048, the widest), eta 4
    ("f64", 50, 20, 3, 1000, 0.1, 1),       # tiny
])
def test_small_kernel_matches_oracle(cuda, rsk_lib, dtype, m, n, eta, K, lam, cpt):
    from paper_2203_10838_amd import rsk
    sysd, idx = _case(m, n, max(1, n // 20), dtype, 4100 + m, eta, K)
    A = to_dev(sysd["A"], cuda)
    plan = rsk.plan_dense(A, eta=eta, kernel=4)
    assert plan["kernel"] == 4 and plan["G"] == 1 and plan["chunks_per_lane"] == cpt, plan
    alpha = alpha_star(sysd["A"], eta)
    res = _solve(sysd, idx, cuda, lam=lam, eta=eta, alpha=alpha, K=K, kernel=4)
    assert res.status == 0 and res.k_done == K
    ref = oracle.rska_dense(sysd["A"], sysd["b"], lam, eta, alpha, K, idx)
    check_iterate(res.x_star, res.x, ref, lam, TOL[dtype])


def test_small_kernel_is_the_float64_default_for_small_steps(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    A = torch.zeros((1000, 500), dtype=torch.float64, device=cuda)
    assert rsk.plan_dense(A, eta=10)["kernel"] == 4          # 40 KB a step
    assert rsk.plan_dense(A, eta=16)["kernel"] == 4          # two columns a thread: up to 16 rows
    assert rsk.plan_dense(A, eta=17)["kernel"] == 1          # beyond its eta
    assert rsk.plan_dense(A, eta=10, grid=16)["kernel"] == 1
    wide = torch.zeros((100, 3000), dtype=torch.float64, device=cuda)
    assert rsk.plan_dense(wide, eta=2)["kernel"] == 1        # n > 2048: the multi-workgroup kernels
    assert rsk.plan_dense(A.float(), eta=10)["kernel"] != 4  # float32 keeps the register tile
    with pytest.raises(rsk.RskError) as e:
        rsk.plan_dense(torch.zeros((10, 2052), dtype=torch.float64, device=cuda), eta=2, kernel=4)
    assert e.value.name == "RSK_ERR_UNSUPPORTED"
    with pytest.raises(rsk.RskError) as e:
        rsk.plan_dense(A, eta=17, kernel=4)
    assert e.value.name == "RSK_ERR_UNSUPPORTED"


def test_small_kernel_weights_alpha_k_resume_determinism(cuda, rsk_lib):
    import torch
    sysd, idx = _case(800, 300, 15, "f64", 4200, 12, 600)
    w = inputs.row_weights(800, 4201, dtype="f64", lo=0.2, hi=1.0)
    ak = np.linspace(2.0, 9.0, 600)
    kw = dict(lam=0.6, eta=12, alpha=1.0, kernel=4)
    W, AK = to_dev(w, cuda), to_dev(ak, cuda)
    r1 = _solve(sysd, idx, cuda, K=600, row_w=W, alpha_k=AK, **kw)
    r2 = _solve(sysd, idx, cuda, K=600, row_w=W, alpha_k=AK, **kw)
    assert torch.equal(r1.x_star, r2.x_star) and torch.equal(r1.x, r2.x)
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 0.6, 12, 1.0, 600, idx, alpha_k=ak, row_w=w)
    check_iterate(r1.x_star, r1.x, ref, 0.6, 1e-10)
    # 250 + 350 steps from the first half's x*: the same bits
    h = _solve(sysd, idx, cuda, K=250, row_w=W, alpha_k=AK, **kw)
    r3 = _solve(sysd, idx, cuda, K=350, row_w=W, alpha_k=AK[250:].contiguous(), x_star=h.x_star.clone(),
                warm_start=True, stream_offset=250 * 12, **kw)
    assert torch.equal(r3.x_star, r1.x_star) and torch.equal(r3.x, r1.x)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_small_kernel_dual_with_repeated_rows(cuda, rsk_lib, dtype):
    """y_i -= c_t for every slot t of row i: a stream of 30 rows sampled 10 a step repeats rows within
    most steps; y against the oracle's from y_0 != 0, and the same bits on a second run."""
    import torch
    sysd, _ = _case(30, 40, 3, dtype, 4300, 10, 1)
    rng = np.random.default_rng(4301)
    K, eta = 400, 10
    idx = rng.integers(0, 30, size=K * eta).astype(np.int32)
    alpha = alpha_star(sysd["A"], eta)
    y0 = rng.standard_normal(30).astype(sysd["A"].dtype)
    y = to_dev(y0, cuda)
    res = _solve(sysd, idx, cuda, lam=0.2, eta=eta, alpha=alpha, K=K, kernel=4, y_out=y)
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 0.2, eta, alpha, K, idx, want_y=True, y0=y0.astype(np.float64))
    check_vec(y, ref["y"], TOL[dtype], what="y")
    check_iterate(res.x_star, res.x, ref, 0.2, TOL[dtype], min_support=0)
    y2 = to_dev(y0, cuda)
    _solve(sysd, idx, cuda, lam=0.2, eta=eta, alpha=alpha, K=K, kernel=4, y_out=y2)
    assert torch.equal(y, y2)


def test_small_kernel_monitor_and_early_stop(cuda, rsk_lib):
    K = 5000
    sysd, idx = _case(1000, 500, 25, "f64", 20310838, 10, K)
    alpha = alpha_star(sysd["A"], 10)
    xr = to_dev(sysd["xhat"], cuda)
    res = _solve(sysd, idx, cuda, lam=1.0, eta=10, alpha=alpha, K=K, x_ref=xr, check_every=50, kernel=4)
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 1.0, 10, alpha, K, idx, check_every=50, xref=sysd["xhat"])
    assert np.allclose(res.err_hist.cpu().numpy(), ref["hist"], rtol=1e-6, atol=1e-13)
    assert ref["hist"].min() <= 1e-5
    kstar = (int(np.argmax(ref["hist"] <= 1e-5)) + 1) * 50
    res2 = _solve(sysd, idx, cuda, lam=1.0, eta=10, alpha=alpha, K=K, x_ref=xr, check_every=50, tol=1e-5, kernel=4)
    assert res2.k_done == kstar


def test_small_kernel_device_errors(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    sysd, idx = _case(200, 64, 4, "f32", 11, 4, 30)
    kw = dict(lam=0.5, eta=4, alpha=1.0, K=30, kernel=4)
    # index out of range at step 7: steps 0..6 complete, then the solve stops with the status
    bad = idx.copy()
    bad[7 * 4 + 2] = 200
    with pytest.raises(rsk.RskError) as e:
        _solve(sysd, bad, cuda, **kw)
    assert e.value.name == "RSK_ERR_INDEX_RANGE"
    r = _solve(sysd, bad, cuda, check=False, **kw)
    torch.cuda.synchronize()
    assert r.status_dev.cpu().tolist() == [6, 7]
    r7 = _solve(sysd, idx, cuda, **dict(kw, K=7))
    assert torch.equal(r.x_star, r7.x_star)
    # a bad index in the first step: nothing runs
    bad0 = idx.copy()
    bad0[1] = -3
    r = _solve(sysd, bad0, cuda, check=False, **kw)
    torch.cuda.synchronize()
    assert r.status_dev.cpu().tolist() == [6, 0] and torch.count_nonzero(r.x_star) == 0
    # a referenced zero row: the first step that samples it does not complete
    z = dict(sysd)
    z["A"] = sysd["A"].copy()
    row = int(idx[5 * 4 + 1])
    z["A"][row] = 0.0
    first = int(np.argmax(idx[:30 * 4] == row)) // 4
    r = _solve(z, idx, cuda, check=False, **kw)
    torch.cuda.synchronize()
    assert r.status_dev.cpu().tolist() == [5, first]
    # relaxation far beyond the stability bound: the iterate blows up
    with pytest.raises(rsk.RskError) as e:
        _solve(sysd, inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), 3000, 4, 5), cuda,
               **dict(kw, alpha=1e6, K=3000))
    assert e.value.name == "RSK_ERR_NONFINITE"
    # K = 0 from a warm start returns it unchanged (x = S_lambda(x*))
    xs = to_dev(np.linspace(-1, 1, 64).astype(np.float32), cuda)
    r0 = _solve(sysd, idx, cuda, x_star=xs.clone(), warm_start=True, **dict(kw, K=0))
    assert r0.k_done == 0 and torch.equal(r0.x_star, xs)
