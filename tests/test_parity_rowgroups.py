"""GPU parity of the float32 register-tile kernel over two row groups (kernel = 3) against the
FP64 oracle: each workgroup reads half of a step's rows over a slice twice as wide, and the two
workgroups of a slice add their parts of the update (Algorithm 1's x* step) in a third exchange.

Bars as for the one-group kernel: element-wise 1e-4 of ||x*_K||_inf on x*_K and x_K (tests/parity.py),
bitwise determinism and exact resume; every stop condition ends every workgroup at the same step,
without an expired wait.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import check_iterate, check_vec

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _to(t, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(t)).to(dev)


def _alpha_star(A, eta):
    A64 = np.asarray(A, dtype=np.float64)
    s = np.linalg.svd(A64, compute_uv=False)
    return oracle.optimal_alpha(eta, float((A64 * A64).sum()), float(s[0] ** 2))


def _case(m, n, eta, K, seed):
    sysd = inputs.dense_system(m, n, max(1, n // 25), dtype="f32", seed=seed, noise_rel=0.01)
    idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, seed + 1)
    return sysd, idx


def _solve(sysd, idx, dev, **kw):
    from paper_2203_10838_amd import rsk
    return rsk.solve_dense(_to(sysd["A"], dev), _to(sysd["b"], dev), index_stream=_to(idx, dev), **kw)


@pytest.mark.parametrize("m,n,eta,K,grid", [
    (2000, 1280, 128, 80, 16),    # one-hop reduce: 8 slices x 64 group rows, one pass
    (3000, 1280, 200, 60, 32),    # 1024 threads, one pass of 128 group rows, 3 chunks a lane
    (3000, 1280, 300, 60, 16),    # 1024 threads, 2 passes of 128 group rows, 5 chunks a lane
    (3000, 1280, 700, 30, 32),    # 1024 threads, 3 passes, 3 chunks a lane
    (4000, 2048, 1024, 20, 128),  # 512 threads, 8 passes, 64 slices of 2 units
    (2500, 1000, 901, 25, 64),    # ragged: groups of 451 and 450 rows, 62.5 units over 32 slices
    (3000, 1600, 800, 20, 0),     # the library's grid (one workgroup per CU)
])
def test_two_row_groups_match_oracle(cuda, rsk_lib, m, n, eta, K, grid):
    import torch
    sysd, idx = _case(m, n, eta, K, 7000 + eta)
    alpha = _alpha_star(sysd["A"], eta)
    res = _solve(sysd, idx, cuda, lam=1.0, eta=eta, alpha=alpha, K=K, grid=grid, kernel=3)
    assert res.status == 0 and res.k_done == K
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 1.0, eta, alpha, K, idx)
    check_iterate(res.x_star, res.x, ref, 1.0, TOL, min_support=5)
    again = _solve(sysd, idx, cuda, lam=1.0, eta=eta, alpha=alpha, K=K, grid=grid, kernel=3)
    assert torch.equal(again.x_star, res.x_star) and torch.equal(again.x, res.x)


def test_two_row_groups_resume_dual_and_monitor(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    sysd, idx = _case(3000, 1280, 600, 80, 71)
    alpha = _alpha_star(sysd["A"], 600)
    A, b, ix = _to(sysd["A"], cuda), _to(sysd["b"], cuda), _to(idx, cuda)
    kw = dict(lam=0.5, eta=600, alpha=alpha, grid=32, kernel=3)
    full = rsk.solve_dense(A, b, K=80, index_stream=ix, **kw)
    head = rsk.solve_dense(A, b, K=35, index_stream=ix, **kw)
    rest = rsk.solve_dense(A, b, K=45, index_stream=ix, stream_offset=35 * 600, x_star=head.x_star.clone(),
                           warm_start=True, **kw)
    assert torch.equal(rest.x_star, full.x_star) and torch.equal(rest.x, full.x)
    # the dual: y[tau_t] -= c_t over both groups' rows, x* = A^T y
    y = torch.zeros(3000, dtype=torch.float32, device=cuda)
    rd = rsk.solve_dense(A, b, K=80, index_stream=ix, y_out=y, **kw)
    assert torch.equal(rd.x_star, full.x_star)
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 0.5, 600, alpha, 80, idx, want_y=True, check_every=10,
                            xref=sysd["xhat"])
    check_vec(y, ref["y"], TOL, what="y")
    check_iterate(rd.x_star, rd.x, ref, 0.5, TOL, min_support=5)
    # the monitor counts each slice once
    rm = rsk.solve_dense(A, b, K=80, index_stream=ix, x_ref=_to(sysd["xhat"], cuda), check_every=10, **kw)
    assert torch.equal(rm.x_star, full.x_star)
    assert np.allclose(rm.err_hist.cpu().numpy(), ref["hist"], rtol=1e-3, atol=1e-6)


def test_two_row_groups_tolerance_stop(cuda, rsk_lib):
    """The monitor's early stop ends both groups at the same check: the result is bitwise the run
    of exactly that many steps."""
    import torch
    from paper_2203_10838_amd import rsk
    sysd, idx = _case(3000, 1280, 400, 400, 75)
    alpha = _alpha_star(sysd["A"], 400)
    A, b, ix, xr = _to(sysd["A"], cuda), _to(sysd["b"], cuda), _to(idx, cuda), _to(sysd["xhat"], cuda)
    kw = dict(lam=0.05, eta=400, alpha=alpha, grid=32, kernel=3, index_stream=ix)
    full = rsk.solve_dense(A, b, K=400, x_ref=xr, check_every=10, **kw)
    h = full.err_hist.cpu().numpy()
    tol = float(h[len(h) // 3])
    early = rsk.solve_dense(A, b, K=400, x_ref=xr, check_every=10, tol=tol, **kw)
    assert early.status == 0 and early.k_done < 400 and early.k_done % 10 == 0
    assert h[early.k_done // 10 - 1] <= tol
    same = rsk.solve_dense(A, b, K=early.k_done, **kw)
    assert torch.equal(same.x_star, early.x_star)


@pytest.mark.parametrize("group", [0, 1])
def test_two_row_groups_stop_together(cuda, rsk_lib, group):
    """A bad index, a zero row or a blow-up in either group's rows ends the launch with its code,
    at once (an expired wait would take seconds and end in RSK_ERR_ABORTED)."""
    from paper_2203_10838_amd import rsk
    eta, K = 600, 40
    sysd, idx = _case(3000, 1280, eta, K, 72)
    alpha = _alpha_star(sysd["A"], eta)
    pos = 9 * eta + (10 if group == 0 else eta - 5)
    bad = idx.copy()
    bad[pos] = 3000
    t0 = time.time()
    with pytest.raises(rsk.RskError) as e:
        _solve(sysd, bad, cuda, lam=0.5, eta=eta, alpha=alpha, K=K, grid=32, kernel=3)
    assert e.value.name == "RSK_ERR_INDEX_RANGE"
    Az = sysd["A"].copy()
    Az[idx[pos]] = 0.0
    z = dict(sysd, A=Az)
    with pytest.raises(rsk.RskError) as e:
        _solve(z, idx, cuda, lam=0.5, eta=eta, alpha=alpha, K=K, grid=32, kernel=3)
    assert e.value.name == "RSK_ERR_ZERO_ROW"
    with pytest.raises(rsk.RskError) as e:
        _solve(sysd, idx, cuda, lam=0.5, eta=eta, alpha=1e30, K=K, grid=32, kernel=3)
    assert e.value.name == "RSK_ERR_NONFINITE"
    assert time.time() - t0 < 2.0


def test_two_row_groups_stop_step_matches_one_group(cuda, rsk_lib):
    """A bad index at step 12: both layouts complete the 12 steps before it, with the same x*."""
    import torch
    from paper_2203_10838_amd import rsk
    eta, K = 900, 30
    sysd, idx = _case(2500, 1280, eta, K, 73)
    bad = idx.copy()
    bad[12 * eta + 800] = -4
    A, b = _to(sysd["A"], cuda), _to(sysd["b"], cuda)
    out = {}
    for kern in (2, 3):
        r = rsk.solve_dense(A, b, lam=0.5, eta=eta, alpha=400.0, K=K, index_stream=_to(bad, cuda), grid=64,
                            kernel=kern, check=False)
        out[kern] = (r.status_dev.cpu().tolist(), r.x_star.double().cpu().numpy())
    assert out[2][0] == out[3][0] and out[3][0][1] == 12
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 0.5, eta, 400.0, 12, idx)
    check_vec(out[3][1], ref["z"], TOL, what="x* after the 12 steps before the fault")


def test_two_row_groups_rejects(cuda, rsk_lib):
    from paper_2203_10838_amd import rsk
    sysd, idx = _case(400, 256, 200, 4, 74)
    s64 = dict(sysd, A=sysd["A"].astype(np.float64), b=sysd["b"].astype(np.float64))
    with pytest.raises(rsk.RskError) as e:
        _solve(s64, idx, cuda, lam=0.5, eta=200, alpha=1.0, K=4, kernel=3)
    assert e.value.name == "RSK_ERR_UNSUPPORTED"
    c = inputs.csr_system(400, 256, 10, 5, seed=75)
    with pytest.raises(rsk.RskError) as e:
        rsk.solve_csr(_to(c["row_ptr"], cuda), _to(c["col"], cuda), _to(c["val"], cuda), c["n"], _to(c["b"], cuda),
                      lam=0.5, eta=8, alpha=1.0, K=2, index_stream=_to(idx[:16] % 400, cuda), kernel=3)
    assert e.value.name == "RSK_ERR_INVALID_ARG"


@pytest.mark.timeout(300)
def test_two_row_groups_headline_workload(cuda, rsk_lib):
    """100000 x 20000 float32, eta = 1024 (the headline shape), 40 steps with two row groups; the
    oracle runs on the rows the stream touches (a step reads no others), indices remapped."""
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.dense_system_device(100000, 20000, 200, seed=20310838 + 600, noise_rel=0.01, device=cuda)
    K, eta = 40, 1024
    idx = inputs.index_stream(sysd["weights"], K, eta, 20310838 + 601)
    res = rsk.solve_dense(sysd["A"], torch.from_numpy(sysd["b"]).to(cuda), lam=2.0, eta=eta, alpha=800.0, K=K,
                          index_stream=_to(idx, cuda), kernel=3)
    assert res.status == 0
    rows, local = np.unique(idx, return_inverse=True)
    sub = sysd["A"][torch.from_numpy(rows).to(cuda)].cpu().numpy()
    ref = oracle.rska_dense(sub, sysd["b"][rows], 2.0, eta, 800.0, K, local.astype(np.int32), threads=8)
    check_iterate(res.x_star, res.x, ref, 2.0, TOL, min_support=10)


def test_library_choice_of_row_groups(cuda, rsk_lib):
    """kernel = 0 plans two row groups for 88 <= eta <= 800 unless one group's whole next-step tile
    fits the LDS prefetch (eta <= 256 at 20000 columns: one pass of five slots a thread), and one
    group outside that range, on a 20000-column float32 system (rsk_plan_dense); runs bitwise what the
    explicit kernel runs, and matches the oracle on the rows the stream touches."""
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.dense_system_device(6000, 20000, 100, seed=77, noise_rel=0.01, device=cuda)
    A, b = sysd["A"], torch.from_numpy(sysd["b"]).to(cuda)
    for eta, twin in ((88, 2), (256, 2), (257, 3), (300, 3), (800, 3), (801, 2), (1024, 2), (87, 2), (64, 2)):
        plan = rsk.plan_dense(A, eta=eta)
        assert plan["kernel"] == twin and plan["row_groups"] == (2 if twin == 3 else 1), (eta, plan)
        K = 12
        idx = inputs.index_stream(sysd["weights"], K, eta, 78 + eta)
        auto = rsk.solve_dense(A, b, lam=0.3, eta=eta, alpha=0.8 * eta, K=K, index_stream=_to(idx, cuda), kernel=0)
        same = rsk.solve_dense(A, b, lam=0.3, eta=eta, alpha=0.8 * eta, K=K, index_stream=_to(idx, cuda),
                               kernel=twin)
        assert torch.equal(auto.x_star, same.x_star), eta
        if eta in (300, 1024):
            rows, local = np.unique(idx, return_inverse=True)
            sub = A[torch.from_numpy(rows.astype(np.int64)).to(cuda)].cpu().numpy()
            ref = oracle.rska_dense(sub, sysd["b"][rows], 0.3, eta, 0.8 * eta, K, local.astype(np.int32), threads=8)
            check_iterate(auto.x_star, auto.x, ref, 0.3, TOL, min_support=1, what=f"eta={eta}")


@pytest.mark.parametrize("case", range(10))
def test_register_tiles_random_shapes(cuda, rsk_lib, case):
    """Seeded random shapes (ragged slices, ragged row groups, both thread counts): kernels 2 and 3
    against the oracle; shapes a kernel does not take must be refused with RSK_ERR_UNSUPPORTED."""
    from paper_2203_10838_amd import rsk
    rng = np.random.default_rng(9000 + case)
    n = 4 * int(rng.integers(40, 500))
    m = int(rng.integers(n // 2, 3 * n))
    eta = int(rng.choice([int(rng.integers(130, 768)), int(rng.integers(769, 1025))]))
    K = int(max(4, min(40, 3e7 // (eta * n))))
    grid = int(rng.choice([0, 64, 128, 200, 256]))
    sysd, idx = _case(m, n, eta, K, 9100 + case)
    alpha = _alpha_star(sysd["A"], eta)
    ref = oracle.rska_dense(sysd["A"], sysd["b"], 0.5, eta, alpha, K, idx)
    ran = 0
    for kern in (2, 3):
        try:
            res = _solve(sysd, idx, cuda, lam=0.5, eta=eta, alpha=alpha, K=K, grid=grid, kernel=kern)
        except rsk.RskError as e:
            assert e.name == "RSK_ERR_UNSUPPORTED", (kern, m, n, eta, grid)
            continue
        ran += 1
        assert res.status == 0 and res.k_done == K
        check_iterate(res.x_star, res.x, ref, 0.5, TOL, min_support=0, what=f"kernel {kern} {m}x{n} eta={eta}")
    assert ran >= 1
