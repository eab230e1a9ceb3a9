"""GPU parity of the multi-RHS (matrix-core) RSKA path: every column against the single-RHS FP64
oracle on the shared stream, element by element (tests/parity.py)."""
import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs, params
from parity import alpha_star, check_columns

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("kernel", [0, 1, 3])
@pytest.mark.parametrize("m,n,R,eta,K", [(3000, 1000, 64, 100, 40), (2000, 516, 12, 37, 60), (5000, 2048, 128, 300, 15),
                                         (300, 64, 4, 5, 200), (4000, 1288, 200, 150, 12), (3000, 700, 200, 50, 30)])
def test_multirhs_matches_oracle_per_column(cuda, rsk_lib, m, n, R, eta, K, kernel):
    """Kernel 0 is the library's choice (the wide tiles when R > 64 and eta >= 128, else 64 x 64),
    1 the 64 x 64 product tiles, 3 the wide tiles (128 x 128, 128 x 64 for R <= 64 and for the fused
    update): ragged n (516, 700, 1288), R below, at and above
    one wide tile (12, 64, 128, 200), the row-split update (S2 > 1) and the direct one (eta <= 64,
    also at R = 200: four 64-column update tiles, the last one ragged)."""
    from paper_2203_10838_amd import rsk
    sysd = inputs.multirhs_system(m, n, R, max(1, n // 20), seed=m + R)
    A, B = sysd["A"], sysd["B"]
    idx = inputs.index_stream(inputs.row_sampling_weights(A), K, eta, 7 + m)
    A64 = A.astype(np.float64)
    s = np.linalg.svd(A64, compute_uv=False)
    alpha = oracle.optimal_alpha(eta, float((A64 * A64).sum()), float(s[0] ** 2))
    At, Bt = _t(A, cuda), _t(B, cuda)
    plan = rsk.plan_multirhs(At, R, eta=eta, K=K, kernel=kernel)
    if kernel == 3 or (kernel == 0 and R > 64 and eta >= 128):
        assert plan["kernel"] == 3 and plan["eta_pad"] % 128 == 0, plan
    else:
        assert plan["kernel"] == 1, plan
    res = rsk.solve_multirhs(At, Bt, lam=0.5, eta=eta, alpha=alpha, K=K, index_stream=_t(idx, cuda), kernel=kernel)
    assert res.status == 0 and res.k_done == K
    ref = oracle.rska_multirhs(A, B, 0.5, eta, alpha, K, idx)
    check_columns(res.x_star, res.x, ref, 0.5, 1e-4, min_support=R)


@pytest.mark.parametrize("kernel", [1, 3])
def test_multirhs_per_step_alpha_and_errors(cuda, rsk_lib, kernel):
    """Per-step alpha_k against the oracle; an out-of-range index at step 5 stops the solve there
    (status [INDEX_RANGE, 5]) without any kernel reading the bad row, on either tile size."""
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.multirhs_system(1200, 400, 8, 10, seed=5)
    A, B = sysd["A"], sysd["B"]
    K, eta = 30, 16
    idx = inputs.index_stream(inputs.row_sampling_weights(A), K, eta, 6)
    ak = np.linspace(5.0, 12.0, K).astype(np.float32)
    res = rsk.solve_multirhs(_t(A, cuda), _t(B, cuda), lam=0.3, eta=eta, alpha=1.0, K=K, index_stream=_t(idx, cuda),
                             alpha_k=_t(ak, cuda), kernel=kernel)
    ref = oracle.rska_multirhs(A, B, 0.3, eta, 1.0, K, idx, alpha_k=ak.astype(np.float64))
    check_columns(res.x_star, res.x, ref, 0.3, 1e-4, min_support=8)
    bad = idx.copy()
    bad[5 * eta + 3] = 1200
    with pytest.raises(rsk.RskError) as e:
        rsk.solve_multirhs(_t(A, cuda), _t(B, cuda), lam=0.3, eta=eta, alpha=8.0, K=K, index_stream=_t(bad, cuda),
                           kernel=kernel)
    assert e.value.name == "RSK_ERR_INDEX_RANGE"
    r = rsk.solve_multirhs(_t(A, cuda), _t(B, cuda), lam=0.3, eta=eta, alpha=8.0, K=K, index_stream=_t(bad, cuda),
                           check=False, kernel=kernel)
    torch.cuda.synchronize()
    assert r.status_dev.cpu().tolist() == [6, 5]
    # the first five steps ran: x* equals the clean run's after 5 steps
    r5 = rsk.solve_multirhs(_t(A, cuda), _t(B, cuda), lam=0.3, eta=eta, alpha=8.0, K=5, index_stream=_t(idx, cuda),
                            kernel=kernel)
    assert torch.equal(r.x_star, r5.x_star)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("kernel", [1, 3])
def test_multirhs_shared_a_workload_shape_sampled_columns(cuda, rsk_lib, kernel):
    """The shared-A workload at its own shape: A 32768 x 8192 float32 N(0,1) drawn on the device,
    R = 256 right-hand sides B = A X_hat (5% N(0,1) nonzeros a column), eta = 820, alpha = alpha*,
    lambda = 1, 20 steps. Kernel 1: its 512 output tiles of 64 x 64 run the A_tau^T C update
    without a row split over 13 stages of 64 rows. Kernel 3: R_tau on 128 x 128 tiles (eta padded to
    896), the fused update on 128 x 64 tiles (256 of them, no row split) over 26 stages of 32 rows.
    Eight seeded columns against the FP64 oracle on the rows the stream touches."""
    import torch
    from paper_2203_10838_amd import rsk
    m, n, R, eta, K, lam, seed = 32768, 8192, 256, 820, 20, 1.0, 20310838 + 300 + 7
    g = torch.Generator(device=cuda)
    g.manual_seed(seed)
    A = torch.randn((m, n), generator=g, device=cuda, dtype=torch.float32)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    Xh = np.stack([inputs.sparse_vector(n, int(round(0.05 * n)), rng, np.float32) for _ in range(R)], axis=1)
    Xd = torch.from_numpy(Xh.astype(np.float64)).to(cuda)
    B = torch.empty((m, R), dtype=torch.float32, device=cuda)
    w = torch.empty(m, dtype=torch.float64, device=cuda)
    for r0 in range(0, m, 4096):
        blk = A[r0:r0 + 4096].double()
        B[r0:r0 + 4096] = (blk @ Xd).float()
        w[r0:r0 + 4096] = (blk * blk).sum(1)
    del Xd, blk
    wn = w.cpu().numpy()
    v = torch.ones(n, dtype=torch.float32, device=cuda)
    for _ in range(30):  # sigma_max^2 by power iteration (only to set alpha*)
        v = A.t().mv(A.mv(v))
        s2 = float(v.double().norm())
        v = v / v.norm()
    alpha = params.optimal_alpha(eta, float(wn.sum()), s2)
    plan = rsk.plan_multirhs(A, R, eta=eta, K=K, kernel=kernel)
    if kernel == 1:
        assert plan["S2"] == 1 and plan["eta_pad"] == 832, plan
    else:
        # 64 x 4 update tiles of 128 x 64 fill the 256 CUs: no row split
        assert plan["kernel"] == 3 and plan["S2"] == 1 and plan["eta_pad"] == 896, plan
    idx = inputs.index_stream(wn, K, eta, seed + 1)
    res = rsk.solve_multirhs(A, B, lam=lam, eta=eta, alpha=alpha, K=K, index_stream=_t(idx, cuda), kernel=kernel)
    assert res.status == 0 and res.k_done == K
    cols = sorted(np.random.default_rng(seed + 2).choice(R, 8, replace=False).tolist())
    uniq, local = np.unique(idx, return_inverse=True)
    sub = A[torch.from_numpy(uniq.astype(np.int64)).to(cuda)].double().cpu().numpy()
    Bs = B[torch.from_numpy(uniq.astype(np.int64)).to(cuda)][:, cols].double().cpu().numpy()
    refs = [oracle.rska_dense(sub, Bs[:, q], lam, eta, alpha, K, local.astype(np.int32), threads=8)
            for q in range(len(cols))]
    ref = {"z": np.stack([r_["z"] for r_ in refs], 1), "x": np.stack([r_["x"] for r_ in refs], 1)}
    check_columns(res.x_star[:, cols], res.x[:, cols], ref, lam, 1e-4, min_support=40)


@pytest.mark.parametrize("m,n,R,eta,K", [(3000, 1000, 64, 100, 40), (2000, 516, 12, 37, 60), (5000, 2048, 128, 300, 15),
                                         (300, 64, 4, 5, 200), (1500, 704, 8, 1000, 10)])
def test_multirhs_persistent_matches_oracle_and_step_kernels(cuda, rsk_lib, m, n, R, eta, K):
    """One persistent launch for all K steps (kernel 2): every column against the single-RHS oracle,
    and bitwise the step kernels' result wherever both split the n columns alike."""
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.multirhs_system(m, n, R, max(1, n // 20), seed=m + R + 1)
    A, B = _t(sysd["A"], cuda), _t(sysd["B"], cuda)
    idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, 9 + m)
    alpha = alpha_star(sysd["A"], eta)
    p1 = rsk.plan_multirhs(A, R, eta=eta, K=K, kernel=1)
    p2 = rsk.plan_multirhs(A, R, eta=eta, K=K, kernel=2)
    assert p2["kernel"] == 2 and p2["kspan"] % 64 == 0 and p2["S2"] == p1["S2"]
    res2 = rsk.solve_multirhs(A, B, lam=0.5, eta=eta, alpha=alpha, K=K, index_stream=_t(idx, cuda), kernel=2)
    assert res2.status == 0 and res2.k_done == K
    ref = oracle.rska_multirhs(sysd["A"], sysd["B"], 0.5, eta, alpha, K, idx)
    check_columns(res2.x_star, res2.x, ref, 0.5, 1e-4, min_support=R)
    again = rsk.solve_multirhs(A, B, lam=0.5, eta=eta, alpha=alpha, K=K, index_stream=_t(idx, cuda), kernel=2)
    assert torch.equal(again.x_star, res2.x_star)
    if p1["kspan"] == p2["kspan"]:
        res1 = rsk.solve_multirhs(A, B, lam=0.5, eta=eta, alpha=alpha, K=K, index_stream=_t(idx, cuda), kernel=1)
        assert torch.equal(res1.x_star, res2.x_star) and torch.equal(res1.x, res2.x)


def test_multirhs_persistent_checkpoints_resume_and_faults(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.multirhs_system(2400, 768, 16, 30, seed=71)
    A, B = _t(sysd["A"], cuda), _t(sysd["B"], cuda)
    K, eta = 24, 96
    idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, 72)
    ak = np.linspace(20.0, 60.0, K).astype(np.float32)
    kw = dict(lam=0.4, eta=eta, alpha=1.0, index_stream=_t(idx, cuda), alpha_k=_t(ak, cuda))
    ck1 = torch.full((3, 768, 16), float("nan"), device=cuda)
    ck2 = torch.full((3, 768, 16), float("nan"), device=cuda)
    r1 = rsk.solve_multirhs(A, B, K=K, ckpt=ck1, ckpt_every=10, kernel=1, **kw)
    r2 = rsk.solve_multirhs(A, B, K=K, ckpt=ck2, ckpt_every=10, kernel=2, **kw)
    ref = oracle.rska_multirhs(sysd["A"], sysd["B"], 0.4, eta, 1.0, K, idx, alpha_k=ak.astype(np.float64))
    check_columns(r2.x_star, r2.x, ref, 0.4, 1e-4, min_support=16)
    same_split = rsk.plan_multirhs(A, 16, eta=eta, kernel=1)["kspan"] == rsk.plan_multirhs(A, 16, eta=eta,
                                                                                          kernel=2)["kspan"]
    if same_split:
        assert torch.equal(ck1, ck2) and torch.equal(r1.x_star, r2.x_star)
    assert torch.equal(ck2[0], torch.zeros_like(ck2[0]))
    # resume: 10 + 14 steps from the checkpoint-free x* equal 24 steps
    h = rsk.solve_multirhs(A, B, K=10, kernel=2, **kw)
    kw2 = dict(kw, alpha_k=_t(ak[10:], cuda))
    rest = rsk.solve_multirhs(A, B, K=K - 10, kernel=2, X_star=h.x_star.clone(), warm_start=True,
                              stream_offset=10 * eta, **kw2)
    assert torch.equal(rest.x_star, r2.x_star)
    # an index out of range at step 5 stops the launch there; a blow-up is reported
    bad = idx.copy()
    bad[5 * eta + 3] = 2400
    r = rsk.solve_multirhs(A, B, lam=0.4, eta=eta, alpha=8.0, K=K, index_stream=_t(bad, cuda), kernel=2, check=False)
    torch.cuda.synchronize()
    assert r.status_dev.cpu().tolist() == [6, 5]
    with pytest.raises(rsk.RskError) as e:
        rsk.solve_multirhs(A, B, lam=0.4, eta=eta, alpha=1e30, K=K, index_stream=_t(idx, cuda), kernel=2)
    assert e.value.name == "RSK_ERR_NONFINITE"
