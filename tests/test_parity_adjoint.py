"""GPU parity of the adjoint of K unrolled multi-RHS steps (float32 MFMA) against the FP64 oracle adjoint,
FP64 central differences and FP64 torch autograd. Every gradient is compared element by element
(each entry within the tolerance times the reference's largest entry, tests/parity.py)."""
import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import check_columns, check_vec

pytestmark = pytest.mark.gpu


def _t(a, dev, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t if dtype is None else t.to(dtype)


def _instance(K=24, seed=60, lam=0.05):
    s = inputs.multirhs_system(64, 32, 4, 3, dtype="f32", seed=seed)
    A, B, Xh = s["A"], s["B"], s["Xhat"]
    eta = 4
    A64 = A.astype(np.float64)
    a_star = oracle.optimal_alpha(eta, float((A64 * A64).sum()), float(np.linalg.svd(A64, compute_uv=False)[0] ** 2))
    ak = (a_star * np.linspace(0.8, 1.1, K)).astype(np.float32)
    idx = inputs.index_stream(inputs.row_sampling_weights(A), K, eta, seed + 1)
    return A, B, Xh, eta, K, lam, ak, idx


def _gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, C, xbar_fn, cuda):
    import torch
    from paper_2203_10838_amd import rsk
    At, Bt, It, akt = _t(A, cuda), _t(B, cuda), _t(idx, cuda), _t(ak, cuda)
    n, R = A.shape[1], B.shape[1]
    ckpt = torch.empty((max(1, -(-K // C)), n, R), dtype=torch.float32, device=cuda)
    f = rsk.solve_multirhs(At, Bt, lam=lam, eta=eta, alpha=1.0, K=K, index_stream=It, alpha_k=akt, ckpt=ckpt,
                           ckpt_every=C)
    xbar = _t(xbar_fn(f.x.cpu().numpy()).astype(np.float32), cuda)
    adj = rsk.adjoint_multirhs(At, Bt, lam=lam, eta=eta, alpha_k=akt, K=K, index_stream=It, ckpt=ckpt, ckpt_every=C,
                               X_star_K=f.x_star, Xbar_K=xbar)
    return f, adj


def _oracle_grads(A, B, eta, K, lam, ak, idx, xbar):
    R = B.shape[1]
    bb, lb, ab = [], 0.0, np.zeros(K)
    for r in range(R):
        b_, l_, a_ = oracle.rska_dense_adjoint(A, B[:, r], lam, eta, ak.astype(np.float64), K, idx, xbar[:, r])
        bb.append(b_)
        lb += l_
        ab += a_
    return np.stack(bb, axis=1), lb, ab


def _oracle_loss(A, B, Xh, eta, K, lam, ak, idx):
    L = 0.0
    for r in range(B.shape[1]):
        x = oracle.rska_dense(A, B[:, r], lam, eta, 1.0, K, idx, alpha_k=ak.astype(np.float64))["x"]
        L += float(np.sum((x - Xh[:, r].astype(np.float64)) ** 2))
    return L


@pytest.mark.parametrize("C", [5, 24])
def test_adjoint_matches_oracle_adjoint(cuda, rsk_lib, C):
    A, B, Xh, eta, K, lam, ak, idx = _instance()
    fo = oracle.rska_multirhs(A, B, lam, eta, 1.0, K, idx, alpha_k=ak.astype(np.float64))
    xo = fo["x"]
    xbar = 2 * (xo - Xh.astype(np.float64))
    f, adj = _gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, C, lambda _x: xbar, cuda)
    check_columns(f.x_star, f.x, fo, lam, 1e-4, min_support=4)
    bb, lb, ab = _oracle_grads(A, B, eta, K, lam, ak, idx, xbar)
    check_vec(adj.Bbar, bb, 1e-4, what="dL/dB")
    assert abs(float(adj.lambda_bar.cpu()[0]) - lb) <= 1e-4 * max(1.0, abs(lb))
    check_vec(adj.alpha_bar, ab, 1e-4, what="dL/dalpha_k")


def test_adjoint_wide_tiles_match_oracle_adjoint(cuda, rsk_lib):
    """The adjoint with the wide product tiles (a tuned choice of kernel 3 for the instance's key:
    the forward, the recomputation and the reverse products all take it) against the FP64 oracle."""
    from paper_2203_10838_amd import _abi, autotune
    A, B, Xh, eta, K, lam, ak, idx = _instance()
    m, n, R = A.shape[0], A.shape[1], B.shape[1]
    autotune.set_entry(_abi.RSK_TUNE_MULTIRHS, _abi.RSK_F32, m=m, n=n, eta=eta, R=R, v0=1, v1=1, v2=3)
    try:
        fo = oracle.rska_multirhs(A, B, lam, eta, 1.0, K, idx, alpha_k=ak.astype(np.float64))
        xbar = 2 * (fo["x"] - Xh.astype(np.float64))
        f, adj = _gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, 5, lambda _x: xbar, cuda)
    finally:
        autotune.erase(_abi.RSK_TUNE_MULTIRHS, _abi.RSK_F32, m=m, n=n, eta=eta, R=R)
    check_columns(f.x_star, f.x, fo, lam, 1e-4, min_support=4)
    bb, lb, ab = _oracle_grads(A, B, eta, K, lam, ak, idx, xbar)
    check_vec(adj.Bbar, bb, 1e-4, what="dL/dB")
    assert abs(float(adj.lambda_bar.cpu()[0]) - lb) <= 1e-4 * max(1.0, abs(lb))
    check_vec(adj.alpha_bar, ab, 1e-4, what="dL/dalpha_k")


def test_adjoint_matches_fp64_central_differences(cuda, rsk_lib):
    A, B, Xh, eta, K, lam, ak, idx = _instance()
    f, adj = _gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, 7, lambda x: 2 * (x - Xh), cuda)
    L = lambda **kw: _oracle_loss(kw.get("A", A), kw.get("B", B), Xh, eta, K, kw.get("lam", lam), kw.get("ak", ak), idx)
    h = 1e-6  # FP64 loss; a wider step would cross kinks of S_lambda in the unrolled iteration
    fd_l = (L(lam=lam + h) - L(lam=lam - h)) / (2 * h)
    assert abs(float(adj.lambda_bar.cpu()[0]) - fd_l) <= 1e-3 * max(1.0, abs(fd_l))
    ak64 = ak.astype(np.float64)
    fd_a = np.array([(L(ak=ak64 + h * e) - L(ak=ak64 - h * e)) / (2 * h) for e in np.eye(K)])
    check_vec(adj.alpha_bar, fd_a, 1e-3, what="dL/dalpha_k vs central differences")
    B64 = B.astype(np.float64)
    rng = np.random.default_rng(5)
    picks = [(int(i), int(r)) for i, r in zip(rng.integers(0, 64, 12), rng.integers(0, 4, 12))]
    g = adj.Bbar.cpu().numpy()
    fd_b, gb = [], []
    for i, r in picks:
        E = np.zeros_like(B64)
        E[i, r] = h
        fd_b.append((L(B=B64 + E) - L(B=B64 - E)) / (2 * h))
        gb.append(g[i, r])
    check_vec(gb, fd_b, 1e-3, what="dL/dB vs central differences")


def test_adjoint_checkpoint_spacing_is_exact(cuda, rsk_lib):
    """Recomputed segments reproduce the forward bitwise: every spacing gives identical gradients."""
    A, B, Xh, eta, K, lam, ak, idx = _instance(K=23)
    outs = [_gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, C, lambda x: 2 * (x - Xh), cuda)[1] for C in (1, 4, 23, 50)]
    for o in outs[1:]:
        assert np.array_equal(o.Bbar.cpu().numpy(), outs[0].Bbar.cpu().numpy())
        assert np.array_equal(o.alpha_bar.cpu().numpy(), outs[0].alpha_bar.cpu().numpy())
        assert float(o.lambda_bar.cpu()[0]) == float(outs[0].lambda_bar.cpu()[0])


def test_adjoint_repeated_rows_and_k0(cuda, rsk_lib):
    A, B, Xh, eta, K, lam, ak, idx = _instance(K=6)
    idx = idx.copy()
    idx[0:4] = [5, 5, 9, 5]           # a row three times in one step
    idx[8:12] = [17, 3, 17, 40]
    xo = np.stack([oracle.rska_dense(A, B[:, r], lam, eta, 1.0, K, idx, alpha_k=ak.astype(np.float64))["x"]
                   for r in range(B.shape[1])], axis=1)
    xbar = 2 * (xo - Xh.astype(np.float64))
    f, adj = _gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, 4, lambda _x: xbar, cuda)
    bb, lb, ab = _oracle_grads(A, B, eta, K, lam, ak, idx, xbar)
    check_vec(adj.Bbar, bb, 1e-4, what="dL/dB")
    check_vec(adj.alpha_bar, ab, 1e-4, what="dL/dalpha_k")
    # K = 0: only the seed (x_K = S_lambda(0) = 0 has an empty mask)
    f0, adj0 = _gpu_forward_adjoint(A, B, eta, 0, lam, ak[:0], idx, 4, lambda x: 2 * (x - Xh), cuda)
    assert np.all(adj0.Bbar.cpu().numpy() == 0) and float(adj0.lambda_bar.cpu()[0]) == 0.0


def test_autograd_function_matches_fp64_torch_unroll(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd.autograd import rska_unrolled
    A, B, Xh, eta, K, lam, ak, idx = _instance()
    Bt = _t(B, cuda).requires_grad_(True)
    lt = torch.tensor(lam, dtype=torch.float32, device=cuda, requires_grad=True)
    at = _t(ak, cuda).requires_grad_(True)
    X = rska_unrolled(Bt, lt, at, _t(A, cuda), _t(idx, cuda), eta, ckpt_every=5)
    loss = ((X - _t(Xh, cuda)) ** 2).sum()
    loss.backward()
    # FP64 reference: the same unrolled iteration differentiated by torch on the CPU
    A64 = torch.tensor(A, dtype=torch.float64)
    B64 = torch.tensor(B, dtype=torch.float64, requires_grad=True)
    l64 = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    a64 = torch.tensor(ak, dtype=torch.float64, requires_grad=True)
    r2 = (A64 * A64).sum(1)
    Z = torch.zeros((A.shape[1], B.shape[1]), dtype=torch.float64)
    it = torch.tensor(idx.astype(np.int64))
    for k in range(K):
        Xk = torch.sign(Z) * torch.relu(Z.abs() - l64)
        tk = it[k * eta:(k + 1) * eta]
        Rk = A64[tk] @ Xk - B64[tk]
        Ck = (a64[k] / eta) * Rk / r2[tk, None]
        Z = Z - A64[tk].T.contiguous() @ Ck
    XK = torch.sign(Z) * torch.relu(Z.abs() - l64)
    ((XK - torch.tensor(Xh, dtype=torch.float64)) ** 2).sum().backward()
    check_vec(Bt.grad, B64.grad.numpy(), 1e-3, what="dL/dB vs torch autograd")
    assert abs(float(lt.grad) - float(l64.grad)) <= 1e-3 * max(1.0, abs(float(l64.grad)))
    check_vec(at.grad, a64.grad.numpy(), 1e-3, what="dL/dalpha_k vs torch autograd")


def test_adjoint_full_size_sampled_columns(cuda, rsk_lib):
    """8192 x 4096, R = 64, eta = 410, K = 200, checkpoints every 20: gradients of a loss on two
    columns only (the adjoint is linear in dL/dx_K) against the FP64 oracle adjoint of those columns."""
    import torch
    from paper_2203_10838_amd import params, rsk
    m, n, R, eta, K, C, lam = 8192, 4096, 64, 410, 200, 20, 1.0
    s = inputs.multirhs_system(m, n, R, 40, dtype="f32", seed=20310838 + 400)
    A, B, Xh = s["A"], s["B"], s["Xhat"]
    w = inputs.row_sampling_weights(A)
    At = _t(A, cuda)
    v = torch.ones(n, dtype=torch.float64, device=cuda)
    A64 = At.double()
    for _ in range(60):  # sigma_max^2 by power iteration on A^T A
        v = A64.t() @ (A64 @ v)
        g = float(v.norm())
        v = v / g
    ak = np.full(K, params.optimal_alpha(eta, float(w.sum()), g), dtype=np.float32)
    idx = inputs.index_stream(w, K, eta, 20310838 + 401)
    cols = [3, 40]
    xbar_fn = lambda x: np.where(np.isin(np.arange(R), cols)[None, :], 2 * (x - Xh), 0.0)
    f, adj = _gpu_forward_adjoint(A, B, eta, K, lam, ak, idx, C, xbar_fn, cuda)
    xbar = xbar_fn(f.x.cpu().numpy())
    bb, lb, ab = np.zeros((m, R)), 0.0, np.zeros(K)
    for r in cols:
        b_, l_, a_ = oracle.rska_dense_adjoint(A, B[:, r], lam, eta, ak.astype(np.float64), K, idx, xbar[:, r])
        bb[:, r] = b_
        lb += l_
        ab += a_
    check_vec(adj.Bbar, bb, 1e-3, what="dL/dB")
    assert abs(float(adj.lambda_bar.cpu()[0]) - lb) <= 1e-3 * max(1.0, abs(lb))
    check_vec(adj.alpha_bar, ab, 1e-3, what="dL/dalpha_k")
