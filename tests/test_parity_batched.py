"""GPU parity of the batched path: every system against its own single-system FP64 oracle run,
element by element (tests/parity.py)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import check_iterate, check_vec

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _alpha(A, eta):
    A64 = A.astype(np.float64)
    s = np.linalg.svd(A64, compute_uv=False)
    return oracle.optimal_alpha(eta, float((A64 * A64).sum()), float(s[0] ** 2))


def _batch(nsys, seed, dtype, mult4, K, m_hi=700):
    """mult4: True (n % 4 == 0), False (any n) or "pad" (any n; the device rows are padded to a
    multiple of 4 floats, so the register tile takes them)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nsys):
        m = int(rng.integers(60, m_hi))
        n = int(rng.integers(20, max(21, m // 2)))
        if mult4 is True:
            n = max(4, n - n % 4)
        sysd = inputs.dense_system(m, n, max(1, n // 20), dtype=dtype, seed=seed * 1000 + i)
        eta = 1 + n // 10
        idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, seed * 1000 + i + 500)
        out.append((sysd, eta, idx, _alpha(sysd["A"], eta), 0.2 + 0.1 * (i % 5)))
    return out


def _padded(A, cuda, fill=float("nan")):
    """A on the device in rows padded to a multiple of 4 floats; the padding holds `fill` (NaN by
    default: a kernel that read it into a dot or an update would show it)."""
    import torch
    m, n = A.shape
    ld = n + (-n) % 4
    buf = torch.full((m, ld), fill, dtype=torch.float32, device=cuda)
    buf[:, :n] = _t(A, cuda)
    return buf[:, :n]


def _systems(batch, K, cuda, pad=False, **kw):
    from paper_2203_10838_amd import rsk
    return [rsk.BatchSystem(A=_padded(s["A"], cuda) if pad else _t(s["A"], cuda), b=_t(s["b"], cuda),
                            index_stream=_t(idx, cuda), eta=eta, K=K, alpha=al, lam=lam, **kw)
            for s, eta, idx, al, lam in batch]


@pytest.mark.parametrize("dtype,mult4,wg_bytes,tol,kernel,expect", [
    # library's choice: the register tile where every float32 system takes it, else the general kernel
    ("f32", True, 0, 1e-4, 0, 2), ("f32", False, 0, 1e-4, 0, 1), ("f64", False, 0, 1e-10, 0, 1),
    ("f32", "pad", 0, 1e-4, 0, 2),
    # small targets split every system over several workgroups (one-hop and two-hop exchange)
    ("f32", True, 2048, 1e-4, 1, 1), ("f64", False, 1024, 1e-10, 0, 1), ("f32", False, 256, 1e-4, 0, 1),
    ("f32", True, 2048, 1e-4, 2, 2), ("f32", "pad", 1024, 1e-4, 2, 2), ("f32", "pad", 256, 1e-4, 2, 2)])
def test_batched_matches_single_system_oracle(cuda, rsk_lib, dtype, mult4, wg_bytes, tol, kernel, expect):
    from paper_2203_10838_amd import rsk
    K = 150
    batch = _batch(37, 3 if mult4 else 4, dtype, mult4, K, m_hi=700 if wg_bytes != 256 else 2400)
    systems = _systems(batch, K, cuda, pad=mult4 == "pad")
    plan = rsk.plan_batched(systems, wg_bytes=wg_bytes, kernel=kernel)
    assert plan["kernel"] == expect
    if wg_bytes and wg_bytes <= 2048:
        assert sum(g > 1 for g in plan["groups"]) >= len(batch) // 2, plan
    res = rsk.solve_batched(systems, wg_bytes=wg_bytes, kernel=kernel)
    assert all(k == K for k in res.k_done)
    support = 0
    for i, (s, eta, idx, al, lam) in enumerate(batch):
        ref = oracle.rska_dense(s["A"], s["b"], lam, eta, al, K, idx)
        support += check_iterate(res.x_star[i], res.x[i], ref, lam, tol, min_support=0, what=f"system {i}")[1]
    assert support >= 5 * len(batch)


def test_batched_group_equals_single_system_kernel(cuda, rsk_lib):
    """A system alone in a batch runs the single-system kernel's code on the same G: bitwise equal."""
    from paper_2203_10838_amd import rsk
    K = 60
    (s, eta, idx, al, lam), = _batch(1, 11, "f32", True, K, m_hi=2000)
    n = s["A"].shape[1]
    for wg_bytes in (0, 4096):
        res = rsk.solve_batched(_systems([(s, eta, idx, al, lam)], K, cuda), wg_bytes=wg_bytes, kernel=1)
        G = max(1, min(256, -(-eta * n * 4 // (wg_bytes or 48 * 1024)), -(-n // 4)))
        single = rsk.solve_dense(_t(s["A"], cuda), _t(s["b"], cuda), lam=lam, eta=eta, alpha=al, K=K,
                                 index_stream=_t(idx, cuda), grid=G, kernel=1)
        a, b = res.x_star[0].cpu().numpy(), single.x_star.cpu().numpy()
        if G % 8:
            assert np.array_equal(a, b), (wg_bytes, G)
        else:  # the single-system kernel permutes slices over XCDs: another partial-sum order
            check_vec(a, b, 1e-5, what=f"wg_bytes={wg_bytes} G={G}")


@pytest.mark.parametrize("dtype,kernel,tol", [("f64", 1, 1e-6), ("f32", 2, 1e-4)])
def test_batched_early_stop_and_errors(cuda, rsk_lib, dtype, kernel, tol):
    """The monitor stops each system at the oracle's first check within tol (the float32 register
    tile against a tolerance well above its rounding drift), and a bad index stops its system only."""
    import torch
    from paper_2203_10838_amd import rsk
    K = 6000
    batch = _batch(6, 9, dtype, "pad" if dtype == "f32" else False, K)
    pad = dtype == "f32"
    for wg_bytes in (0, 1024):
        systems = [rsk.BatchSystem(A=_padded(s["A"], cuda) if pad else _t(s["A"], cuda), b=_t(s["b"], cuda),
                                   index_stream=_t(idx, cuda), eta=eta, K=K, alpha=al, lam=lam,
                                   x_ref=_t(s["xhat"], cuda), check_every=25, tol=tol)
                   for s, eta, idx, al, lam in batch]
        assert rsk.plan_batched(systems, wg_bytes=wg_bytes, kernel=kernel)["kernel"] == kernel
        res = rsk.solve_batched(systems, wg_bytes=wg_bytes, kernel=kernel)
        for i, (s, eta, idx, al, lam) in enumerate(batch):
            ref = oracle.rska_dense(s["A"], s["b"], lam, eta, al, K, idx, check_every=25, xref=s["xhat"])
            h = ref["hist"]
            expect = (int(np.argmax(h <= tol)) + 1) * 25 if (h <= tol).any() else K
            if dtype == "f64":
                assert res.k_done[i] == expect, (wg_bytes, i, res.k_done[i], expect)
            else:
                # float32 rounding may move a crossing of tol by one check
                assert abs(res.k_done[i] - expect) <= 25, (wg_bytes, i, res.k_done[i], expect)
                e = float((res.x[i].double().cpu() - torch.from_numpy(s["xhat"]).double()).norm()
                          / np.linalg.norm(s["xhat"]))
                assert e <= tol * 1.5 or res.k_done[i] == K, (i, e)
        # a bad index in one system stops that system only
        s, eta, idx, al, lam = batch[2]
        bad = idx.copy()
        bad[3 * eta] = s["A"].shape[0]
        systems[2] = rsk.BatchSystem(A=_padded(s["A"], cuda) if pad else _t(s["A"], cuda), b=_t(s["b"], cuda),
                                     index_stream=_t(bad, cuda), eta=eta, K=100, alpha=al, lam=lam)
        r = rsk.solve_batched(systems, check=False, wg_bytes=wg_bytes, kernel=kernel)
        torch.cuda.synchronize()
        st = r.status_dev.cpu().numpy()
        assert st[2, 0] == 6 and st[2, 1] == 3
        assert all(st[i, 0] == 0 for i in range(6) if i != 2)


@pytest.mark.parametrize("kernel", [1, 2])
def test_batched_device_descriptor_outside_plan(cuda, rsk_lib, kernel):
    """A device descriptor whose plan exceeds the launch (the general kernel's LDS, the register
    tile's eta) is skipped with RSK_ERR_INVALID_ARG."""
    import torch
    from paper_2203_10838_amd import _abi, rsk
    K = 20
    batch = _batch(3, 21, "f32", True, K)
    systems = _systems(batch, K, cuda)
    res = rsk.solve_batched(systems, kernel=kernel)  # builds descriptors and checks the good path
    items = (_abi.RskBatchItem * 3).from_buffer_copy(res.items_dev.cpu().numpy().tobytes())
    dev_items = (_abi.RskBatchItem * 3).from_buffer_copy(bytes(items))
    dev_items[1].eta = 20000  # needs far more LDS than planned; never read further
    items_dev = torch.frombuffer(bytearray(bytes(dev_items)), dtype=torch.uint8).to(cuda)
    nbytes = ctypes.c_size_t(0)
    lib = rsk._lib()
    assert lib.rsk_workspace_size_batched(3, 0, ctypes.addressof(items), 0, kernel, ctypes.byref(nbytes)) == 0
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=cuda)
    assert lib.rsk_avg_solve_batched(3, 0, ctypes.addressof(items), items_dev.data_ptr(), None, 0, kernel,
                                     ws.data_ptr(), ws.numel(), rsk._stream()) == 0
    torch.cuda.synchronize()
    st = res.status_dev.cpu().numpy()
    assert st[1, 0] == 1 and st[1, 1] == 0
    assert st[0, 0] == 0 and st[0, 1] == K and st[2, 0] == 0 and st[2, 1] == K


def test_batched_host_checks(cuda, rsk_lib):
    from paper_2203_10838_amd import rsk
    K = 5
    batch = _batch(2, 5, "f32", True, K)
    systems = _systems(batch, K, cuda)
    systems[1].alpha = -1.0
    with pytest.raises(rsk.RskError, match="INVALID_ARG"):
        rsk.solve_batched(systems)


@pytest.mark.parametrize("dtype,wg_bytes,tol,kernel", [("f32", 0, 1e-4, 1), ("f32", 4096, 1e-4, 1),
                                                       ("f32", 0, 1e-4, 2), ("f32", 4096, 1e-4, 2),
                                                       ("f64", 0, 1e-10, 1), ("f64", 2048, 1e-10, 1)])
def test_batched_pipelined_tiles_with_nan_padding(cuda, rsk_lib, dtype, wg_bytes, tol, kernel):
    """Rows padded past n with NaN to a whole number of 16-byte chunks (the general kernel's
    pipelined tile and the register tile load whole chunks, so the padding reaches LDS or VGPRs and
    must never be used); ragged n. Every system matches its oracle run."""
    import torch
    from paper_2203_10838_amd import rsk
    K = 120
    batch = _batch(24, 31, dtype, False, K, m_hi=600)
    vec = 4 if dtype == "f32" else 2
    tdt = torch.float32 if dtype == "f32" else torch.float64
    systems = []
    for s, eta, idx, al, lam in batch:
        m, n = s["A"].shape
        full = torch.full((m, -(-n // vec) * vec + vec), float("nan"), dtype=tdt, device=cuda)
        full[:, :n] = _t(s["A"], cuda)
        systems.append(rsk.BatchSystem(A=full[:, :n], b=_t(s["b"], cuda), index_stream=_t(idx, cuda), eta=eta,
                                       K=K, alpha=al, lam=lam))
    assert rsk.plan_batched(systems, wg_bytes=wg_bytes, kernel=kernel)["kernel"] == kernel
    res = rsk.solve_batched(systems, wg_bytes=wg_bytes, kernel=kernel)
    assert all(k == K for k in res.k_done)
    support = 0
    for i, (s, eta, idx, al, lam) in enumerate(batch):
        ref = oracle.rska_dense(s["A"], s["b"], lam, eta, al, K, idx)
        support += check_iterate(res.x_star[i], res.x[i], ref, lam, tol, min_support=0, what=f"system {i}")[1]
    assert support >= 3 * len(batch)
