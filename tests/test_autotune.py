"""The autotuner on the device: it times candidate launches, installs the fastest in the library's
tuning table, and the choices the caller leaves to the library then run the tuned launch.

For each path the tuned solve must equal the explicit-parameter solve of the same choice bit for
bit, and match the FP64 oracle element by element (tests/parity.py). The table is cleared before
and after, so no other test sees a tuned choice.
"""
import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import alpha_star, check_columns, check_iterate, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def clean_table(rsk_lib):
    from paper_2203_10838_amd import autotune
    autotune.clear()
    yield
    autotune.clear()


def test_tuned_dense_choice_is_the_explicit_launch(cuda):
    import torch
    from paper_2203_10838_amd import _abi, autotune, rsk
    m, n, eta, K, lam = 3000, 2560, 300, 40, 0.5
    sysd = inputs.dense_system(m, n, 100, dtype="f32", seed=4100)
    idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, 4101)
    A, b, ix = to_dev(sysd["A"], cuda), to_dev(sysd["b"], cuda), to_dev(idx, cuda)
    alpha = alpha_star(sysd["A"], eta)
    cands = [(2, 64), (3, 64), (1, 32), (2, 160)]
    out = autotune.tune_dense(A, b, eta=eta, lam=lam, alpha=alpha, index_stream=ix, steps=10, reps=2,
                              candidates=cands)
    kernel, grid = out["choice"]
    assert (kernel, grid) in cands and len(out["table"]) == len(cands)
    e = autotune.get_entry(_abi.RSK_TUNE_DENSE, _abi.RSK_F32, m=m, n=n, eta=eta)
    assert (e["v0"], e["v1"]) == (kernel, grid)
    plan = rsk.plan_dense(A, eta=eta)
    assert plan == rsk.plan_dense(A, eta=eta, grid=grid, kernel=kernel)
    tuned = rsk.solve_dense(A, b, lam=lam, eta=eta, alpha=alpha, K=K, index_stream=ix)
    explicit = rsk.solve_dense(A, b, lam=lam, eta=eta, alpha=alpha, K=K, index_stream=ix, kernel=kernel, grid=grid)
    assert torch.equal(tuned.x_star, explicit.x_star) and torch.equal(tuned.x, explicit.x)
    ref = oracle.rska_dense(sysd["A"], sysd["b"], lam, eta, alpha, K, idx)
    check_iterate(tuned.x_star, tuned.x, ref, lam, 1e-4, min_support=5)
    # another eta has no entry: the built-in choice
    assert rsk.plan_dense(A, eta=eta + 1) == rsk.plan_dense(A, eta=eta + 1, grid=0, kernel=0)
    autotune.clear()
    assert rsk.plan_dense(A, eta=eta)["kernel"] in (1, 2, 3)


def test_tuned_dense_entry_that_does_not_apply_falls_back(cuda):
    """An entry for a kernel the matrix cannot take (the register tile on an odd n) leaves the
    built-in choice in place."""
    import torch
    from paper_2203_10838_amd import _abi, autotune, rsk
    sysd = inputs.dense_system(500, 301, 10, dtype="f32", seed=4200)
    A = to_dev(sysd["A"], cuda)
    before = rsk.plan_dense(A, eta=16)
    autotune.set_entry(_abi.RSK_TUNE_DENSE, _abi.RSK_F32, m=500, n=301, eta=16, v0=2, v1=8)
    assert rsk.plan_dense(A, eta=16) == before
    autotune.set_entry(_abi.RSK_TUNE_DENSE, _abi.RSK_F32, m=500, n=301, eta=16, v0=1, v1=3)
    assert rsk.plan_dense(A, eta=16)["G"] == 3


def test_tuned_multirhs_split_matches_oracle(cuda, tmp_path):
    import torch
    from paper_2203_10838_amd import _abi, autotune, rsk
    m, n, R, eta, K, lam = 3000, 1024, 64, 100, 12, 0.5
    s = inputs.multirhs_system(m, n, R, 40, seed=4300)
    idx = inputs.index_stream(inputs.row_sampling_weights(s["A"]), K, eta, 4301)
    A, B, ix = to_dev(s["A"], cuda), to_dev(s["B"], cuda), to_dev(idx, cuda)
    alpha = alpha_star(s["A"], eta)
    out = autotune.tune_multirhs(A, B, eta=eta, lam=lam, alpha=alpha, index_stream=ix, steps=3, reps=2,
                                 candidates=[(1, 1, 1), (2, 2, 1), (4, 1, 1), (4, 2, 2), (2, 1, 2)])
    S, S2, kernel = out["choice"]
    plan = rsk.plan_multirhs(A, R, eta=eta)
    assert plan["S2"] == S2 and plan["kernel"] == kernel
    tuned = rsk.solve_multirhs(A, B, lam=lam, eta=eta, alpha=alpha, K=K, index_stream=ix)
    # the same split and kernel set by hand: the explicit choice
    autotune.clear()
    autotune.set_entry(_abi.RSK_TUNE_MULTIRHS, _abi.RSK_F32, m=m, n=n, eta=eta, R=R, v0=S, v1=S2)
    explicit = rsk.solve_multirhs(A, B, lam=lam, eta=eta, alpha=alpha, K=K, index_stream=ix, kernel=kernel)
    assert torch.equal(tuned.x_star, explicit.x_star)
    ref = oracle.rska_multirhs(s["A"], s["B"], lam, eta, alpha, K, idx)
    check_columns(tuned.x_star, tuned.x, ref, lam, 1e-4, min_support=R)
    # save, clear, load: the cache file restores the choice
    f = str(tmp_path / "tune.txt")
    autotune.save(f)
    autotune.clear()
    autotune.load(f)
    assert rsk.plan_multirhs(A, R, eta=eta) == plan


def test_tuned_batched_classes_match_oracle(cuda):
    """Per size class of the step bytes a tuned workgroup target; a system's result depends only on
    its own plan, so each equals the system solved alone with its class's target, bit for bit."""
    import torch
    from paper_2203_10838_amd import autotune, rsk
    K = 60
    rng = np.random.default_rng(4400)
    batch = []
    for i in range(12):
        m = int(rng.integers(400, 3000))
        n = int(rng.integers(40, m // 2)) // 4 * 4
        sysd = inputs.dense_system(m, n, max(1, n // 20), seed=4400 + i)
        eta = 1 + n // 10
        idx = inputs.index_stream(inputs.row_sampling_weights(sysd["A"]), K, eta, 4500 + i)
        batch.append((sysd, eta, idx, alpha_star(sysd["A"], eta), 0.3))

    def systems(subset):
        return [rsk.BatchSystem(A=to_dev(s["A"], cuda), b=to_dev(s["b"], cuda), index_stream=to_dev(ix, cuda),
                                eta=eta, K=K, alpha=al, lam=lam) for s, eta, ix, al, lam in subset]
    bounds = (16 << 10, 128 << 10, 1 << 62)
    out = autotune.tune_batched(systems(batch), bounds=bounds, candidates_kib=(4, 16, 64), reps=1)
    assert out["classes"]
    res = rsk.solve_batched(systems(batch))
    assert all(k == K for k in res.k_done)
    wg_of = {c["step_bytes_hi"]: c["wg_kib"] << 10 for c in out["classes"]}
    for i, (s, eta, ix, al, lam) in enumerate(batch):
        step = eta * s["A"].shape[1] * 4
        hi = next(h for h in sorted(wg_of) if step <= h)
        alone = rsk.solve_batched(systems([batch[i]]), wg_bytes=wg_of[hi])
        assert torch.equal(alone.x_star[0], res.x_star[i]), i
        ref = oracle.rska_dense(s["A"], s["b"], lam, eta, al, K, ix)
        check_iterate(res.x_star[i], res.x[i], ref, lam, 1e-4, min_support=0, what=f"system {i}")
