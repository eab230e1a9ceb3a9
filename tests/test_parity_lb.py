"""GPU parity of the linearized Bregman comparator and the power iteration against the FP64 oracle
(element-wise checks of tests/parity.py)."""
import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs
from parity import check_iterate, check_vec

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _step(A):
    return 1.0 / float(np.linalg.norm(np.asarray(A, dtype=np.float64), 2) ** 2)


# shapes: one chunk a thread, a ragged tail (n not a multiple of the 16-byte chunk: the
# one-element path), several chunks a thread, and the largest n the pass takes per dtype
@pytest.mark.parametrize("dtype,tol", [("f32", 2e-5), ("f64", 1e-11)])
@pytest.mark.parametrize("m,n,K,lam", [(700, 1000, 60, 0.5), (1500, 5003, 40, 1.0), (900, 6144, 30, 0.2),
                                       (300, 0, 20, 0.04), (3000, 300, 80, 0.1)])
def test_lb_matches_oracle(cuda, rsk_lib, dtype, tol, m, n, K, lam):
    from paper_2203_10838_amd import rsk
    if n == 0:
        n = 6144 * (4 if dtype == "f32" else 2)  # the largest n: 12 16-byte chunks a thread
    c = inputs.dense_system(m, n, max(1, n // 50), dtype=dtype, seed=m + n, noise_rel=0.01)
    s = _step(c["A"])
    res = rsk.lb_solve(_t(c["A"], cuda), _t(c["b"], cuda), lam=lam, step=s, K=K, residuals=True)
    assert res.status == 0 and res.k_done == K
    ref = oracle.lb_dense(c["A"], c["b"], lam, s, K)
    check_iterate(res.x_star, res.x, ref, lam, tol, min_support=1)
    assert np.allclose(res.res_hist.cpu().numpy(), ref["res"], rtol=max(tol, 1e-12) * 10, atol=0)


def test_lb_unaligned_leading_dimension_and_offset(cuda, rsk_lib):
    """A viewed at an odd column offset with ld = n + 3: the one-element chunk path."""
    import torch
    from paper_2203_10838_amd import rsk
    m, n = 800, 2001
    c = inputs.dense_system(m, n + 4, 30, seed=41)
    full = _t(c["A"], cuda)
    A = full[:, 1:n + 1]
    An = c["A"][:, 1:n + 1]
    b = torch.from_numpy(c["b"]).to(cuda)
    s = _step(An)
    res = rsk.lb_solve(A, b, lam=0.3, step=s, K=40)
    ref = oracle.lb_dense(An, c["b"], 0.3, s, 40)
    check_iterate(res.x_star, res.x, ref, 0.3, 2e-5, min_support=1)


def test_lb_deterministic_resume_and_monitor(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    c = inputs.dense_system(2000, 4000, 40, dtype="f64", seed=43)
    A, b = _t(c["A"], cuda), _t(c["b"], cuda)
    s = _step(c["A"])
    r1 = rsk.lb_solve(A, b, lam=1.0, step=s, K=100, x_ref=_t(c["xhat"], cuda), check_every=10)
    r2 = rsk.lb_solve(A, b, lam=1.0, step=s, K=100)
    assert torch.equal(r1.x_star, r2.x_star) and torch.equal(r1.x, r2.x)
    h = rsk.lb_solve(A, b, lam=1.0, step=s, K=35)
    rest = rsk.lb_solve(A, b, lam=1.0, step=s, K=65, x_star=h.x_star.clone(), warm_start=True)
    assert torch.equal(rest.x_star, r1.x_star) and torch.equal(rest.x, r1.x)
    ref = oracle.lb_dense(c["A"], c["b"], 1.0, s, 100, check_every=10, xref=c["xhat"])
    assert np.allclose(r1.err_hist.cpu().numpy(), ref["hist"], rtol=1e-9, atol=1e-14)


def test_lb_k0_and_nonfinite(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    c = inputs.dense_system(300, 200, 5, seed=44)
    A, b = _t(c["A"], cuda), _t(c["b"], cuda)
    z0 = torch.randn(200, device=cuda)
    r = rsk.lb_solve(A, b, lam=0.5, step=1e-3, K=0, x_star=z0.clone(), warm_start=True)
    assert torch.equal(r.x_star, z0)
    assert torch.equal(r.x, torch.sign(z0) * torch.clamp(z0.abs() - 0.5, min=0))
    r0 = rsk.lb_solve(A, b, lam=0.5, step=1e-3, K=0)
    assert not r0.x_star.any() and not r0.x.any()
    # a step far beyond 2/||A||^2 diverges until x* leaves the finite range
    with pytest.raises(rsk.RskError) as e:
        rsk.lb_solve(A, b, lam=0.0, step=1e3, K=400)
    assert e.value.name == "RSK_ERR_NONFINITE"


def test_lb_host_errors(cuda, rsk_lib):
    import torch
    from paper_2203_10838_amd import rsk
    A = torch.randn(100, 6145 * 4, device=cuda)
    with pytest.raises(rsk.RskError) as e:
        rsk.lb_solve(A, torch.zeros(100, device=cuda), lam=0.1, step=1.0, K=1)
    assert e.value.name == "RSK_ERR_UNSUPPORTED"
    A = torch.randn(100, 50, device=cuda)
    for kw in ({"step": 0.0}, {"step": float("inf")}, {"lam": -1.0}):
        args = {"lam": 0.1, "step": 1.0, "K": 1}
        args.update(kw)
        with pytest.raises(rsk.RskError) as e:
            rsk.lb_solve(A, torch.zeros(100, device=cuda), **args)
        assert e.value.name == "RSK_ERR_INVALID_ARG"


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-12)])
@pytest.mark.parametrize("m,n", [(500, 300), (2000, 5003), (300, 1200)])
def test_spectral_norm2_matches_oracle(cuda, rsk_lib, dtype, tol, m, n):
    import torch
    from paper_2203_10838_amd import rsk
    c = inputs.dense_system(m, n, 5, dtype=dtype, seed=m * 7 + n)
    v = torch.empty(n, dtype=torch.float32 if dtype == "f32" else torch.float64, device=cuda)
    est = rsk.spectral_norm2(_t(c["A"], cuda), 50, v=v)
    ref = oracle.power_ata(c["A"], 50)
    assert abs(est - ref) <= tol * ref
    assert abs(float(torch.linalg.vector_norm(v.double())) - 1.0) <= 10 * tol
    # enough iterations reach sigma_max^2 of the stored matrix
    est2 = rsk.spectral_norm2(_t(c["A"], cuda), 2000)
    sv = float(np.linalg.norm(np.asarray(c["A"], dtype=np.float64), 2) ** 2)
    assert abs(est2 - sv) <= 1e-3 * sv


def test_lb_headline_workload_first_iteration_columns(cuda, rsk_lib):
    """100000 x 20000 float32 Gaussian system (the headline dense workload), one iteration.

    From x*_0 = 0 the first residual is -b whatever A is, so x*_1 restricted to a
    column set J is the oracle's one iteration on A[:, J]; the residual norm of
    step 0 is ||b||.
    """
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.dense_system_device(100000, 20000, 200, seed=20310838 + 300, noise_rel=0.01, device=cuda)
    A = sysd["A"]
    b = torch.from_numpy(sysd["b"]).to(cuda)
    s = 1.0 / 2.1e5  # about 1/sigma_max^2: sigma_max ~ sqrt(m) + sqrt(n) for N(0,1) entries
    r = rsk.lb_solve(A, b, lam=2.0, step=s, K=1, residuals=True)
    r2 = rsk.lb_solve(A, b, lam=2.0, step=s, K=1)
    assert torch.equal(r.x_star, r2.x_star)
    J = np.random.default_rng(5).choice(20000, 96, replace=False)
    J.sort()
    AJ = A[:, torch.from_numpy(J).to(cuda)].cpu().numpy()
    ref = oracle.lb_dense(AJ, sysd["b"], 2.0, s, 1)
    got = r.x_star.cpu().numpy()[J]
    check_vec(got, ref["z"], 1e-5, what="x*_1 on 96 columns")
    assert abs(float(r.res_hist[0]) - float(np.linalg.norm(sysd["b"].astype(np.float64)))) <= 1e-5 * float(
        np.linalg.norm(sysd["b"].astype(np.float64)))
