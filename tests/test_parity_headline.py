"""GPU parity at the full size the benchmark times: the 100000 x 20000 float32 system
(N(0,1) entries drawn on the device, x_hat with 200 N(0,1) nonzeros, b = A x_hat + 1% noise).

* The library's choice at eta = 1024 is the launch the benchmark times: the register-tile kernel
  with one row group of 256 workgroups, 512 threads, 8 row passes of 128 rows and 5 float4 chunks
  a lane, two exchange hops. 60 steps of it (lambda = 2, so that x has support within K) against
  the FP64 oracle on the rows the stream touches (a step reads no other rows), element by element.
* A drift curve of the same launch with the benchmark's own parameters (lambda = 5, alpha*) over
  2000 steps, run as 8 resumed segments of 250 steps (a resume is bitwise the uninterrupted run):
  at every segment end x*_k and x_k against the oracle's, element by element within 1e-4 of
  ||x*_k||_inf. The oracle spreads a step's independent rows and column blocks over host threads
  (the same bits as one thread). With RSK_PARITY_CURVE_DIR set, the curve is written there as JSON.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs, params
from parity import check_iterate

pytestmark = pytest.mark.gpu

M, N, S, NOISE = 100_000, 20_000, 200, 0.01
DATA_SEED = 20310838 + 100          # the benchmark's matrix
TOL = 1e-4
BENCH_PLAN = {"kernel": 2, "G": 256, "threads": 512, "row_passes": 8, "chunks_per_lane": 5, "row_groups": 1,
              "hops": 2, "vec": 4, "row_tile": 0}


def _threads():
    return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)))


def _smax2(A, iters=40):
    """sigma_max(A)^2 by power iteration with torch (only to set alpha*; not part of the checks)."""
    import torch
    g = torch.Generator(device=A.device)
    g.manual_seed(1)
    v = torch.randn(A.shape[1], generator=g, device=A.device, dtype=torch.float32)
    v /= v.norm()
    est = 0.0
    for _ in range(iters):
        w = A.t().mv(A.mv(v))
        est = float(w.double().norm())
        v = w / w.norm()
    return est


@pytest.fixture(scope="module")
def headline(cuda):
    import torch
    d = inputs.dense_system_device(M, N, S, seed=DATA_SEED, noise_rel=NOISE, device=cuda)
    d["b_dev"] = torch.from_numpy(d["b"]).to(cuda)
    d["fro2"] = float(d["weights"].sum())
    d["smax2"] = _smax2(d["A"])
    yield d
    del d["A"], d["b_dev"]
    torch.cuda.empty_cache()


def _rows(A, dev):
    import torch
    return lambda rows: A[torch.from_numpy(np.asarray(rows, dtype=np.int64)).to(dev)].cpu().numpy()


def test_headline_plan_is_the_benchmarked_instantiation(cuda, rsk_lib, headline):
    from paper_2203_10838_amd import rsk
    plan = rsk.plan_dense(headline["A"], eta=1024)
    assert plan == BENCH_PLAN, plan


@pytest.mark.timeout(300)
def test_headline_library_choice_matches_oracle(cuda, rsk_lib, headline):
    import torch
    from paper_2203_10838_amd import rsk
    eta, K, lam = 1024, 60, 2.0
    A = headline["A"]
    alpha = params.optimal_alpha(eta, headline["fro2"], headline["smax2"])
    idx = inputs.index_stream(headline["weights"], K, eta, DATA_SEED + 61)
    res = rsk.solve_dense(A, headline["b_dev"], lam=lam, eta=eta, alpha=alpha, K=K,
                          index_stream=torch.from_numpy(idx).to(cuda))
    assert res.status == 0 and res.k_done == K
    ref = oracle.rska_dense_rows(_rows(A, cuda), headline["b"], M, N, lam, eta, alpha, K, idx, threads=_threads())
    check_iterate(res.x_star, res.x, ref, lam, TOL, min_support=10, what="100000x20000 eta=1024")


@pytest.mark.timeout(900)
def test_headline_drift_curve_2000_steps(cuda, rsk_lib, headline):
    import torch
    from paper_2203_10838_amd import rsk
    eta, seg, nseg, lam = 1024, 250, 8, 5.0
    A = headline["A"]
    alpha = params.optimal_alpha(eta, headline["fro2"], headline["smax2"])
    idx = inputs.index_stream(headline["weights"], seg * nseg, eta, DATA_SEED + 62)
    ix = torch.from_numpy(idx).to(cuda)
    t0 = time.time()
    A64 = A.cpu().numpy().astype(np.float64)
    b64 = headline["b"].astype(np.float64)
    xs = torch.zeros(N, dtype=torch.float32, device=cuda)
    z = np.zeros(N)
    curve = []
    for q in range(nseg):
        res = rsk.solve_dense(A, headline["b_dev"], lam=lam, eta=eta, alpha=alpha, K=seg, index_stream=ix,
                              stream_offset=q * seg * eta, x_star=xs, warm_start=q > 0)
        assert res.status == 0 and res.k_done == seg
        ref = oracle.rska_dense(A64, b64, lam, eta, alpha, seg, idx, off=q * seg * eta, z0=z, threads=_threads())
        z = ref["z"]
        k = (q + 1) * seg
        zg = res.x_star.double().cpu().numpy()
        xg = res.x.double().cpu().numpy()
        curve.append({"k": k,
                      "max_abs_err_x_star_over_inf_norm": float(np.abs(zg - z).max() / np.abs(z).max()),
                      "rel_2norm_err_x_star": float(np.linalg.norm(zg - z) / np.linalg.norm(z)),
                      "rel_2norm_err_x": float(np.linalg.norm(xg - ref["x"]) / max(np.linalg.norm(ref["x"]), 1e-300)),
                      "oracle_support": int(np.count_nonzero(ref["x"])),
                      "oracle_rel_err_to_xhat": float(np.linalg.norm(ref["x"] - headline["xhat"])
                                                      / np.linalg.norm(headline["xhat"]))})
        check_iterate(res.x_star, res.x, ref, lam, TOL, min_support=0 if k < 200 else 50, what=f"k={k}")
    out = os.environ.get("RSK_PARITY_CURVE_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "dense_rt_eta1024_100000x20000_drift.json"), "w") as f:
            json.dump({"workload": "dense 100000x20000 float32, noisy 1%, lambda=5, eta=1024, alpha*",
                       "alpha": alpha, "plan": rsk.plan_dense(A, eta=eta), "tolerance_elementwise": TOL,
                       "oracle_threads": _threads(), "seconds": round(time.time() - t0, 1), "curve": curve},
                      f, indent=1)
