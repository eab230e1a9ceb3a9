"""GPU parity of the device row sampler (Philox4x32-10 + inverse CDF) and of the device CDF."""
import numpy as np
import pytest

import oracle
from paper_2203_10838_amd import inputs

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("m,K,eta,seed,k0", [(37, 50, 9, (1 << 40) + 7, 0), (1000, 30, 128, 20310838, 1 << 33),
                                             (1, 5, 3, 1, 0), (513, 7, 1000, 0, 123456789)])
def test_device_stream_equals_oracle(cuda, rsk_lib, m, K, eta, seed, k0):
    from paper_2203_10838_amd import rsk
    w = np.random.default_rng(m).random(m) + 0.01
    if m > 10:
        w[::7] = 0.0  # rows that must never be drawn
    cdf = oracle.sampling_cdf(w)
    ref = oracle.sample_stream(cdf, seed, K, eta, k0=k0)
    got = rsk.sample_stream(_t(cdf, cuda), seed=seed, K=K, eta=eta, k0=k0).cpu().numpy()
    assert np.array_equal(got, ref)
    if m > 10:
        assert not np.isin(got, np.arange(0, m, 7)).any()


@pytest.mark.parametrize("dtype,m,n", [("f32", 5000, 300), ("f64", 2049, 64), ("f32", 1, 8), ("f32", 70001, 33)])
def test_device_cdf_matches_running_sum(cuda, rsk_lib, dtype, m, n):
    from paper_2203_10838_amd import rsk
    A = inputs.dense_system(m, n, 1, dtype=dtype, seed=m)["A"]
    ref = oracle.sampling_cdf(inputs.row_sampling_weights(A))
    got = rsk.sampling_cdf(_t(A, cuda)).cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-13 * ref)
    got2 = rsk.sampling_cdf(_t(A, cuda)).cpu().numpy()
    assert np.array_equal(got, got2)


def test_device_sampler_distribution(cuda, rsk_lib):
    from scipy.stats import chisquare
    from paper_2203_10838_amd import rsk
    w = np.array([3.0, 0.2, 1.0, 5.0, 0.7, 2.0, 0.05, 1.5])
    idx = rsk.sample_stream(_t(oracle.sampling_cdf(w), cuda), seed=99, K=10000, eta=64).cpu().numpy()
    counts = np.bincount(idx, minlength=len(w))
    assert chisquare(counts, w / w.sum() * len(idx)).pvalue > 1e-3


def test_device_sampler_full_size(cuda, rsk_lib):
    """The 100000 x 20000 float32 matrix of the large dense workload; a stream of 8000 steps of 1024
    rows; whole steps spot-checked against the oracle given the device cdf."""
    import torch
    from paper_2203_10838_amd import rsk
    sysd = inputs.dense_system_device(100000, 20000, 200, seed=20310838 + 100, noise_rel=0.01, device=cuda)
    cdf = rsk.sampling_cdf(sysd["A"])
    ref_cdf = np.cumsum(sysd["weights"])  # FP64 row norms summed in another order: equal to rounding
    got_cdf = cdf.cpu().numpy()
    assert np.all(np.abs(got_cdf - ref_cdf) <= 1e-12 * ref_cdf)
    K, eta, seed = 8000, 1024, 20310838 + 101
    idx = rsk.sample_stream(cdf, seed=seed, K=K, eta=eta)
    torch.cuda.synchronize()
    got = idx.cpu().numpy().reshape(K, eta)
    for k in (0, 1, 4095, 7999):
        assert np.array_equal(got[k], oracle.sample_stream(got_cdf, seed, 1, eta, k0=k))
    counts = np.bincount(got.ravel(), minlength=100000)
    p = sysd["weights"] / sysd["weights"].sum()
    # expected count ~82 per row: the heaviest and lightest rows stay within a wide band
    z = (counts - p * K * eta) / np.sqrt(p * K * eta)
    assert np.abs(z).max() < 6.5
