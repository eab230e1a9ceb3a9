"""The gather-rate measurement (rsk_gather_rate_dense) reads exactly the solve's row pieces: over
all workgroups, every sampled row of every step is read once, whole, so the sum of the sink is the
sum of those rows' entries."""
import numpy as np
import pytest

from paper_2203_10838_amd import inputs

pytestmark = pytest.mark.gpu


_SHAPES = [(512, 1024, 40, 3, 16, 1), (700, 2000, 129, 4, 64, 2), (300, 160, 7, 5, 8, 8), (2000, 20000, 1024, 2, 256, 1)]
# layout 1 (the register tile's own lanes) takes one row group and slices of at most 80 floats
_CASES = [(*sh, layout) for sh in _SHAPES for layout in (0, 1)
          if layout == 0 or (sh[5] == 1 and -(-(sh[1] // 4) // 4) <= 5 * sh[4])]


@pytest.mark.parametrize("m,n,eta,K,grid,rg,layout", _CASES)
def test_gather_reads_every_sampled_row_once(cuda, rsk_lib, m, n, eta, K, grid, rg, layout):
    import torch
    from paper_2203_10838_amd import rsk
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    idx = inputs.index_stream(np.ones(m), K, eta, m + 1)
    sink = rsk.gather_rate(torch.from_numpy(A).to(cuda), torch.from_numpy(idx).to(cuda), eta=eta, K=K, grid=grid,
                           row_groups=rg, layout=layout)
    got = float(sink.double().sum())
    rows = idx.reshape(K, eta)
    want = float(A.astype(np.float64)[rows.ravel()].sum())
    scale = float(np.abs(A.astype(np.float64)[rows.ravel()]).sum())
    assert abs(got - want) <= 1e-5 * scale, (got, want)
