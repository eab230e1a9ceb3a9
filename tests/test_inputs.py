"""The seeded input generators: distributions and shapes (no GPU)."""
import numpy as np
from scipy import stats

from paper_2203_10838_amd import inputs


def test_index_stream_follows_squared_row_norms():
    """Rows drawn with replacement, P(i) proportional to ||a_i||^2 (Sec. 1.1, variant v2 of Sec. 5): chi-square."""
    rng = np.random.Generator(np.random.PCG64(0))
    A = rng.normal(size=(12, 6)) * rng.uniform(0.2, 3.0, size=(12, 1))
    w = inputs.row_sampling_weights(A)
    idx = inputs.index_stream(w, 20000, 5, 1)
    assert idx.dtype == np.int32 and idx.shape == (100000,)
    counts = np.bincount(idx, minlength=12)
    expected = w / w.sum() * idx.size
    assert stats.chisquare(counts, expected).pvalue > 1e-4
    # reproducible from the seed
    assert np.array_equal(idx, inputs.index_stream(w, 20000, 5, 1))


def test_dense_system_construction():
    s = inputs.dense_system(50, 30, 7, dtype="f32", seed=3, noise_rel=0.1)
    assert s["A"].dtype == np.float32 and s["b"].dtype == np.float32
    assert np.count_nonzero(s["xhat"]) == 7
    bc = s["A"].astype(np.float64) @ s["xhat"].astype(np.float64)
    noise = s["b"].astype(np.float64) - bc
    assert abs(np.linalg.norm(noise) / np.linalg.norm(bc) - 0.1) < 1e-5


def test_csr_system_rows_have_distinct_sorted_columns():
    c = inputs.csr_system(500, 100, 9, 5, seed=4)
    assert np.all(np.diff(c["row_ptr"]) == 9)
    cols = c["col"].reshape(500, 9)
    assert np.all(np.diff(cols, axis=1) > 0)
    w = inputs.csr_sampling_weights(c["row_ptr"], c["val"])
    assert np.allclose(w, (c["val"].astype(np.float64).reshape(500, 9) ** 2).sum(axis=1))


def test_batched_shapes_ranges():
    sh = inputs.batched_shapes(200, 5)
    assert all(500 <= m <= 8000 and 200 <= n <= max(200, m // 2) for m, n in sh)
