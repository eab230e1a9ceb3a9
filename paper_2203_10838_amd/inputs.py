"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method itself. It draws the data the
paper's experiments use (Sec. 5: i.i.d. N(0,1) matrices, sparse solutions with
N(0,1) nonzeros at random positions, right-hand sides b = A x_hat, optionally
noise of a fixed relative norm in a uniformly random direction) and the row
index stream tau_0, tau_1, ... (eta indices per step, drawn with replacement
with probability proportional to the squared row norm, Sec. 1.1 and variant
v2 of Sec. 5). The stream is the only randomness the iteration consumes; it is
handed to both the HIP library and the oracle as an input array.

Generation is in float64 with numpy's PCG64; a float32 problem is the float64
draw rounded, with b computed in float64 from the rounded A and x_hat, then
rounded. For matrices too large for the host, ``dense_system_device`` draws A
with torch's device generator instead (stated wherever it is used).
"""
from __future__ import annotations

import numpy as np

_DT = {"f32": np.float32, "float32": np.float32, "f64": np.float64, "float64": np.float64}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def sparse_vector(n: int, s: int, rng: np.random.Generator, dtype=np.float64) -> np.ndarray:
    """s distinct uniformly random positions, N(0,1) values, zeros elsewhere (Sec. 5)."""
    x = np.zeros(n, dtype=np.float64)
    if s > 0:
        supp = rng.choice(n, size=min(s, n), replace=False)
        x[supp] = rng.standard_normal(len(supp))
    return x.astype(dtype)


def noise_vector(b: np.ndarray, rel: float, rng: np.random.Generator) -> np.ndarray:
    """rel * ||b|| * g/||g||, g ~ N(0, I): uniform direction on the sphere of that radius (Sec. 5.4)."""
    g = rng.standard_normal(b.shape[0])
    return rel * np.linalg.norm(b) * g / np.linalg.norm(g)


def dense_system(m: int, n: int, s: int, *, dtype="f32", seed: int = 0, noise_rel: float = 0.0):
    """Dense Gaussian system. Returns dict(A, xhat, b, b_clean) with A, b in ``dtype``.

    xhat is rounded to ``dtype`` as well, so that b_clean = A xhat holds for the
    stored numbers up to the final rounding of b.
    """
    dt = _DT[dtype]
    rng = _rng(seed)
    A = rng.standard_normal((m, n)).astype(dt)
    xhat = sparse_vector(n, s, rng, dt)
    b_clean = A.astype(np.float64) @ xhat.astype(np.float64)
    b = b_clean + (noise_vector(b_clean, noise_rel, rng) if noise_rel > 0 else 0.0)
    return {"A": A, "xhat": xhat, "b": b.astype(dt), "b_clean": b_clean.astype(dt)}


def multirhs_system(m: int, n: int, R: int, s: int, *, dtype="f32", seed: int = 0):
    """Shared A, R right-hand sides B = A Xhat with s nonzeros per column."""
    dt = _DT[dtype]
    rng = _rng(seed)
    A = rng.standard_normal((m, n)).astype(dt)
    Xhat = np.stack([sparse_vector(n, s, rng, dt) for _ in range(R)], axis=1)
    B = (A.astype(np.float64) @ Xhat.astype(np.float64)).astype(dt)
    return {"A": A, "Xhat": Xhat, "B": np.ascontiguousarray(B)}


def csr_system(m: int, n: int, nnz_row: int, s: int, *, seed: int = 0, dtype="f32"):
    """Sparse matrix with exactly ``nnz_row`` distinct uniform columns per row (sorted), N(0,1) values.

    Returns dict(row_ptr int64, col int32, val, xhat, b).
    """
    dt = _DT[dtype]
    rng = _rng(seed)
    cols = rng.integers(0, n, size=(m, nnz_row), dtype=np.int64)
    cols.sort(axis=1)
    while True:
        dup = (np.diff(cols, axis=1) == 0).any(axis=1)
        nd = int(dup.sum())
        if nd == 0:
            break
        fresh = rng.integers(0, n, size=(nd, nnz_row), dtype=np.int64)
        fresh.sort(axis=1)
        cols[dup] = fresh
    val = rng.standard_normal((m, nnz_row)).astype(dt)
    xhat = sparse_vector(n, s, rng, dt)
    b = (val.astype(np.float64) * xhat.astype(np.float64)[cols]).sum(axis=1)
    row_ptr = np.arange(m + 1, dtype=np.int64) * nnz_row
    return {"row_ptr": row_ptr, "col": cols.reshape(-1).astype(np.int32), "val": val.reshape(-1),
            "xhat": xhat, "b": b.astype(dt), "m": m, "n": n}


def row_weights(m: int, seed: int, dtype="f32", lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Per-row weights w_i drawn i.i.d. from U[lo, hi] (variants v3/v4 of Sec. 5 use U[0, 1])."""
    return _rng(seed).uniform(lo, hi, size=m).astype(_DT[dtype])


def row_sampling_weights(A) -> np.ndarray:
    """Sampling weights proportional to ||a_i||^2 of the stored rows (float64).

    These define the distribution the stream is drawn from (variant v2 of
    Sec. 5); the solvers never read them.
    """
    A64 = np.asarray(A, dtype=np.float64)
    return np.einsum("ij,ij->i", A64, A64)


def csr_sampling_weights(row_ptr, val) -> np.ndarray:
    v = np.asarray(val, dtype=np.float64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    cs = np.concatenate([[0.0], np.cumsum(v * v)])
    return cs[rp[1:]] - cs[rp[:-1]]


def index_stream(weights: np.ndarray, K: int, eta: int, seed: int) -> np.ndarray:
    """K*eta row indices, i.i.d. with P(i) = w_i / sum(w), step-major (int32).

    u ~ U[0,1) in float64; i = first index whose cumulative weight exceeds u*total.
    """
    w = np.asarray(weights, dtype=np.float64)
    cdf = np.cumsum(w)
    u = _rng(seed).random(int(K) * int(eta))
    idx = np.searchsorted(cdf, u * cdf[-1], side="right")
    return np.minimum(idx, len(w) - 1).astype(np.int32)


def batched_shapes(nsys: int, seed: int, m_lo=500, m_hi=8000, n_lo=200):
    """(m_i, n_i) with m ~ U{m_lo..m_hi}, n ~ U{n_lo..floor(m/2)}."""
    rng = _rng(seed)
    out = []
    for _ in range(nsys):
        m = int(rng.integers(m_lo, m_hi + 1))
        n = int(rng.integers(n_lo, max(n_lo, m // 2) + 1))
        out.append((m, n))
    return out


def dense_system_device(m: int, n: int, s: int, *, seed: int, noise_rel: float = 0.0, device="cuda",
                        chunk_rows: int = 8192):
    """Large float32 Gaussian system drawn on the device with torch's generator.

    A is N(0,1) float32 from ``torch.randn`` on ``device`` (seeded), xhat and
    the noise direction come from numpy PCG64 as above. b is formed in float64
    from the stored A in row chunks, then rounded. Also returns the float64
    sampling weights ||a_i||^2 (computed in row chunks) for ``index_stream``.
    """
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    A = torch.randn((m, n), generator=g, device=device, dtype=torch.float32)
    rng = _rng(seed + 7)
    xhat = sparse_vector(n, s, rng, np.float32)
    xd = torch.from_numpy(xhat.astype(np.float64)).to(device)
    b_clean = torch.empty(m, dtype=torch.float64, device=device)
    w = torch.empty(m, dtype=torch.float64, device=device)
    for r0 in range(0, m, chunk_rows):
        blk = A[r0:r0 + chunk_rows].to(torch.float64)
        b_clean[r0:r0 + chunk_rows] = blk @ xd
        w[r0:r0 + chunk_rows] = (blk * blk).sum(dim=1)
        del blk
    bc = b_clean.cpu().numpy()
    b = bc + (noise_vector(bc, noise_rel, rng) if noise_rel > 0 else 0.0)
    return {"A": A, "xhat": xhat, "b": b.astype(np.float32), "b_clean": bc.astype(np.float32),
            "weights": w.cpu().numpy()}


def csr_system_ragged(m: int, n: int, nnz_lo: int, nnz_hi: int, s: int, *, seed: int = 0, dtype="f32"):
    """Sparse matrix whose rows hold a uniform number of distinct columns in [nnz_lo, nnz_hi] (sorted)."""
    dt = _DT[dtype]
    rng = _rng(seed)
    lens = rng.integers(nnz_lo, nnz_hi + 1, size=m)
    cols = [np.sort(rng.choice(n, size=int(L), replace=False)) for L in lens]
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate(cols).astype(np.int32) if m else np.zeros(0, np.int32)
    val = rng.standard_normal(int(row_ptr[-1])).astype(dt)
    xhat = sparse_vector(n, s, rng, dt)
    b = np.add.reduceat(val.astype(np.float64) * xhat.astype(np.float64)[col], row_ptr[:-1]) if m else np.zeros(0)
    b[lens == 0] = 0.0
    return {"row_ptr": row_ptr, "col": col, "val": val, "xhat": xhat, "b": b.astype(dt), "m": m, "n": n}


def index_stream_device(weights, K: int, eta: int, seed: int, device="cuda"):
    """``index_stream`` drawn on the device: u ~ U[0,1) float64 from torch's generator, same CDF rule."""
    import torch

    w = torch.as_tensor(np.asarray(weights, dtype=np.float64), device=device)
    cdf = torch.cumsum(w, 0)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    u = torch.rand(int(K) * int(eta), generator=g, device=device, dtype=torch.float64)
    idx = torch.searchsorted(cdf, u * cdf[-1], right=True)
    return torch.clamp_(idx, max=w.shape[0] - 1).to(torch.int32)


def batched_workload(nsys: int, seed: int, device="cuda", m_lo=500, m_hi=8000, n_lo=200, frac_nnz=0.05):
    """Batch of independent Gaussian float32 systems on the device, shapes from ``batched_shapes``.

    System i uses seed ``seed + 1000*(i+1)`` for its data and ``+1`` for its row stream
    (drawn by the caller). x_hat_i has round(frac_nnz * n_i) nonzeros; b_i = A_i x_hat_i.
    """
    out = []
    for i, (m, n) in enumerate(batched_shapes(nsys, seed, m_lo, m_hi, n_lo)):
        si = seed + 1000 * (i + 1)
        d = dense_system_device(m, n, int(round(frac_nnz * n)), seed=si, device=device)
        d["seed"] = si
        out.append(d)
    return out
