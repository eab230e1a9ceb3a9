"""Element-wise parity checks of a GPU result against the FP64 oracle (shared by the GPU tests).

Every check is element by element, never through a 2-norm alone:

* a vector v (x*_K, the dual y, a gradient, one column of X*_K):
      |v_gpu[j] - v_ref[j]| <= tol * max(||v_ref||_inf, floor)   for every j;
* x_K = S_lambda(x*_K): S_lambda is 1-Lipschitz (Sec. 1.1), so every element of x obeys the
  same bound with the scale of x*; on top of that the supports of x agree wherever x*_ref[j]
  is decided, i.e. | |x*_ref[j]| - lambda | exceeds the band tol * ||x*_ref||_inf within which
  an admissible perturbation could move it across lambda; and x_gpu = S_lambda(x*_gpu) exactly
  in the kernel's own precision.

`min_support` makes a check fail when the oracle's x has fewer nonzeros than that: a
comparison of x = 0 with x = 0 proves nothing about the shrinkage or the update.
"""
from __future__ import annotations

import numpy as np


def _f64(a):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def check_vec(got, ref, tol, *, floor=0.0, what="v"):
    """Every element within tol * max(||ref||_inf, floor); returns the largest error / scale."""
    g = _f64(got).ravel()
    r = _f64(ref).ravel()
    assert g.shape == r.shape, f"{what}: shape {g.shape} vs {r.shape}"
    assert np.all(np.isfinite(g)), f"{what}: non-finite values"
    scale = max(float(np.abs(r).max()) if r.size else 0.0, float(floor))
    err = np.abs(g - r)
    bad = np.nonzero(err > tol * scale)[0]
    if bad.size:
        j = int(bad[np.argmax(err[bad])])
        raise AssertionError(f"{what}: {bad.size} of {r.size} elements beyond {tol:g} * {scale:.4e}; "
                             f"worst j={j}: gpu {g[j]:.10e} oracle {r[j]:.10e}")
    return float(err.max() / scale) if (err.size and scale > 0) else 0.0


def shrink_exact(z, lam):
    """S_lambda(z) = max(|z| - lambda, 0) sign(z) in z's own precision (|z| == lambda gives 0)."""
    z = np.asarray(z)
    lam_t = np.asarray(lam, dtype=z.dtype)
    return np.where(np.abs(z) - lam_t > 0, np.sign(z) * (np.abs(z) - lam_t), 0).astype(z.dtype)


def check_iterate(z_gpu, x_gpu, ref, lam, tol, *, min_support=1, what="", exact_shrink=True):
    """x*_K and x_K of one run (or one right-hand side) against the oracle's dict (z, x).

    Returns (relative error of x*, number of oracle nonzeros in x)."""
    zg = z_gpu.detach().cpu().numpy() if hasattr(z_gpu, "detach") else np.asarray(z_gpu)
    xg = x_gpu.detach().cpu().numpy() if hasattr(x_gpu, "detach") else np.asarray(x_gpu)
    zr = _f64(ref["z"]).ravel()
    xr = _f64(ref["x"]).ravel()
    zg, xg = zg.ravel(), xg.ravel()
    scale = float(np.abs(zr).max()) if zr.size else 0.0
    ez = check_vec(zg, zr, tol, what=f"{what} x*")
    check_vec(xg, xr, tol, floor=scale, what=f"{what} x")
    band = tol * scale
    decided = np.abs(np.abs(zr) - lam) > band
    sg, sr = xg != 0, xr != 0
    flips = np.nonzero(decided & (sg != sr))[0]
    assert flips.size == 0, f"{what}: support differs at {flips.size} decided elements (first j={int(flips[0])})"
    if exact_shrink:
        assert np.array_equal(xg, shrink_exact(zg, lam)), f"{what}: x != S_lambda(x*) in the kernel's precision"
    nnz = int(np.count_nonzero(xr))
    assert nnz >= min_support, f"{what}: vacuous comparison, the oracle's x has {nnz} nonzeros (< {min_support})"
    return ez, nnz


def check_columns(Zg, Xg, ref, lam, tol, *, min_support=1, what=""):
    """Per right-hand side: column r of (X*, X) against column r of the oracle's (z, x)."""
    Zg = Zg.detach().cpu().numpy() if hasattr(Zg, "detach") else np.asarray(Zg)
    Xg = Xg.detach().cpu().numpy() if hasattr(Xg, "detach") else np.asarray(Xg)
    zr, xr = _f64(ref["z"]), _f64(ref["x"])
    total = 0
    for r in range(zr.shape[1]):
        _, nnz = check_iterate(Zg[:, r], Xg[:, r], {"z": zr[:, r], "x": xr[:, r]}, lam, tol, min_support=0,
                               what=f"{what} column {r}")
        total += nnz
    assert total >= min_support, f"{what}: vacuous comparison, the oracle's X has {total} nonzeros"
    return total


def alpha_star(A, eta):
    """alpha* of the Corollary (uniform weights) from the exact FP64 SVD of a small A."""
    import oracle
    A64 = np.asarray(A, dtype=np.float64)
    s = np.linalg.svd(A64, compute_uv=False)
    return oracle.optimal_alpha(eta, float((A64 * A64).sum()), float(s[0] ** 2))


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)
