"""FP64 CPU oracle for the averaged randomized sparse Kaczmarz method (RSKA).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product (the
HIP library and its Python binding) never imports it, and the two share no
code: the only thing both sides see is the seeded input generator, which holds
none of the method's arithmetic.

What is here (each function cites the passage it follows):

* ``rska_dense`` / ``rska_csr`` -- the RSKA iteration, eq. (rska) and
  Algorithm 1, in plain double-precision C loops (``rska_oracle.c``), driven by
  an explicit row-index stream.
* ``rska_multirhs`` / ``rska_batched`` -- column by column / system by system
  repetitions of ``rska_dense`` (one shared stream for all right-hand sides;
  one stream per system).
* ``rska_dense_adjoint`` -- reverse mode of K unrolled steps, every iterate
  stored (no checkpointing).
* ``lb_dense`` / ``power_ata`` -- the full-batch linearized Bregman comparator
  (the remark on its rate in Sec. 4) and sigma_max(A)^2 by power iteration;
* ``bsk_dense`` -- the block sparse Kaczmarz iteration, eq. (bsk) of Sec. 1.1,
  on the rows an explicit index stream names, with ||A_tau||_2^2 taken as the
  largest eigenvalue of the block's Gram matrix (numpy);
* ``philox4x32_10``, ``sampling_cdf``, ``sample_stream`` -- the row sampler
  (p_i proportional to ||a_i||^2, Sec. 1.1) driven by the counter-based
  generator Philox4x32-10 of Salmon et al. (SC'11) and an inverse-CDF search;
* numpy helpers for the closed forms of Sec. 2 and Sec. 4: ``soft_threshold``
  (Sec. 1.1), ``f_value`` / ``f_conjugate`` (Example exmp:f),
  ``bregman_distance`` (Example exmp:D), ``optimal_alpha`` and
  ``L_of_alpha`` (Theorem 1 and its Corollary), ``sampling_matrix``
  (Definition 1).

Parity status of every function is recorded in the design notes; every
function here is pinned by a ``-m "not gpu"`` test against something other
than itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rska_oracle.c")
_LIB = os.path.join(_HERE, "librska_oracle.so")
_lock = threading.Lock()
_lib = None

OK, INVALID, ZERO_ROW, INDEX_RANGE, NONFINITE = 0, 1, 5, 6, 7
_NAMES = {OK: "OK", INVALID: "INVALID_ARG", ZERO_ROW: "ZERO_ROW", INDEX_RANGE: "INDEX_RANGE",
          NONFINITE: "NONFINITE"}


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"oracle {where}: {_NAMES.get(code, code)}")
        self.code = code
        self.name = _NAMES.get(code, str(code))


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, no BLAS, no fast-math; OpenMP only spreads independent
    rows and column blocks of a step over threads, never reorders a sum)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
            lib.oracle_rownorm2_dense.argtypes = [i64, i64, i64, vp, vp]
            lib.oracle_rownorm2_csr.argtypes = [i64, vp, vp, vp]
            lib.oracle_rska_dense.argtypes = [i64, i64, i64, vp, vp, dbl, i32, dbl, vp, vp, i64, vp, i64,
                                              vp, vp, vp, i64, vp, vp, vp]
            lib.oracle_rska_dense_threads.argtypes = lib.oracle_rska_dense.argtypes + [i32]
            lib.oracle_rska_csr.argtypes = [i64, i64, vp, vp, vp, vp, dbl, i32, dbl, vp, vp, i64, vp, i64,
                                            vp, vp, vp, i64, vp, vp, vp]
            lib.oracle_rska_dense_adjoint.argtypes = [i64, i64, i64, vp, vp, dbl, i32, vp, i64, vp, i64,
                                                      vp, vp, vp, vp]
            lib.oracle_philox4x32_10.argtypes = [vp, vp, vp]
            lib.oracle_philox4x32_10.restype = None
            lib.oracle_sampling_cdf.argtypes = [i64, vp, vp]
            lib.oracle_sample_stream.argtypes = [i64, vp, ctypes.c_uint64, i64, i64, i32, vp]
            lib.oracle_lb_dense.argtypes = [i64, i64, i64, vp, vp, dbl, dbl, i64, vp, vp, i64, vp, vp, vp]
            lib.oracle_power_ata.argtypes = [i64, i64, i64, vp, i64, vp, vp]
            for f in (lib.oracle_rownorm2_dense, lib.oracle_rownorm2_csr, lib.oracle_rska_dense,
                      lib.oracle_rska_dense_threads,
                      lib.oracle_rska_csr, lib.oracle_rska_dense_adjoint, lib.oracle_sampling_cdf,
                      lib.oracle_sample_stream, lib.oracle_lb_dense, lib.oracle_power_ata):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


# ---------------------------------------------------------------------------
# Closed forms (numpy)
# ---------------------------------------------------------------------------

def soft_threshold(v, lam):
    """S_lambda(v) = max(|v| - lambda, 0) * sign(v), Sec. 1.1 (RSK)."""
    v = np.asarray(v, dtype=np.float64)
    return np.maximum(np.abs(v) - lam, 0.0) * np.sign(v)


def f_value(x, lam):
    """f(x) = lambda ||x||_1 + 1/2 ||x||^2, eq. (spf) in Example exmp:f."""
    x = np.asarray(x, dtype=np.float64)
    return lam * np.abs(x).sum() + 0.5 * (x * x).sum()


def f_conjugate(xs, lam):
    """f*(x*) = 1/2 ||S_lambda(x*)||^2, Example exmp:f."""
    s = soft_threshold(xs, lam)
    return 0.5 * (s * s).sum()


def bregman_distance(x, xs, y, lam):
    """D_f^{x*}(x, y) = f*(x*) - <x*, y> + f(y), the Fenchel form after Def. def:D.

    With x = S_lambda(x*) this equals 1/2||x - y||^2 + lambda (||y||_1 - <s, y>),
    x* = x + lambda s (Example exmp:D).
    """
    return f_conjugate(xs, lam) - float(np.dot(xs, y)) + f_value(y, lam)


def L_of_alpha(alpha, eta, fro2, smax2, smax_W=None):
    """L(alpha) of Theorem 1 (th:RSKA); smax_W defaults to alpha (uniform W = alpha I)."""
    sw = alpha if smax_W is None else smax_W
    return alpha - alpha / (2.0 * eta) * (alpha / fro2 * (eta - 1) * smax2 + sw)


def optimal_alpha(eta, fro2, smax2):
    """alpha* for uniform weights W = alpha I, Corollary cor:linear_convergence (b)."""
    return eta / (1.0 + (eta - 1.0) * smax2 / fro2)


def sampling_matrix(A, tau, weights):
    """M_k = (1/eta) sum_{i in tau} w_i e_i e_i^T / ||a_i||^2 (Definition 1), as a dense m x m matrix."""
    A = _f64(A)
    m = A.shape[0]
    M = np.zeros((m, m))
    eta = len(tau)
    r2 = (A * A).sum(axis=1)
    for i, w in zip(tau, weights):
        M[i, i] += w / (eta * r2[i])
    return M


# ---------------------------------------------------------------------------
# C loops
# ---------------------------------------------------------------------------

def rownorm2_dense(A):
    """||a_i||^2 of every row (j ascending, FP64): the squared diagonal of D in Definition 1."""
    A = _f64(A)
    m, n = A.shape
    r2 = np.empty(m)
    st = _load().oracle_rownorm2_dense(m, n, n, _p(A), _p(r2))
    if st:
        raise OracleError(st, "rownorm2_dense")
    return r2


def rownorm2_csr(row_ptr, val):
    """||a_i||^2 of every CSR row (stored order, FP64)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    val = _f64(val)
    m = len(row_ptr) - 1
    r2 = np.empty(m)
    st = _load().oracle_rownorm2_csr(m, _p(row_ptr), _p(val), _p(r2))
    if st:
        raise OracleError(st, "rownorm2_csr")
    return r2


def _common_out(n, m, z0, want_y, y0, K, check_every):
    z = np.zeros(n) if z0 is None else _f64(z0).copy()
    x = np.empty(n)
    y = None
    if want_y:
        y = np.zeros(m) if y0 is None else _f64(y0).copy()
    nh = (K // check_every) if check_every and check_every > 0 else 0
    hist = np.full(max(nh, 1), np.nan)
    return z, x, y, hist, nh


def rska_dense(A, b, lam, eta, alpha, K, idx, *, off=0, alpha_k=None, row_w=None, z0=None, want_y=False,
               y0=None, check_every=0, xref=None, raise_on_error=True, threads=1):
    """Dense RSKA, eq. (rska) / Algorithm 1, in FP64 (see ``rska_oracle.c``).

    A (m x n) and b are upcast exactly to float64. ``row_w`` (m, optional) are
    per-row weights w_i (the matrix W of Definition 1; variants v3/v4 of Sec. 5):
    row i is relaxed by alpha (or alpha_k[k]) times w_i. Returns a dict with
    z (= x*_K), x (= S_lambda(z)), y (dual, if want_y), hist (relative errors
    every ``check_every`` steps if xref is given), k_done and status.

    ``threads`` > 1 computes a step's eta residuals, and blocks of the columns of delta_k, on
    several threads; every sum keeps its order, so the result is the same bits.
    """
    A = _f64(A)
    b = _f64(b)
    m, n = A.shape
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ak = None if alpha_k is None else _f64(alpha_k)
    rw = None if row_w is None else _f64(row_w)
    z, x, y, hist, nh = _common_out(n, m, z0, want_y, y0, K, check_every)
    xr = None if xref is None else _f64(xref)
    kd = np.zeros(1, dtype=np.int64)
    st = _load().oracle_rska_dense_threads(m, n, n, _p(A), _p(b), float(lam), int(eta), float(alpha), _p(ak),
                                           _p(rw), int(K), _p(idx), int(off), _p(z), _p(x), _p(y),
                                           int(check_every) if xr is not None else 0, _p(xr), _p(hist), _p(kd),
                                           int(threads))
    if st and raise_on_error:
        raise OracleError(st, "rska_dense")
    return {"z": z, "x": x, "y": y, "hist": hist[:nh], "k_done": int(kd[0]), "status": st}


def rska_csr(row_ptr, col, val, n, b, lam, eta, alpha, K, idx, *, off=0, alpha_k=None, row_w=None, z0=None,
             want_y=False, y0=None, check_every=0, xref=None, raise_on_error=True):
    """CSR RSKA: the same iteration with rows stored as (row_ptr, col, val)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = _f64(val)
    b = _f64(b)
    m = len(row_ptr) - 1
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ak = None if alpha_k is None else _f64(alpha_k)
    rw = None if row_w is None else _f64(row_w)
    z, x, y, hist, nh = _common_out(n, m, z0, want_y, y0, K, check_every)
    xr = None if xref is None else _f64(xref)
    kd = np.zeros(1, dtype=np.int64)
    st = _load().oracle_rska_csr(m, n, _p(row_ptr), _p(col), _p(val), _p(b), float(lam), int(eta),
                                 float(alpha), _p(ak), _p(rw), int(K), _p(idx), int(off), _p(z), _p(x), _p(y),
                                 int(check_every) if xr is not None else 0, _p(xr), _p(hist), _p(kd))
    if st and raise_on_error:
        raise OracleError(st, "rska_csr")
    return {"z": z, "x": x, "y": y, "hist": hist[:nh], "k_done": int(kd[0]), "status": st}


def rska_dense_rows(rows_of, b, m, n, lam, eta, alpha, K, idx, *, off=0, alpha_k=None, row_w=None, z0=None,
                    threads=1):
    """Dense RSKA on a matrix too large to hand over whole.

    Only the rows that the stream references enter the iteration, so the
    oracle runs on those rows alone (``rows_of(unique_rows) -> array``), with
    the stream renumbered onto them. This is a selection of inputs, not a
    change of arithmetic: every step touches exactly the same numbers.
    """
    idx = np.asarray(idx, dtype=np.int64)
    used = idx[off: off + K * eta]
    if used.size and (used.min() < 0 or used.max() >= m):
        raise OracleError(INDEX_RANGE, "rska_dense_rows")
    uniq, inv = np.unique(used, return_inverse=True)
    Asub = _f64(rows_of(uniq))
    bsub = _f64(np.asarray(b)[uniq]) if not callable(b) else _f64(b(uniq))
    rw = None if row_w is None else _f64(np.asarray(row_w)[uniq])
    return rska_dense(Asub, bsub, lam, eta, alpha, K, inv.astype(np.int32), alpha_k=alpha_k, row_w=rw, z0=z0,
                      threads=threads)


def rska_multirhs(A, B, lam, eta, alpha, K, idx, **kw):
    """Shared-A, shared-stream multi-RHS: column r is an independent single-RHS run."""
    B = _f64(B)
    out = [rska_dense(A, B[:, r], lam, eta, alpha, K, idx, **kw) for r in range(B.shape[1])]
    return {"z": np.stack([o["z"] for o in out], axis=1), "x": np.stack([o["x"] for o in out], axis=1)}


def rska_batched(systems, **kw):
    """Independent systems, each with its own stream: a list of single-system runs."""
    return [rska_dense(s["A"], s["b"], s["lam"], s["eta"], s["alpha"], s["K"], s["idx"], **kw)
            for s in systems]


def rska_dense_adjoint(A, b, lam, eta, alpha_k, K, idx, xbar_K, *, off=0):
    """Reverse mode of K unrolled dense RSKA steps from z_0 = 0 (one RHS).

    Returns (bbar, lambda_bar, alpha_bar) for a loss whose gradient with respect
    to x_K is xbar_K.
    """
    A = _f64(A)
    b = _f64(b)
    m, n = A.shape
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ak = _f64(alpha_k)
    xb = _f64(xbar_K)
    bbar = np.zeros(m)
    lbar = np.zeros(1)
    abar = np.zeros(max(K, 1))
    st = _load().oracle_rska_dense_adjoint(m, n, n, _p(A), _p(b), float(lam), int(eta), _p(ak), int(K),
                                           _p(idx), int(off), _p(xb), _p(bbar), _p(lbar), _p(abar))
    if st:
        raise OracleError(st, "rska_dense_adjoint")
    return bbar, float(lbar[0]), abar[:K]


# ---------------------------------------------------------------------------
# Row sampler (counter-based generator + inverse CDF)
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) of a 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sampling_cdf(weights):
    """Running sums of the sampling weights ||a_i||^2 (i ascending)."""
    w = _f64(weights)
    cdf = np.zeros_like(w)
    st = _load().oracle_sampling_cdf(len(w), _p(w), _p(cdf))
    if st:
        raise OracleError(st, "sampling_cdf")
    return cdf


def sample_stream(cdf, seed, K, eta, k0=0):
    """K*eta row indices (steps k0 .. k0+K-1, step-major) drawn with Philox4x32-10 and the inverse CDF."""
    c = _f64(cdf)
    out = np.zeros(max(int(K) * int(eta), 1), dtype=np.int32)
    st = _load().oracle_sample_stream(len(c), _p(c), ctypes.c_uint64(int(seed)), int(k0), int(K), int(eta), _p(out))
    if st:
        raise OracleError(st, "sample_stream")
    return out[:int(K) * int(eta)]


# ---------------------------------------------------------------------------
# Linearized Bregman (full batch) and power iteration
# ---------------------------------------------------------------------------

def lb_dense(A, b, lam, step, K, *, check_every=0, xref=None):
    """K linearized Bregman steps x* -= step A^T(Ax - b), x = S_lambda(x*). Returns dict(z, x, res, hist)."""
    A = _f64(A)
    b = _f64(b)
    m, n = A.shape
    z = np.zeros(n)
    x = np.zeros(n)
    res = np.zeros(max(int(K), 1))
    nh = (int(K) // check_every) if (xref is not None and check_every > 0) else 0
    hist = np.full(max(nh, 1), np.nan)
    xr = None if xref is None else _f64(xref)
    st = _load().oracle_lb_dense(m, n, n, _p(A), _p(b), float(lam), float(step), int(K), _p(z), _p(x),
                                 int(check_every) if xr is not None else 0, _p(xr), _p(hist), _p(res))
    if st:
        raise OracleError(st, "lb_dense")
    return {"z": z, "x": x, "res": res[:int(K)], "hist": hist[:nh]}


def power_ata(A, iters, v0=None):
    """sigma_max(A)^2 by power iteration on A^T A (v0 defaults to v_j = 1 + (j mod 7) / 7)."""
    A = _f64(A)
    m, n = A.shape
    v = _f64(v0) if v0 is not None else 1.0 + (np.arange(n) % 7) / 7.0
    est = np.zeros(1)
    st = _load().oracle_power_ata(m, n, n, _p(A), int(iters), _p(v), _p(est))
    if st:
        raise OracleError(st, "power_ata")
    return float(est[0])


def bsk_dense(A, b, lam, w, K, idx, eta, *, off=0, z0=None, check_every=0, xref=None):
    """Block sparse Kaczmarz, eq. (bsk) (Sec. 1.1): per step k the rows tau_k = idx[off + k eta ..
    off + (k+1) eta) form A_tau (repeated indices give repeated rows), and

        x*_{k+1} = x*_k - w A_tau^T (A_tau x_k - b_tau) / ||A_tau||_2^2,   x_{k+1} = S_lambda(x*_{k+1}),

    from x*_0 = 0 (or z0), x_0 = S_lambda(x*_0). ||A_tau||_2^2 is the largest eigenvalue of
    A_tau A_tau^T. Returns dict(z, x, s2 (per step), hist).
    """
    A = _f64(A)
    b = _f64(b)
    idx = np.asarray(idx, dtype=np.int64)
    m, n = A.shape
    if eta < 1 or K < 0 or lam < 0 or not (w > 0):
        raise OracleError(INVALID, "bsk_dense")
    if K > 0 and (idx.size < off + K * eta or idx[off:off + K * eta].min() < 0
                  or idx[off:off + K * eta].max() >= m):
        raise OracleError(INDEX_RANGE, "bsk_dense")
    z = np.zeros(n) if z0 is None else _f64(z0).copy()
    x = soft_threshold(z, lam)
    s2 = np.zeros(int(K))
    nh = (int(K) // check_every) if (xref is not None and check_every > 0) else 0
    hist = np.full(nh, np.nan)
    xr = None if xref is None else _f64(xref)
    for k in range(int(K)):
        tau = idx[off + k * eta: off + (k + 1) * eta]
        At = A[tau]
        r = At @ x - b[tau]
        s2[k] = float(np.linalg.eigvalsh(At @ At.T)[-1])
        if not s2[k] > 0:
            raise OracleError(ZERO_ROW, "bsk_dense")
        z = z - (w / s2[k]) * (At.T @ r)
        x = soft_threshold(z, lam)
        if not np.all(np.isfinite(z)):
            raise OracleError(NONFINITE, "bsk_dense")
        if nh and (k + 1) % check_every == 0:
            nr = np.linalg.norm(xr)
            hist[(k + 1) // check_every - 1] = np.linalg.norm(x - xr) / (nr if nr > 0 else 1.0)
    return {"z": z, "x": x, "s2": s2, "hist": hist}

