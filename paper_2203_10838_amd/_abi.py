"""ctypes declarations of the C ABI in include/rsk.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librsk.so")

RSK_F32, RSK_F64 = 0, 1
NOALLOC_SCRATCH_BYTES = 8 << 20
STATUS_NAMES = {
    0: "RSK_OK", 1: "RSK_ERR_INVALID_ARG", 2: "RSK_ERR_UNSUPPORTED", 3: "RSK_ERR_WORKSPACE",
    4: "RSK_ERR_HIP", 5: "RSK_ERR_ZERO_ROW", 6: "RSK_ERR_INDEX_RANGE", 7: "RSK_ERR_NONFINITE",
    8: "RSK_ERR_ABORTED",
}

c_i64, c_i32, c_dbl, c_vp, c_sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class RskDense(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("ld", c_i64), ("dtype", c_i32), ("val", c_vp)]


class RskCsr(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("nnz", c_i64), ("dtype", c_i32), ("row_ptr", c_vp),
                ("col", c_vp), ("val", c_vp)]


class RskParams(ctypes.Structure):
    _fields_ = [("lambda_", c_dbl), ("eta", c_i32), ("alpha", c_dbl), ("alpha_k", c_vp), ("K", c_i64),
                ("index_stream", c_vp), ("stream_offset", c_i64), ("rownorm2", c_vp), ("warm_start", c_i32),
                ("x_ref", c_vp), ("check_every", c_i64), ("tol", c_dbl), ("err_hist", c_vp), ("y_out", c_vp),
                ("status_dev", c_vp), ("grid", c_i32), ("kernel", c_i32), ("row_w", c_vp)]


class RskBatchItem(ctypes.Structure):
    _fields_ = [("A", c_vp), ("m", c_i64), ("n", c_i64), ("ld", c_i64), ("b", c_vp), ("rownorm2", c_vp),
                ("index_stream", c_vp), ("K", c_i64), ("eta", c_i32), ("warm_start", c_i32), ("alpha", c_dbl),
                ("lambda_", c_dbl), ("x_star", c_vp), ("x", c_vp), ("x_ref", c_vp), ("check_every", c_i64),
                ("tol", c_dbl), ("err_hist", c_vp), ("status_dev", c_vp)]


class RskTuneEntry(ctypes.Structure):
    _fields_ = [("path", c_i32), ("dtype", c_i32), ("m", c_i64), ("n", c_i64), ("eta", c_i32), ("R", c_i32),
                ("v0", c_i64), ("v1", c_i64), ("v2", c_i64), ("us", c_dbl)]


RSK_TUNE_DENSE, RSK_TUNE_MULTIRHS, RSK_TUNE_BATCHED = 0, 1, 2


class RskLbParams(ctypes.Structure):
    _fields_ = [("lambda_", c_dbl), ("step", c_dbl), ("K", c_i64), ("warm_start", c_i32), ("x_ref", c_vp),
                ("check_every", c_i64), ("err_hist", c_vp), ("res_hist", c_vp), ("status_dev", c_vp)]


# name -> (restype, argtypes); every symbol include/rsk.h declares
SIGNATURES = {
    "rsk_abi_version": (c_i32, []),
    "rsk_tune_set": (c_i32, [ctypes.POINTER(RskTuneEntry)]),
    "rsk_tune_get": (c_i32, [ctypes.POINTER(RskTuneEntry), ctypes.POINTER(RskTuneEntry), ctypes.POINTER(c_i32)]),
    "rsk_tune_erase": (c_i32, [ctypes.POINTER(RskTuneEntry)]),
    "rsk_tune_clear": (c_i32, [c_i32]),
    "rsk_tune_load": (c_i32, [ctypes.c_char_p]),
    "rsk_tune_save": (c_i32, [ctypes.c_char_p]),
    "rsk_status_string": (ctypes.c_char_p, [c_i32]),
    "rsk_rownorm2_dense": (c_i32, [ctypes.POINTER(RskDense), c_vp, c_vp]),
    "rsk_workspace_size_dense": (c_i32, [ctypes.POINTER(RskDense), ctypes.POINTER(RskParams),
                                         ctypes.POINTER(c_sz)]),
    "rsk_avg_solve_dense": (c_i32, [ctypes.POINTER(RskDense), c_vp, ctypes.POINTER(RskParams), c_vp, c_vp,
                                    c_vp, c_sz, c_vp]),
    "rsk_avg_solve_dense_noalloc": (c_i32, [ctypes.POINTER(RskDense), c_vp, ctypes.POINTER(RskParams), c_vp, c_vp,
                                            c_vp]),
    "rsk_plan_dense": (c_i32, [ctypes.POINTER(RskDense), ctypes.POINTER(RskParams), ctypes.POINTER(c_i32)]),
    "rsk_rownorm2_csr": (c_i32, [ctypes.POINTER(RskCsr), c_vp, c_vp]),
    "rsk_avg_solve_multirhs_ckpt": (c_i32, [ctypes.POINTER(RskDense), c_vp, c_i32, ctypes.POINTER(RskParams), c_i32,
                                            c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "rsk_workspace_size_adjoint": (c_i32, [ctypes.POINTER(RskDense), c_i32, ctypes.POINTER(RskParams), c_i32,
                                           ctypes.POINTER(c_sz)]),
    "rsk_avg_adjoint": (c_i32, [ctypes.POINTER(RskDense), c_vp, c_i32, ctypes.POINTER(RskParams), c_i32, c_vp, c_vp,
                                c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "rsk_workspace_size_sampling_cdf": (c_i32, [c_i64, ctypes.POINTER(c_sz)]),
    "rsk_sampling_cdf_dense": (c_i32, [ctypes.POINTER(RskDense), c_vp, c_vp, c_sz, c_vp]),
    "rsk_sampling_cdf_dense_weighted": (c_i32, [ctypes.POINTER(RskDense), c_vp, c_vp, c_vp, c_sz, c_vp]),
    "rsk_sampling_cdf_weights": (c_i32, [c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "rsk_sample_stream": (c_i32, [c_vp, c_i64, ctypes.c_uint64, c_i64, c_i64, c_i32, c_vp, c_vp]),
    "rsk_workspace_size_lb_dense": (c_i32, [ctypes.POINTER(RskDense), ctypes.POINTER(c_sz)]),
    "rsk_lb_solve_dense": (c_i32, [ctypes.POINTER(RskDense), c_vp, ctypes.POINTER(RskLbParams), c_vp, c_vp, c_vp, c_sz,
                                   c_vp]),
    "rsk_spectral_norm2_dense": (c_i32, [ctypes.POINTER(RskDense), c_i64, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "rsk_workspace_size_bsk_dense": (c_i32, [ctypes.POINTER(RskDense), ctypes.POINTER(RskParams),
                                             ctypes.POINTER(c_sz)]),
    "rsk_bsk_solve_dense": (c_i32, [ctypes.POINTER(RskDense), c_vp, ctypes.POINTER(RskParams), c_vp, c_vp, c_vp,
                                    c_vp, c_sz, c_vp]),
    "rsk_workspace_size_batched": (c_i32, [c_i32, c_i32, c_vp, c_i64, c_i32, ctypes.POINTER(c_sz)]),
    "rsk_avg_solve_batched": (c_i32, [c_i32, c_i32, c_vp, c_vp, c_vp, c_i64, c_i32, c_vp, c_sz, c_vp]),
    "rsk_plan_batched": (c_i32, [c_i32, c_i32, c_vp, c_i64, c_i32, c_vp, c_vp]),
    "rsk_gather_rate_dense": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i32, c_i32, c_vp, c_vp]),
    "rsk_workspace_size_multirhs": (c_i32, [ctypes.POINTER(RskDense), c_i32, ctypes.POINTER(RskParams),
                                            ctypes.POINTER(c_sz)]),
    "rsk_avg_solve_multirhs": (c_i32, [ctypes.POINTER(RskDense), c_vp, c_i32, ctypes.POINTER(RskParams), c_vp, c_vp,
                                       c_vp, c_sz, c_vp]),
    "rsk_plan_multirhs": (c_i32, [ctypes.POINTER(RskDense), c_i32, ctypes.POINTER(RskParams), ctypes.POINTER(c_i32)]),
    "rsk_workspace_size_csr": (c_i32, [ctypes.POINTER(RskCsr), ctypes.POINTER(RskParams), ctypes.POINTER(c_sz)]),
    "rsk_avg_solve_csr": (c_i32, [ctypes.POINTER(RskCsr), c_vp, ctypes.POINTER(RskParams), c_vp, c_vp,
                                  c_vp, c_sz, c_vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load librsk.so and declare its signatures. Raises if the library is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"librsk.so not built ({path}); run `python -m paper_2203_10838_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
