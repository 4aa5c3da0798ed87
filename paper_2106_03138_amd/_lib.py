"""ctypes binding to libqrdm.so (include/qrdm.h).  Argument marshalling only:
every step of the factorization runs in the library's HIP kernels.  PyTorch
provides device memory and the stream."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqrdm.so")

STOP_PAPER, STOP_MAXNORM, STOP_NONE = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
ERR_NONFINITE, ERR_NOMEM, ERR_UNSUPPORTED, ERR_INTERNAL, ERR_WORKSPACE, ERR_SCRATCH, ERR_HIP = 1, 2, 3, 4, 5, 6, 1000
NOALLOC_WS_MAX = 96 << 20


class Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("delta", ctypes.c_double), ("kmax", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("eps1_scale", ctypes.c_double),
                ("precision", ctypes.c_int32), ("poll_lag", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("certified", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int64), ("nbreaks", ctypes.c_int64), ("nfallback", ctypes.c_int64),
                ("nrecompute", ctypes.c_int64), ("ncols_factored", ctypes.c_int64),
                ("gemm1_ms", ctypes.c_double), ("gemm2_ms", ctypes.c_double), ("gemm_flop", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("dm_ms", ctypes.c_double), ("panel_ms", ctypes.c_double),
                ("downdate_ms", ctypes.c_double), ("qp3_ms", ctypes.c_double), ("panel_flop", ctypes.c_double),
                ("panel_bytes", ctypes.c_double), ("npanel", ctypes.c_int64),
                ("qp3_run_ms", ctypes.c_double), ("qp3_bytes", ctypes.c_double), ("nqp3_launch", ctypes.c_int64),
                ("qp3_start", ctypes.c_int64), ("ngram", ctypes.c_int64),
                ("nqp3_tail", ctypes.c_int64), ("zsum_ms", ctypes.c_double), ("gemm2_bytes", ctypes.c_double)]


class Block(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int64), ("nL", ctypes.c_int32), ("ks", ctypes.c_int32),
                ("l", ctypes.c_int32), ("fallback", ctypes.c_int32), ("umax", ctypes.c_double),
                ("gamma", ctypes.c_double), ("sigma_bound", ctypes.c_double)]


class BatchParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("delta", ctypes.c_double), ("kmax", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class BatchTune(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32)]


BATCH_NMAX, BATCH_KMAX, BATCH_CLASSES = 512, 64, 4
NFEAT, MLP_HIDDEN, MLP_OUT, MLP_NPARAM, MLP_NDELTA = 16, 64, 3, 5443, 131


class QrdmError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with code {code}: {msg}")
        self.code = code


# (name, restype, argtypes) of every exported symbol declared in include/qrdm.h
_vp, _i64, _i32, _d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_P = ctypes.POINTER
SIGNATURES = {
    "qrdm_default_params": (None, [_P(Params)]),
    "qrdm_factor": (ctypes.c_int, [_vp, _i64, _i64, _i64, _d, _d, _i32, _vp, _vp, _P(_i64), _vp]),
    "qrdm_factor_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _P(Params), _vp, _vp, _P(_i64), _P(Stats),
                                      _P(Block), _i64, _P(_i64), _vp]),
    "qrdm_workspace_size": (ctypes.c_size_t, [_i64, _i64, _P(Params)]),
    "qrdm_factor_ws": (ctypes.c_int, [_vp, _i64, _i64, _i64, _P(Params), _vp, _vp, _vp, _P(Stats), _vp,
                                      ctypes.c_size_t, _vp]),
    "qrdm_factor_noalloc": (ctypes.c_int, [_vp, _i64, _i64, _i64, _P(Params), _vp, _vp, _vp, _vp]),
    "qrp_factor": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _vp, _P(_i64), _vp]),
    "qrp_factor_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _P(Params), _i32, _vp, _vp, _P(_i64), _P(Stats), _vp]),
    "qrdm_colnorms": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _vp]),
    "qrdm_dm_step": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _vp, _d, _d, _i32, _P(_i32), _P(_i32),
                                    _P(_d), _P(_i32), _P(_i32), _vp]),
    "qrdm_lstsq": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _vp]),
    "qrdm_truncate_rank": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _d, _vp, _vp]),
    "qrdm_release": (None, []),
    "qrdm_batch_plan_create": (ctypes.c_int, [_P(_i32), _P(_i32), _P(_i32), _i32, _P(Params), _P(BatchTune),
                                              _P(_vp)]),
    "qrdm_batch_factor": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "qrdm_batch_factor_checked": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp,
                                                 _vp]),
    "qrdm_batch_features": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "qrdm_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "qrdm_mlp_gradient": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "qrdm_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, _vp]),
    "qrdm_mlp_to_params": (ctypes.c_int, [_vp, _i32, _vp, _vp]),
    "qrdm_batch_check": (ctypes.c_int, [_vp, _vp, _vp, _d, _vp, _vp, _vp]),
    "qrdm_batch_plan_destroy": (None, [_vp]),
    "qrdm_batch_lstsq": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp]),
    "qrdm_batch_truncate_rank": (ctypes.c_int, [_vp, _vp, _vp, _d, _vp, _vp]),
    "qrdm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_LIB = None


def load(path: str = LIB_PATH):
    """Load libqrdm.so.  Raises if it has not been built: there is no fallback."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2106_03138_amd.build` "
                           "(the HIP library is required; there is no CPU fallback)")
    # One HIP runtime per process: torch ships libamdhip64.so.7 and must be loaded
    # first so that libqrdm.so binds to the same runtime (device memory and
    # streams come from torch).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(fn: str, code: int):
    if code != 0:
        msg = load().qrdm_strerror(code).decode()
        raise QrdmError(fn, code, msg)
