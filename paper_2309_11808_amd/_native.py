"""ctypes loader for libspod.so (the C ABI declared in include/spod.h).

Importing this module never builds anything and never falls back to another
implementation: if the shared library is missing the import fails with a
message that says how to build it.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspod.so")

SPOD_OK = 0
SPOD_ERR_INVALID_ARG = -1
SPOD_ERR_UNSUPPORTED = -2
SPOD_ERR_ALLOC = -3
SPOD_ERR_HIP = -4
SPOD_ERR_NUMERIC = -5
SPOD_ERR_WORKSPACE = -6
SPOD_ERR_IO = -7
SPOD_ERR_INTERNAL = -8

SPOD_F32 = 0
SPOD_F64 = 1

SPOD_INFO_NONFINITE = -2147483648   # spod_eig info of a non-finite Gram matrix
SPOD_CSD_NOALLOC_MAX_BYTES = 64 << 20

SPOD_PREC_FP64 = 0
SPOD_PREC_FP32 = 1
SPOD_PREC_BF16X4 = 2
SPOD_PREC_FP16X4 = 3

SPOD_OPT_MAX_SWEEPS = 0
SPOD_OPT_GRAM_SPLIT = 1
SPOD_OPT_FFT_TILE = 2
SPOD_OPT_QHAT_FORMAT = 3
SPOD_OPT_MODES_KERNEL = 4
SPOD_OPT_GENERAL_PASSES = 5

SPOD_QHAT_COMPLEX = 0
SPOD_QHAT_BFP20 = 1

SPOD_BATCH_GROUPED = 0
SPOD_BATCH_GRAPH = 1
SPOD_BATCH_GRAM_TARGET = 2
SPOD_BATCH_FFT_TILE = 3
SPOD_BATCH_EIG_THREADS = 4
SPOD_BATCH_PERSISTENT = 5


class SpodProblem(C.Structure):
    _fields_ = [("nspace", C.c_int64), ("nvar", C.c_int64), ("nt", C.c_int64),
                ("nfft", C.c_int64), ("noverlap", C.c_int64), ("window", C.c_void_p),
                ("weights", C.c_void_p)]


class SpodBatchItem(C.Structure):
    _fields_ = [("M", C.c_int64), ("nblocks", C.c_int64), ("nfreq", C.c_int64),
                ("n_modes", C.c_int64), ("mean", C.c_size_t), ("lam", C.c_size_t),
                ("psi", C.c_size_t), ("info", C.c_size_t), ("phi", C.c_size_t),
                ("n_valid", C.c_size_t)]

_i64 = C.c_int64
_p = C.c_void_p
_sz = C.c_size_t

# int (*spod_read_fn)(void* user, int64_t row0, int64_t nrows, void* dst)
READ_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p)

# name -> (restype, argtypes); exactly the functions of include/spod.h
SIGNATURES = {
    "spod_plan_create": (C.c_int, [_i64, _i64, _i64, _i64, _i64, _p, _p, C.POINTER(_p)]),
    "spod_shape": (C.c_int, [_i64, _i64, _i64, C.POINTER(_i64), C.POINTER(_i64)]),
    "spod_plan_set_precision": (C.c_int, [_p, C.c_int]),
    "spod_plan_set_option": (C.c_int, [_p, C.c_int, _i64]),
    "spod_plan_query": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_sz)]),
    "spod_plan_qhat_bytes": (C.c_int, [_p, C.POINTER(_sz)]),
    "spod_blocks_fft": (C.c_int, [_p, _p, C.c_int, _p, _p, _p, _sz, _p]),
    "spod_csd": (C.c_int, [_p, _p, _p, _p, _sz, _p]),
    "spod_csd_noalloc": (C.c_int, [_p, _p, _p, C.POINTER(_i64), _p]),
    "spod_eig": (C.c_int, [_p, _p, _p, _p, _p, _p, _sz, _p]),
    "spod_modes": (C.c_int, [_p, _p, _p, _p, _i64, _p, _p, _p, _sz, _p]),
    "spod_backward": (C.c_int, [_p, _p, C.c_int, _p, _p, _p, _p, _p, _i64, _p, _i64, _p, _p, _p,
                                _sz, _p]),
    "spod_plan_destroy": (None, [_p]),
    "spod_batch_create": (C.c_int, [C.POINTER(SpodProblem), _i64, C.c_int, _i64, C.POINTER(_p)]),
    "spod_batch_set_option": (C.c_int, [_p, C.c_int, _i64]),
    "spod_batch_get_option": (C.c_int, [_p, C.c_int, C.POINTER(_i64)]),
    "spod_batch_query": (C.c_int, [_p, C.POINTER(_sz), C.POINTER(_sz)]),
    "spod_batch_item_info": (C.c_int, [_p, _i64, C.POINTER(SpodBatchItem)]),
    "spod_batch_forward": (C.c_int, [_p, C.POINTER(_p), C.c_int, _p, _p, _sz, _p]),
    "spod_batch_autotune": (C.c_int, [_p, C.POINTER(_p), C.c_int, _p, _p, _sz, _p, C.c_char_p,
                                      C.POINTER(_i64)]),
    "spod_batch_destroy": (None, [_p]),
    "spod_coeffs_query": (C.c_int, [_p, _i64, _i64, C.POINTER(_sz)]),
    "spod_coeffs": (C.c_int, [_p, _p, C.c_int, _p, _p, _i64, _p, _i64, _i64, _p, _p, _p, _sz, _p]),
    "spod_reconstruct": (C.c_int, [_p, _p, _i64, _p, _i64, _i64, _p, _p, _p, C.c_int, _p]),
    "spod_ooc_create": (C.c_int, [_p, C.c_int, _i64, _i64, _i64, C.POINTER(_p)]),
    "spod_ooc_query": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64),
                                 C.POINTER(_sz), C.POINTER(_sz)]),
    "spod_ooc_forward": (C.c_int, [_p, _p, READ_FN, _p, _p, _p, _p, _p, _p, _p, _p]),
    "spod_ooc_destroy": (None, [_p]),
    "spod_status_string": (C.c_char_p, [C.c_int]),
    "spod_last_error": (C.c_char_p, []),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"libspod.so not found at {path}; build it with "
            "`python -m paper_2309_11808_amd.build` (needs ROCm hipcc)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class SpodError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status
