"""ctypes declarations of the libkrp C ABI (include/krp.h).

Argument marshalling only: every computation runs in libkrp's HIP kernels.
Loading fails loudly (RuntimeError) when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrp.so")

KRP_OK, KRP_EINVAL, KRP_ENOMEM, KRP_EHIP, KRP_ECHOL, KRP_ENONFINITE, KRP_ENODEV, KRP_ESINGULAR = range(8)
KRP_F64, KRP_F32 = 0, 1
KRP_P_FP64, KRP_P_FP32, KRP_P_BF16, KRP_P_BF16X3 = 0, 1, 2, 3
KRP_STAT_CHOL_SHIFT, KRP_STAT_CHOL_FAIL, KRP_STAT_NONFINITE, KRP_STAT_SINGULAR = 1, 2, 4, 8
KRP_FLAG_NO_GRAPH, KRP_FLAG_AUTOTUNE, KRP_FLAG_MEMO, KRP_FLAG_GAUSSIAN = 1, 2, 4, 8

# Every function declared in include/krp.h.
EXPORTED = (
    "krp_opts_default", "krp_sketch", "krp_hosvd", "krp_sthosvd", "krp_hankel_lowrank",
    "krp_workspace_size", "krp_hankel_workspace_size", "krp_gaussian", "krp_status_string",
    "krp_last_error", "krp_version", "krp_finalize", "krp_sketch_noalloc", "krp_noalloc_scratch_bytes",
    "krp_range_factors", "krp_sensor_select", "krp_sensor_measure", "krp_sensor_reconstruct",
    "krp_sensor_workspace_size", "krp_kron_lowrank", "krp_kron_nystrom",
)


class KrpOpts(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("draw", ctypes.c_uint32),
        ("prec", ctypes.c_int32),
        ("truncate", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("status_dev", ctypes.c_void_p),
        ("rel_err", ctypes.POINTER(ctypes.c_double)),
    ]


class KrpError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libkrp.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2507_23207_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64P = ctypes.POINTER(ctypes.c_int64)
        I32P = ctypes.POINTER(ctypes.c_int32)
        OP = ctypes.POINTER(KrpOpts)
        i, i32 = ctypes.c_int, ctypes.c_int32
        L.krp_opts_default.argtypes = [OP]
        L.krp_opts_default.restype = None
        L.krp_sketch.argtypes = [P, i, i, I64P, i, I32P, I32P, OP, ctypes.POINTER(P), P]
        L.krp_sketch.restype = i
        L.krp_sketch_noalloc.argtypes = [P, i, i, I64P, i, I32P, I32P, OP, ctypes.POINTER(P), P]
        L.krp_sketch_noalloc.restype = i
        L.krp_noalloc_scratch_bytes.argtypes = []
        L.krp_noalloc_scratch_bytes.restype = ctypes.c_size_t
        for name in ("krp_hosvd", "krp_sthosvd"):
            f = getattr(L, name)
            f.argtypes = [P, i, i, I64P, I32P, i32, OP, P, ctypes.POINTER(P), I64P, P]
            f.restype = i
        L.krp_kron_lowrank.argtypes = [i, i, i, i, i, P, P, i, i, i, i, OP, P, P, P, P]
        L.krp_kron_lowrank.restype = i
        L.krp_kron_nystrom.argtypes = [i, i, i, P, P, i, i, i, OP, P, P, P]
        L.krp_kron_nystrom.restype = i
        L.krp_range_factors.argtypes = [P, i, i, I64P, i, I32P, I32P, OP, ctypes.POINTER(P), P]
        L.krp_range_factors.restype = i
        L.krp_sensor_select.argtypes = [i, I64P, I32P, i, ctypes.POINTER(P), OP, ctypes.POINTER(P),
                                        ctypes.POINTER(P), P]
        L.krp_sensor_select.restype = i
        L.krp_sensor_measure.argtypes = [P, i, i, I64P, ctypes.c_int64, I32P, ctypes.POINTER(P), P, P]
        L.krp_sensor_measure.restype = i
        L.krp_sensor_reconstruct.argtypes = [P, i, i, I64P, ctypes.c_int64, I32P, ctypes.POINTER(P), OP, P, P]
        L.krp_sensor_reconstruct.restype = i
        L.krp_sensor_workspace_size.argtypes = [i, i, I64P, I32P, ctypes.c_int64, i,
                                                ctypes.POINTER(ctypes.c_size_t)]
        L.krp_sensor_workspace_size.restype = i
        L.krp_hankel_lowrank.argtypes = [i, I64P, i, i, P, i, i, i, i, OP, P, P, P, P]
        L.krp_hankel_lowrank.restype = i
        L.krp_workspace_size.argtypes = [i, i, i, I64P, I32P, i32, i, ctypes.POINTER(ctypes.c_size_t)]
        L.krp_workspace_size.restype = i
        L.krp_hankel_workspace_size.argtypes = [i, I64P, i, i, i, i, i, ctypes.POINTER(ctypes.c_size_t)]
        L.krp_hankel_workspace_size.restype = i
        L.krp_gaussian.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64, i, P, P]
        L.krp_gaussian.restype = i
        L.krp_status_string.argtypes = [i]
        L.krp_status_string.restype = ctypes.c_char_p
        L.krp_last_error.argtypes = []
        L.krp_last_error.restype = ctypes.c_char_p
        L.krp_version.argtypes = []
        L.krp_version.restype = ctypes.c_char_p
        L.krp_finalize.argtypes = []
        L.krp_finalize.restype = i
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != KRP_OK:
        L = lib()
        msg = L.krp_last_error().decode() or L.krp_status_string(rc).decode()
        raise KrpError(rc, msg)


def i64_array(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def i32_array(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(int(p) if p else 0) for p in ptrs])
