"""ctypes declarations of libtsspgemm.so (include/tsspgemm.h).

Argument marshalling only: every computation happens in the HIP library. If
the library has not been built, loading fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsspgemm.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_MALFORMED = -2
ERR_OVERFLOW = -3
ERR_CAPACITY = -4
ERR_UNSUPPORTED = -5
ERR_HIP = -6
ERR_NOMEM = -7
ERROR_NAMES = {ERR_INVALID_ARG: "INVALID_ARG", ERR_MALFORMED: "MALFORMED", ERR_OVERFLOW: "OVERFLOW",
               ERR_CAPACITY: "CAPACITY", ERR_UNSUPPORTED: "UNSUPPORTED", ERR_HIP: "HIP", ERR_NOMEM: "NOMEM"}

PLUS_TIMES_F32 = 0
PLUS_TIMES_I32 = 1
OR_AND = 2

MASK_NONE = 0
MASK_COMPLEMENT_CSR = 1
MASK_COMPLEMENT_BITMAP = 2

SPMM_NOALLOC_MAX_BYTES = 64 << 20  # TSSPGEMM_SPMM_NOALLOC_MAX_BYTES


class CsrDesc(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class MaskDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("csr", ctypes.POINTER(CsrDesc)), ("bits", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("group_lanes", ctypes.c_int32), ("wave_max_flops", ctypes.c_int32), ("split_flops", ctypes.c_int32),
                ("sym_split_nnz", ctypes.c_int32), ("accumulator", ctypes.c_int32),
                ("light_max_flops", ctypes.c_int32), ("products", ctypes.c_int32)]


class TSSpGEMMError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


_lib = None

P = ctypes.POINTER
vp = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64

_SIGNATURES = {
    "tsspgemm_bitmap_words": (i32, [i32]),
    "tsspgemm_symbolic": (ctypes.c_int, [P(CsrDesc), P(CsrDesc), i32, P(MaskDesc), P(Tuning), vp, P(i64), P(vp), vp]),
    "tsspgemm_numeric": (ctypes.c_int, [vp, P(CsrDesc), P(CsrDesc), vp, vp, vp]),
    "tsspgemm_plan_stats": (ctypes.c_int, [vp, P(i64), P(i64), P(i64), P(i64), P(i64), P(i64)]),
    "tsspgemm_plan_destroy": (None, [vp]),
    "tsspgemm_masked_bool": (ctypes.c_int, [P(CsrDesc), P(CsrDesc), P(MaskDesc), vp, vp, i64, P(i64), vp]),
    "tsspgemm_msbfs": (ctypes.c_int, [P(CsrDesc), vp, i32, vp, P(i32), vp, i32, vp]),
    "tsspgemm_transpose": (ctypes.c_int, [P(CsrDesc), vp, vp, vp, vp]),
    "tsspgemm_grad_a": (ctypes.c_int, [vp, P(CsrDesc), P(CsrDesc), P(CsrDesc), vp, vp]),
    "tsspgemm_grad_b": (ctypes.c_int, [vp, P(CsrDesc), vp, P(CsrDesc), P(CsrDesc), P(CsrDesc), vp, vp]),
    "tsspgemm_backward": (ctypes.c_int, [vp, P(CsrDesc), vp, P(CsrDesc), P(CsrDesc), P(CsrDesc), vp, vp, vp]),
    "tsspgemm_spmm": (ctypes.c_int, [P(CsrDesc), vp, i64, i64, vp, i64, vp]),
    "tsspgemm_spmm_noalloc": (ctypes.c_int, [P(CsrDesc), vp, i64, i64, vp, i64, vp]),
    "tsspgemm_column_slice_count": (ctypes.c_int, [P(CsrDesc), ctypes.c_int32, ctypes.c_int32, vp, P(i64), vp]),
    "tsspgemm_column_slice_fill": (ctypes.c_int, [P(CsrDesc), ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]),
    "tsspgemm_merge_count": (ctypes.c_int, [ctypes.c_int32, P(CsrDesc), vp, P(i64), vp]),
    "tsspgemm_merge_values": (ctypes.c_int, [ctypes.c_int32, P(CsrDesc), vp, vp, vp, vp]),
    "tsspgemm_embed_epoch": (ctypes.c_int, [P(CsrDesc), i64, i64, vp, vp, ctypes.c_float, i64, i64, i64, vp]),
    "tsspgemm_batched_plan": (ctypes.c_int, [i32, P(CsrDesc), P(CsrDesc), P(Tuning), P(vp), P(i64), P(i64), vp]),
    "tsspgemm_batched_run": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
    "tsspgemm_batched_capture": (ctypes.c_int, [vp, vp, vp, vp, vp]),
    "tsspgemm_batched_launch": (ctypes.c_int, [vp, vp]),
    "tsspgemm_batched_flops": (ctypes.c_int, [vp, P(i64)]),
    "tsspgemm_batched_destroy": (None, [vp]),
    "tsspgemm_last_error": (ctypes.c_char_p, []),
    "tsspgemm_version": (ctypes.c_char_p, []),
}

EXPORTED = tuple(_SIGNATURES)


def load(path: str = LIB_PATH):
    """Load libtsspgemm.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(code: int, where: str):
    if code != OK:
        msg = load().tsspgemm_last_error()
        raise TSSpGEMMError(code, where, msg.decode() if msg else "")
