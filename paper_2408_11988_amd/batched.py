"""Batched plus-times TS-SpGEMM over the C ABI (tsspgemm_batched_*).

All instances run as one set of launches (every phase covers the whole batch);
the run can be captured once in a HIP graph and replayed. torch only supplies
the output buffers and the stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .api import DeviceCsr, _stream_ptr, tuning_struct


class Batched:
    """Plan for C_t = A_t B_t, t = 0..count-1 (patterns fixed, values may change)."""

    def __init__(self, pairs, tunings: list | None = None, stream=None):
        self.pairs = [(A, B) for A, B in pairs]
        count = len(self.pairs)
        self.count = count
        self._as = (_lib.CsrDesc * max(count, 1))(*[A.desc() for A, _ in self.pairs])
        self._bs = (_lib.CsrDesc * max(count, 1))(*[B.desc() for _, B in self.pairs])
        tarr = None
        if tunings is not None:
            assert len(tunings) == count
            tarr = (_lib.Tuning * max(count, 1))(*[tuning_struct(t) for t in tunings])
        self._tunings = tarr
        self.handle = ctypes.c_void_p(None)
        pool = ctypes.c_int64(0)
        rp_total = ctypes.c_int64(0)
        lib = _lib.load()
        rc = lib.tsspgemm_batched_plan(count, self._as, self._bs, tarr, ctypes.byref(self.handle),
                                       ctypes.byref(pool), ctypes.byref(rp_total), _stream_ptr(stream))
        _lib.check(rc, "tsspgemm_batched_plan")
        self.pool = int(pool.value)
        dev = self.pairs[0][0].rowptr.device if count else torch.device("cuda")
        self.c_rowptrs = torch.empty(max(int(rp_total.value), 1), dtype=torch.int32, device=dev)
        self.pool_colidx = torch.empty(max(self.pool, 1), dtype=torch.int32, device=dev)
        self.pool_vals = torch.empty(max(self.pool, 1), dtype=torch.float32, device=dev)
        self.c_offsets = torch.empty(count + 1, dtype=torch.int64, device=dev)
        self.captured = False

    def _ptrs(self):
        return (ctypes.c_void_p(self.c_rowptrs.data_ptr()), ctypes.c_void_p(self.pool_colidx.data_ptr()),
                ctypes.c_void_p(self.pool_vals.data_ptr()), ctypes.c_void_p(self.c_offsets.data_ptr()))

    def run(self, stream=None):
        """Queue one batched run (no host synchronisation)."""
        rc = _lib.load().tsspgemm_batched_run(self.handle, *self._ptrs(), _stream_ptr(stream))
        _lib.check(rc, "tsspgemm_batched_run")

    def capture(self):
        """Record the run into a HIP graph held by the batch."""
        rc = _lib.load().tsspgemm_batched_capture(self.handle, *self._ptrs())
        _lib.check(rc, "tsspgemm_batched_capture")
        self.captured = True

    def replay(self, stream=None):
        rc = _lib.load().tsspgemm_batched_launch(self.handle, _stream_ptr(stream))
        _lib.check(rc, "tsspgemm_batched_launch")

    def outputs(self) -> list[DeviceCsr]:
        """Per-instance C as views into the pool (after the run completed)."""
        off = self.c_offsets.cpu().tolist()
        out = []
        rp0 = 0
        for t, (A, B) in enumerate(self.pairs):
            n = A.nrows
            rp = self.c_rowptrs[rp0:rp0 + n + 1]
            rp0 += n + 1
            out.append(DeviceCsr(n, B.ncols, rp, self.pool_colidx[off[t]:off[t + 1]],
                                 self.pool_vals[off[t]:off[t + 1]]))
        return out

    def flops(self) -> list[int]:
        arr = (ctypes.c_int64 * max(self.count, 1))()
        _lib.check(_lib.load().tsspgemm_batched_flops(self.handle, arr), "tsspgemm_batched_flops")
        return [int(arr[t]) for t in range(self.count)]

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                _lib.load().tsspgemm_batched_destroy(self.handle)
        except Exception:
            pass
