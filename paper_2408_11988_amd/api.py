"""Python face of libtsspgemm.so: marshals torch device tensors into the C ABI.

Nothing here computes: shapes are checked, buffers are allocated with torch
on the current device, and the library is called on torch's current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import TSSpGEMMError  # noqa: F401

SEMIRINGS = {"plus_times": _lib.PLUS_TIMES_F32, "plus_times_f32": _lib.PLUS_TIMES_F32,
             "plus_times_i32": _lib.PLUS_TIMES_I32, "or_and": _lib.OR_AND}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class DeviceCsr:
    """CSR on the GPU: int32 rowptr (nrows+1), int32 colidx (nnz), values or None."""

    nrows: int
    ncols: int
    rowptr: torch.Tensor
    colidx: torch.Tensor
    vals: torch.Tensor | None = None

    @property
    def nnz(self) -> int:
        return int(self.colidx.numel())

    @staticmethod
    def from_host(m, device="cuda", dtype=torch.float32, with_values=True) -> "DeviceCsr":
        """From any host CSR with .nrows .ncols .rp .ci (.val) numpy arrays."""
        rp = torch.from_numpy(np.ascontiguousarray(m.rp, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(m.ci, dtype=np.int32)).to(device)
        v = None
        if with_values and getattr(m, "val", None) is not None:
            v = torch.from_numpy(np.ascontiguousarray(m.val)).to(device=device, dtype=dtype)
        return DeviceCsr(int(m.nrows), int(m.ncols), rp, ci, v)

    def with_vals(self, vals: torch.Tensor | None) -> "DeviceCsr":
        return DeviceCsr(self.nrows, self.ncols, self.rowptr, self.colidx, vals)

    def desc(self) -> _lib.CsrDesc:
        if self.rowptr.dtype != torch.int32 or self.colidx.dtype != torch.int32:
            raise TypeError("rowptr and colidx must be int32")
        if not (self.rowptr.is_cuda and self.colidx.is_cuda):
            raise TypeError("CSR arrays must live on the GPU")
        if self.rowptr.numel() != self.nrows + 1:
            raise ValueError("rowptr must have nrows + 1 entries")
        for t in (self.rowptr, self.colidx, self.vals):
            if t is not None and not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous")
        return _lib.CsrDesc(self.nrows, self.ncols, self.nnz, self.rowptr.data_ptr(),
                            self.colidx.data_ptr() if self.nnz else None,
                            self.vals.data_ptr() if self.vals is not None and self.nnz else None)

    def to_host(self):
        return (self.rowptr.cpu().numpy(), self.colidx.cpu().numpy(),
                None if self.vals is None else self.vals.cpu().numpy())


ACCUMULATORS = {"auto": 0, "lds": 1, "hash": 2}


def accumulator_code(v) -> int:
    """Accumulator as the C enum value (names: auto, lds, hash)."""
    return ACCUMULATORS[v] if isinstance(v, str) else int(v)


PRODUCTS = {"auto": 0, "rows": 1, "flat": 2, "vec4": 3}


def tuning_struct(t: dict) -> _lib.Tuning:
    """A tuning dict (missing keys: defaults) as the C struct."""
    prod = t.get("products", 0)
    return _lib.Tuning(int(t.get("group_lanes", 0)), int(t.get("wave_max_flops", 0)), int(t.get("split_flops", 0)),
                       int(t.get("sym_split_nnz", 0)), accumulator_code(t.get("accumulator", 0)),
                       int(t.get("light_max_flops", 0)), PRODUCTS[prod] if isinstance(prod, str) else int(prod))


def _tuning(t: dict | None):
    if not t:
        return None
    return ctypes.byref(tuning_struct(t))


class Plan:
    """Owns a tsspgemm_plan (symbolic result + workspace); reusable."""

    def __init__(self):
        self.handle = ctypes.c_void_p(None)
        self.semiring = None
        self.c_rowptr = None
        self.nnz = 0

    def stats(self) -> dict:
        vals = [ctypes.c_int64() for _ in range(6)]
        _lib.check(_lib.load().tsspgemm_plan_stats(self.handle, *[ctypes.byref(v) for v in vals]), "plan_stats")
        keys = ("flops", "nnz", "light_rows", "wave_rows", "block_rows", "split_rows")
        return {k: int(v.value) for k, v in zip(keys, vals)}

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                _lib.load().tsspgemm_plan_destroy(self.handle)
        except Exception:
            pass


def _mask_desc(mask, keep):
    """mask: None, a DeviceCsr (complement by pattern) or a uint32/int32 bitmap tensor."""
    if mask is None:
        return None
    if isinstance(mask, DeviceCsr):
        d = mask.desc()
        keep.append(d)
        return ctypes.byref(_lib.MaskDesc(_lib.MASK_COMPLEMENT_CSR, ctypes.pointer(d), None))
    if isinstance(mask, torch.Tensor):
        if not mask.is_cuda or mask.dtype not in (torch.int32, torch.uint32) or not mask.is_contiguous():
            raise TypeError("bitmap mask must be a contiguous int32/uint32 CUDA tensor")
        return ctypes.byref(_lib.MaskDesc(_lib.MASK_COMPLEMENT_BITMAP, None, mask.data_ptr()))
    raise TypeError("mask must be None, a DeviceCsr or a bitmap tensor")


def symbolic(A: DeviceCsr, B: DeviceCsr, semiring="plus_times", mask=None, tuning: dict | None = None,
             plan: Plan | None = None, stream=None):
    """Run the symbolic phase. Returns (plan, c_rowptr int32 tensor, nnz(C))."""
    sr = SEMIRINGS[semiring]
    plan = plan or Plan()
    c_rowptr = torch.empty(A.nrows + 1, dtype=torch.int32, device=A.rowptr.device)
    nnz = ctypes.c_int64(0)
    keep = []
    da, db = A.desc(), B.desc()
    rc = _lib.load().tsspgemm_symbolic(ctypes.byref(da), ctypes.byref(db), sr, _mask_desc(mask, keep),
                                       _tuning(tuning), ctypes.c_void_p(c_rowptr.data_ptr()), ctypes.byref(nnz),
                                       ctypes.byref(plan.handle), _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_symbolic")
    plan.semiring = semiring
    plan.c_rowptr = c_rowptr
    plan.nnz = int(nnz.value)
    return plan, c_rowptr, int(nnz.value)


def numeric(plan: Plan, A: DeviceCsr, B: DeviceCsr, c_colidx: torch.Tensor, c_vals: torch.Tensor | None,
            stream=None):
    da, db = A.desc(), B.desc()
    rc = _lib.load().tsspgemm_numeric(plan.handle, ctypes.byref(da), ctypes.byref(db), _ptr(c_colidx),
                                      _ptr(c_vals), _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_numeric")


def spgemm(A: DeviceCsr, B: DeviceCsr, semiring="plus_times", mask=None, tuning: dict | None = None,
           plan: Plan | None = None, stream=None, return_plan=False):
    """C = A B (Eq. 1) over `semiring`; C is a DeviceCsr (values None for or_and)."""
    plan, c_rowptr, nnz = symbolic(A, B, semiring, mask, tuning, plan, stream)
    dev = A.rowptr.device
    c_colidx = torch.empty(nnz, dtype=torch.int32, device=dev)
    c_vals = None
    if semiring in ("plus_times", "plus_times_f32"):
        c_vals = torch.empty(nnz, dtype=torch.float32, device=dev)
    elif semiring == "plus_times_i32":
        c_vals = torch.empty(nnz, dtype=torch.int32, device=dev)
    numeric(plan, A, B, c_colidx, c_vals, stream)
    C = DeviceCsr(A.nrows, B.ncols, c_rowptr, c_colidx, c_vals)
    return (C, plan) if return_plan else C


def masked_bool(A: DeviceCsr, F: DeviceCsr, visited=None, capacity: int | None = None, stream=None) -> DeviceCsr:
    """One (AND, OR) product with complement mask (Algorithm 3's N \\ S)."""
    dev = A.rowptr.device
    c_rowptr = torch.empty(A.nrows + 1, dtype=torch.int32, device=dev)
    cap = capacity if capacity is not None else max(1, min(A.nrows * F.ncols, 1 << 26))
    keep = []
    da, df = A.desc(), F.desc()
    mdesc = _mask_desc(visited, keep)
    lib = _lib.load()
    while True:
        c_colidx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        nnz = ctypes.c_int64(0)
        rc = lib.tsspgemm_masked_bool(ctypes.byref(da), ctypes.byref(df), mdesc, ctypes.c_void_p(c_rowptr.data_ptr()),
                                      ctypes.c_void_p(c_colidx.data_ptr()), cap, ctypes.byref(nnz), _stream_ptr(stream))
        if rc == _lib.ERR_CAPACITY:
            cap = int(nnz.value)
            continue
        _lib.check(rc, "tsspgemm_masked_bool")
        return DeviceCsr(A.nrows, F.ncols, c_rowptr, c_colidx[:int(nnz.value)].contiguous())


def msbfs(A: DeviceCsr, sources: torch.Tensor, stream=None):
    """Multi-source BFS (Algorithm 3). Returns (levels n x d int32, per-iteration nnz(F))."""
    d = int(sources.numel())
    levels = torch.empty((A.nrows, d), dtype=torch.int32, device=A.rowptr.device)
    it = ctypes.c_int32(0)
    cap = 4096
    fn = (ctypes.c_int64 * cap)()
    src = sources.to(device=A.rowptr.device, dtype=torch.int32).contiguous()
    da = A.desc()
    rc = _lib.load().tsspgemm_msbfs(ctypes.byref(da), ctypes.c_void_p(src.data_ptr()), d,
                                    ctypes.c_void_p(levels.data_ptr()), ctypes.byref(it), fn, cap, _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_msbfs")
    return levels, [int(fn[t]) for t in range(min(it.value, cap))]


def transpose(A: DeviceCsr, stream=None):
    """A^T as (DeviceCsr pattern, perm) where perm maps A^T entries to A entries."""
    dev = A.rowptr.device
    at_rp = torch.empty(A.ncols + 1, dtype=torch.int32, device=dev)
    at_ci = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    da = A.desc()
    rc = _lib.load().tsspgemm_transpose(ctypes.byref(da), ctypes.c_void_p(at_rp.data_ptr()),
                                        ctypes.c_void_p(at_ci.data_ptr()), ctypes.c_void_p(perm.data_ptr()),
                                        _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_transpose")
    return DeviceCsr(A.ncols, A.nrows, at_rp, at_ci[:A.nnz]), perm[:A.nnz]


def bitmap_words(d: int) -> int:
    return int(_lib.load().tsspgemm_bitmap_words(d))


def version() -> str:
    return _lib.load().tsspgemm_version().decode()


def grad_a(plan: Plan, A: DeviceCsr, B: DeviceCsr, G: DeviceCsr, stream=None) -> torch.Tensor:
    """dL/dA on pat(A) (an SDDMM): out[p] = sum_j G(i,j) B(k,j) for the p-th entry (i,k)."""
    out = torch.empty(max(A.nnz, 1), dtype=torch.float32, device=A.rowptr.device)
    da, db, dg = A.desc(), B.desc(), G.desc()
    rc = _lib.load().tsspgemm_grad_a(plan.handle, ctypes.byref(da), ctypes.byref(db), ctypes.byref(dg),
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_grad_a")
    return out[:A.nnz]


def grad_b(plan: Plan, AT: DeviceCsr, perm: torch.Tensor, A: DeviceCsr, B: DeviceCsr, G: DeviceCsr,
           stream=None) -> torch.Tensor:
    """dL/dB on pat(B): out[q] = sum_i A(i,k) G(i,j) for the q-th entry (k,j) (A^T G sampled)."""
    out = torch.empty(max(B.nnz, 1), dtype=torch.float32, device=B.rowptr.device)
    dat, da, db, dg = AT.desc(), A.desc(), B.desc(), G.desc()
    rc = _lib.load().tsspgemm_grad_b(plan.handle, ctypes.byref(dat), _ptr(perm), ctypes.byref(da), ctypes.byref(db),
                                     ctypes.byref(dg), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_grad_b")
    return out[:B.nnz]


def backward(plan: Plan, AT: DeviceCsr | None, perm: torch.Tensor | None, A: DeviceCsr, B: DeviceCsr, G: DeviceCsr,
             need_a: bool = True, need_b: bool = True, stream=None):
    """dL/dA and dL/dB of the same product in one library call (one pass over
    A's rows for dL/dA and the sampled G, one over A^T for dL/dB). Returns
    (grad_a or None, grad_b or None)."""
    if not (need_a or need_b):
        return None, None
    dev = A.rowptr.device
    ga = torch.empty(max(A.nnz, 1), dtype=torch.float32, device=dev) if need_a else None
    gb = torch.empty(max(B.nnz, 1), dtype=torch.float32, device=dev) if need_b else None
    da, db, dg = A.desc(), B.desc(), G.desc()
    dat = AT.desc() if AT is not None else None
    rc = _lib.load().tsspgemm_backward(plan.handle, ctypes.byref(dat) if dat is not None else None,
                                       _ptr(perm) if perm is not None else None, ctypes.byref(da), ctypes.byref(db),
                                       ctypes.byref(dg), _ptr(ga) if ga is not None else None,
                                       _ptr(gb) if gb is not None else None, _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_backward")
    return (ga[:A.nnz] if need_a else None), (gb[:B.nnz] if need_b else None)


def spmm(A: DeviceCsr, B: torch.Tensor, stream=None) -> torch.Tensor:
    """C = A B with B dense (n x d float32, row-major; zeros included): the
    SpMM alternative of Sec. V-C. Returns C dense (n x d float32)."""
    if B.dim() != 2 or B.shape[0] != A.ncols:
        raise ValueError("B must be n x d")
    B = B.to(device=A.rowptr.device, dtype=torch.float32)
    if B.stride(1) != 1:
        B = B.contiguous()
    n, d = A.nrows, B.shape[1]
    C = torch.empty((n, d), dtype=torch.float32, device=A.rowptr.device)
    da = A.desc()
    rc = _lib.load().tsspgemm_spmm(ctypes.byref(da), _ptr(B), d, B.stride(0), _ptr(C), C.stride(0),
                                   _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_spmm")
    return C


def spmm_noalloc(A: DeviceCsr, B: torch.Tensor, C: torch.Tensor, stream=None) -> torch.Tensor:
    """spmm into the caller's C (n x d float32, unit column stride) through the
    library's allocation-free entry point: its workspace is a fixed per-GPU
    device array, so the call allocates nothing (for graph capture or loops
    that must not allocate). Raises TSSpGEMMError(CAPACITY) for a problem
    larger than that array."""
    if B.dim() != 2 or B.shape[0] != A.ncols or B.stride(1) != 1 or B.dtype != torch.float32:
        raise ValueError("B must be n x d float32 with unit column stride")
    if C.dim() != 2 or C.shape[0] != A.nrows or C.shape[1] != B.shape[1] or C.stride(1) != 1 or \
            C.dtype != torch.float32:
        raise ValueError("C must be n x d float32 with unit column stride")
    da = A.desc()
    rc = _lib.load().tsspgemm_spmm_noalloc(ctypes.byref(da), _ptr(B), B.shape[1], B.stride(0), _ptr(C),
                                           C.stride(0), _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_spmm_noalloc")
    return C


def column_slice(A: DeviceCsr, c0: int, c1: int, stream=None) -> DeviceCsr:
    """Column tile A(:, c0:c1) with its column ids (Sec. III-B)."""
    dev = A.rowptr.device
    rp = torch.empty(A.nrows + 1, dtype=torch.int32, device=dev)
    nnz = ctypes.c_int64(0)
    da = A.desc()
    lib = _lib.load()
    _lib.check(lib.tsspgemm_column_slice_count(ctypes.byref(da), c0, c1, _ptr(rp), ctypes.byref(nnz),
                                               _stream_ptr(stream)), "tsspgemm_column_slice_count")
    ci = torch.empty(nnz.value, dtype=torch.int32, device=dev)
    v = None if A.vals is None else torch.empty(nnz.value, dtype=torch.float32, device=dev)
    _lib.check(lib.tsspgemm_column_slice_fill(ctypes.byref(da), c0, c1, _ptr(rp), _ptr(ci) if nnz.value else None,
                                              _ptr(v) if v is not None and nnz.value else None, _stream_ptr(stream)),
               "tsspgemm_column_slice_fill")
    return DeviceCsr(A.nrows, A.ncols, rp, ci, v)


def merge_rows(parts: list, stream=None) -> DeviceCsr:
    """Sum of n x d CSR parts, row by row, parts added in order (the Merge of
    Algorithm 2)."""
    descs = (_lib.CsrDesc * len(parts))(*[p.desc() for p in parts])
    n, d = parts[0].nrows, parts[0].ncols
    dev = parts[0].rowptr.device
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    nnz = ctypes.c_int64(0)
    lib = _lib.load()
    _lib.check(lib.tsspgemm_merge_count(len(parts), descs, _ptr(rp), ctypes.byref(nnz), _stream_ptr(stream)),
               "tsspgemm_merge_count")
    ci = torch.empty(nnz.value, dtype=torch.int32, device=dev)
    v = torch.empty(nnz.value, dtype=torch.float32, device=dev)
    _lib.check(lib.tsspgemm_merge_values(len(parts), descs, _ptr(rp), _ptr(ci) if nnz.value else None,
                                         _ptr(v) if nnz.value else None, _stream_ptr(stream)),
               "tsspgemm_merge_values")
    return DeviceCsr(n, d, rp, ci, v)


def tile_edges(n: int, tiles: int) -> list:
    """Column boundaries of `tiles` near-equal column tiles of an n-column A."""
    return [(t * n) // tiles for t in range(tiles + 1)]


def tiled_spgemm(A: DeviceCsr, B: DeviceCsr, tiles: int, tuning: dict | None = None, stream=None) -> DeviceCsr:
    """C = A B computed tile by tile (Sec. III-B, Algorithm 2 on one GPU): for
    each of `tiles` column ranges of A, the product of that tile with B (it
    reads only B's rows in the range), then the merge of the partial outputs.
    Each partial value is rounded to FP32 before the merge. 1 <= tiles <= 64
    (the merge takes at most 64 parts)."""
    if not 1 <= tiles <= 64:
        raise ValueError("tiled_spgemm: tiles must be in [1, 64]")
    e = tile_edges(A.ncols, tiles)
    parts = [spgemm(column_slice(A, e[t], e[t + 1], stream), B, tuning=tuning, stream=stream) for t in range(tiles)]
    return parts[0] if tiles == 1 else merge_rows(parts, stream)


def embed_epoch(A: DeviceCsr, z_colidx: torch.Tensor, z_vals: torch.Tensor, d: int, k: int, lr: float,
                batch: int, row_begin: int = 0, row_end: int | None = None, stream=None) -> None:
    """Sparse force-directed embedding update (Sec. IV-B), in place: rows
    [row_begin, row_end) of Z (n x d, k entries per row at row * k) in
    minibatches of `batch` rows. A is the signed n x n graph (+1 neighbour,
    -1 negative sample)."""
    n = A.nrows
    for t, dt in ((z_colidx, torch.int32), (z_vals, torch.float32)):
        if t.dtype != dt or not t.is_contiguous() or t.numel() != n * k or t.device != A.rowptr.device:
            raise ValueError("z_colidx / z_vals must be contiguous int32 / float32 of n * k on A's device")
    da = A.desc()
    rc = _lib.load().tsspgemm_embed_epoch(ctypes.byref(da), d, k, _ptr(z_colidx), _ptr(z_vals), float(lr), batch,
                                          row_begin, n if row_end is None else row_end, _stream_ptr(stream))
    _lib.check(rc, "tsspgemm_embed_epoch")


class TSSpGEMMOp:
    """C = A B with fixed patterns and trainable values (the sparse layer of a
    training loop). The symbolic plan and A^T are built once; every call runs
    only the numeric phase, and backward runs dL/dA and dL/dB on the GPU."""

    def __init__(self, A: DeviceCsr, B: DeviceCsr, tuning: dict | None = None):
        self.A = A.with_vals(None)
        self.B = B.with_vals(None)
        self.plan, self.c_rowptr, self.nnz = symbolic(self.A, self.B, "plus_times", tuning=tuning)
        self.c_colidx = torch.empty(self.nnz, dtype=torch.int32, device=A.rowptr.device)
        self._at = None

    def transpose(self):
        if self._at is None:
            self._at = transpose(self.A)
        return self._at

    def c_pattern(self) -> DeviceCsr:
        return DeviceCsr(self.A.nrows, self.B.ncols, self.c_rowptr, self.c_colidx, None)

    def forward_values(self, a_vals: torch.Tensor, b_vals: torch.Tensor) -> torch.Tensor:
        c_vals = torch.empty(self.nnz, dtype=torch.float32, device=a_vals.device)
        numeric(self.plan, self.A.with_vals(a_vals.contiguous()), self.B.with_vals(b_vals.contiguous()),
                self.c_colidx, c_vals)
        return c_vals

    def __call__(self, a_vals: torch.Tensor, b_vals: torch.Tensor) -> torch.Tensor:
        return TSSpGEMMFunction.apply(a_vals, b_vals, self)


class TSSpGEMMFunction(torch.autograd.Function):
    """Autograd node of TSSpGEMMOp: values of A and B in, values of C out."""

    @staticmethod
    def forward(ctx, a_vals, b_vals, op: TSSpGEMMOp):
        ctx.save_for_backward(a_vals, b_vals)
        ctx.op = op
        return op.forward_values(a_vals, b_vals)

    @staticmethod
    def backward(ctx, g):
        a_vals, b_vals = ctx.saved_tensors
        op = ctx.op
        A = op.A.with_vals(a_vals.contiguous())
        B = op.B.with_vals(b_vals.contiguous())
        G = op.c_pattern().with_vals(g.contiguous().to(torch.float32))
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        AT, perm = op.transpose() if need_b else (None, None)
        ga, gb = backward(op.plan, AT, perm, A, B, G, need_a=need_a, need_b=need_b)
        return ga, gb, None
