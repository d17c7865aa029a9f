"""CPU oracle for TS-SpGEMM -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference implementations (``oracle.cpp``,
ordered-map Gustavson in FP64, ordered-set boolean products, Algorithm 3 BFS,
queue BFS, FP64 gradients). Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. It imports
nothing from the GPU library and the GPU library imports nothing from it.

Every function takes host numpy arrays (CSR: int32 row pointers and column
indices; values converted to float64 or int64 here) and returns numpy arrays.
Section / equation / algorithm citations refer to the paper "Distributed-Memory
Parallel Algorithms for Sparse Matrix and Sparse Tall-and-Skinny Matrix
Multiplication" (SC'24).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so with g++ (no GPU code involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", tmp, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _configure(path: str):
    """Open the shared library at `path` and declare its C signatures."""
    lib = ctypes.CDLL(path)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.oracle_row_flops.restype = None
    lib.oracle_row_flops.argtypes = [i64, vp, vp, vp, vp]
    for name in ("oracle_spgemm_f64", "oracle_spgemm_i64"):
        f = getattr(lib, name)
        f.restype = vp
        f.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, i64, ctypes.c_int]
    lib.oracle_spgemm_bool.restype = vp
    lib.oracle_spgemm_bool.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, i64, ctypes.c_int]
    lib.oracle_res_rows.restype = i64
    lib.oracle_res_rows.argtypes = [vp]
    lib.oracle_res_nnz.restype = i64
    lib.oracle_res_nnz.argtypes = [vp]
    lib.oracle_res_copy.restype = None
    lib.oracle_res_copy.argtypes = [vp, vp, vp, vp]
    lib.oracle_res_free.restype = None
    lib.oracle_res_free.argtypes = [vp]
    lib.oracle_transpose.restype = None
    lib.oracle_transpose.argtypes = [i64, i64, vp, vp, vp, vp, vp]
    lib.oracle_msbfs.restype = i32
    lib.oracle_msbfs.argtypes = [i64, vp, vp, vp, i32, vp, vp, vp]
    lib.oracle_bfs_queue.restype = None
    lib.oracle_bfs_queue.argtypes = [i64, vp, vp, vp, i32, vp, ctypes.c_int]
    lib.oracle_grad_a.restype = ctypes.c_int
    lib.oracle_grad_a.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_grad_b.restype = ctypes.c_int
    lib.oracle_grad_b.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_grad_a_rows.restype = ctypes.c_int
    lib.oracle_grad_a_rows.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    lib.oracle_grad_b_rows.restype = ctypes.c_int
    lib.oracle_grad_b_rows.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    lib.oracle_column_slice.restype = i64
    lib.oracle_column_slice.argtypes = [i64, vp, vp, vp, i32, i32, vp, vp, vp]
    lib.oracle_merge_rows.restype = vp
    lib.oracle_merge_rows.argtypes = [i64, i32, vp, vp, vp]
    lib.oracle_embed_force.restype = None
    lib.oracle_embed_force.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, vp]
    lib.oracle_embed_select.restype = None
    lib.oracle_embed_select.argtypes = [i64, i64, vp, vp, ctypes.c_double, vp, vp]
    lib.oracle_embed_epoch.restype = ctypes.c_int
    lib.oracle_embed_epoch.argtypes = [i64, vp, vp, vp, i64, i64, vp, vp, ctypes.c_double, i64, i64, i64]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _configure(_LIB)
    return _lib


def use_library(path: str | None):
    """Point this module at another build of oracle.cpp (used by the tests that
    plant mistakes in a copy of the source); None restores the default."""
    global _lib
    _lib = None if path is None else _configure(path)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return None if x is None else x.ctypes.data


def _rows_arg(rows):
    if rows is None:
        return None, 0
    r = _i32(rows)
    return r, len(r)


def _take(h, with_val: bool):
    lib = _load()
    nr = lib.oracle_res_rows(h)
    nnz = lib.oracle_res_nnz(h)
    rp = np.empty(nr + 1, dtype=np.int64)
    ci = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64) if with_val else None
    lib.oracle_res_copy(h, rp.ctypes.data, ci.ctypes.data, _ptr(val))
    lib.oracle_res_free(h)
    return rp, ci, val


def row_flops(arp, aci, brp) -> np.ndarray:
    """Multiplications per output row (Sec. II-A definition of flops)."""
    arp, aci, brp = _i32(arp), _i32(aci), _i32(brp)
    n = len(arp) - 1
    out = np.empty(n, dtype=np.int64)
    _load().oracle_row_flops(n, arp.ctypes.data, aci.ctypes.data, brp.ctypes.data, out.ctypes.data)
    return out


def spgemm(arp, aci, aval, brp, bci, bval, rows=None, threads: int = 1):
    """Plus-times C = A B in FP64 (Eq. 1). Returns (rp int64, ci int32, val f64)
    for all rows, or for the listed `rows` (rp then indexes that list)."""
    arp, aci, brp, bci = _i32(arp), _i32(aci), _i32(brp), _i32(bci)
    aval, bval = _f64(aval), _f64(bval)
    r, nsel = _rows_arg(rows)
    h = _load().oracle_spgemm_f64(len(arp) - 1, arp.ctypes.data, aci.ctypes.data, aval.ctypes.data, brp.ctypes.data,
                                  bci.ctypes.data, bval.ctypes.data, _ptr(r), nsel, threads)
    return _take(h, True)


def spgemm_int(arp, aci, aval, brp, bci, bval, rows=None, threads: int = 1):
    """Plus-times over integers (int64 accumulation); values returned as int64.
    Raises if any entry does not fit int32 (inputs must keep sums small)."""
    arp, aci, brp, bci = _i32(arp), _i32(aci), _i32(brp), _i32(bci)
    av = np.ascontiguousarray(aval, dtype=np.int64)
    bv = np.ascontiguousarray(bval, dtype=np.int64)
    r, nsel = _rows_arg(rows)
    h = _load().oracle_spgemm_i64(len(arp) - 1, arp.ctypes.data, aci.ctypes.data, av.ctypes.data, brp.ctypes.data,
                                  bci.ctypes.data, bv.ctypes.data, _ptr(r), nsel, threads)
    rp, ci, val = _take(h, True)
    vi = val.astype(np.int64)
    if len(vi) and (vi.max() > 2**31 - 1 or vi.min() < -(2**31)):
        raise OverflowError("integer product does not fit int32")
    return rp, ci, vi


def spgemm_bool(arp, aci, brp, bci, mask_rp=None, mask_ci=None, rows=None, threads: int = 1):
    """(AND, OR) product pattern, minus the complement mask when given."""
    arp, aci, brp, bci = _i32(arp), _i32(aci), _i32(brp), _i32(bci)
    mrp = None if mask_rp is None else _i32(mask_rp)
    mci = None if mask_ci is None else _i32(mask_ci)
    r, nsel = _rows_arg(rows)
    h = _load().oracle_spgemm_bool(len(arp) - 1, arp.ctypes.data, aci.ctypes.data, brp.ctypes.data, bci.ctypes.data,
                                   _ptr(mrp), _ptr(mci), _ptr(r), nsel, threads)
    rp, ci, _ = _take(h, False)
    return rp, ci


def transpose(arp, aci, ncols: int):
    """CSR transpose by a row-order walk. Returns (trp, tci, perm)."""
    arp, aci = _i32(arp), _i32(aci)
    n = len(arp) - 1
    trp = np.empty(ncols + 1, dtype=np.int32)
    tci = np.empty(len(aci), dtype=np.int32)
    perm = np.empty(len(aci), dtype=np.int32)
    _load().oracle_transpose(n, ncols, arp.ctypes.data, aci.ctypes.data, trp.ctypes.data, tci.ctypes.data,
                             perm.ctypes.data)
    return trp, tci, perm


def msbfs(arp, aci, sources, return_flops: bool = False):
    """Algorithm 3 with ordered sets. Returns (levels n x d int32, per-iteration
    nnz(F)), and with `return_flops` also the multiplications of each
    iteration's product A F (Sec. II-A flops)."""
    arp, aci, src = _i32(arp), _i32(aci), _i32(sources)
    n, d = len(arp) - 1, len(src)
    lev = np.empty((n, d), dtype=np.int32)
    fn = np.zeros(4096, dtype=np.int64)
    fl = np.zeros(4096, dtype=np.int64)
    it = _load().oracle_msbfs(n, arp.ctypes.data, aci.ctypes.data, src.ctypes.data, d, lev.ctypes.data,
                              fn.ctypes.data, fl.ctypes.data)
    return (lev, fn[:it], fl[:it]) if return_flops else (lev, fn[:it])


def bfs_queue(arp, aci, sources, threads: int = 1):
    """One plain queue BFS per source (independent check of Algorithm 3)."""
    arp, aci, src = _i32(arp), _i32(aci), _i32(sources)
    n, d = len(arp) - 1, len(src)
    lev = np.empty((n, d), dtype=np.int32)
    _load().oracle_bfs_queue(n, arp.ctypes.data, aci.ctypes.data, src.ctypes.data, d, lev.ctypes.data, threads)
    return lev


def grad_a(arp, aci, brp, bci, bval, crp, cci, g):
    """dL/dA on pat(A) for L = sum(C o W), G = W on pat(C)."""
    arp, aci, brp, bci, crp, cci = map(_i32, (arp, aci, brp, bci, crp, cci))
    bval, g = _f64(bval), _f64(g)
    out = np.empty(len(aci), dtype=np.float64)
    rc = _load().oracle_grad_a(len(arp) - 1, arp.ctypes.data, aci.ctypes.data, brp.ctypes.data, bci.ctypes.data,
                               bval.ctypes.data, crp.ctypes.data, cci.ctypes.data, g.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError("G is missing an entry of pat(C) needed by dL/dA")
    return out


def grad_b(arp, aci, aval, brp, bci, crp, cci, g):
    """dL/dB on pat(B) for L = sum(C o W), G = W on pat(C)."""
    arp, aci, brp, bci, crp, cci = map(_i32, (arp, aci, brp, bci, crp, cci))
    aval, g = _f64(aval), _f64(g)
    out = np.empty(len(bci), dtype=np.float64)
    rc = _load().oracle_grad_b(len(arp) - 1, arp.ctypes.data, aci.ctypes.data, aval.ctypes.data, brp.ctypes.data,
                               bci.ctypes.data, crp.ctypes.data, cci.ctypes.data, g.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError("G is missing an entry of pat(C) needed by dL/dB")
    return out


def grad_a_rows(arp, aci, brp, bci, bval, crp, cci, g, rows):
    """dL/dA restricted to the A entries of the listed rows (concatenated)."""
    arp, aci, brp, bci, crp, cci, rows = map(_i32, (arp, aci, brp, bci, crp, cci, rows))
    bval, g = _f64(bval), _f64(g)
    out = np.empty(int(sum(int(arp[i + 1]) - int(arp[i]) for i in rows)), dtype=np.float64)
    rc = _load().oracle_grad_a_rows(arp.ctypes.data, aci.ctypes.data, brp.ctypes.data, bci.ctypes.data,
                                    bval.ctypes.data, crp.ctypes.data, cci.ctypes.data, g.ctypes.data,
                                    rows.ctypes.data, len(rows), out.ctypes.data)
    if rc:
        raise ValueError("G is missing an entry of pat(C) needed by dL/dA")
    return out


def grad_b_rows(arp, aci, aval, brp, bci, crp, cci, g, krows):
    """dL/dB restricted to the B entries of the listed rows (concatenated)."""
    arp, aci, brp, bci, crp, cci, krows = map(_i32, (arp, aci, brp, bci, crp, cci, krows))
    aval, g = _f64(aval), _f64(g)
    out = np.empty(int(sum(int(brp[k + 1]) - int(brp[k]) for k in krows)), dtype=np.float64)
    rc = _load().oracle_grad_b_rows(len(arp) - 1, arp.ctypes.data, aci.ctypes.data, aval.ctypes.data,
                                    brp.ctypes.data, bci.ctypes.data, crp.ctypes.data, cci.ctypes.data,
                                    g.ctypes.data, krows.ctypes.data, len(krows), out.ctypes.data)
    if rc:
        raise ValueError("G is missing an entry of pat(C) needed by dL/dB")
    return out


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def embed_force(arp, aci, aval, zci, zval, d: int, k: int, i: int) -> np.ndarray:
    """F_i of the sparse embedding update (Sec. IV-B): sum over the signed
    graph's row i of w(a, z_i . z_j) z_j, w = 1 - sig (a > 0), -sig (a < 0)."""
    arp, aci, zci = _i32(arp), _i32(aci), _i32(zci)
    aval, zval = _f32(aval), _f32(zval)
    F = np.empty(d, dtype=np.float64)
    _load().oracle_embed_force(arp.ctypes.data, aci.ctypes.data, aval.ctypes.data, d, k, zci.ctypes.data,
                               zval.ctypes.data, i, F.ctypes.data)
    return F


def embed_select(zi_dense, F, lr: float, k: int):
    """u = z_i + lr F rounded to FP32; the k largest |u| (ties: lower column),
    sorted by column. Returns (columns int32, values float32)."""
    zi, F = _f64(zi_dense), _f64(F)
    ci = np.empty(k, dtype=np.int32)
    val = np.empty(k, dtype=np.float32)
    _load().oracle_embed_select(len(zi), k, zi.ctypes.data, F.ctypes.data, float(lr), ci.ctypes.data,
                                val.ctypes.data)
    return ci, val


def embed_epoch(arp, aci, aval, zci, zval, d: int, k: int, lr: float, batch: int, row_begin: int = 0,
                row_end: int | None = None):
    """Rows [row_begin, row_end) of the embedding updated in minibatches of
    `batch` rows (Sec. IV-B). Returns new (zci, zval); the inputs are not
    modified. lr is used as given (pass the FP32 value the GPU sees)."""
    arp, aci = _i32(arp), _i32(aci)
    aval = _f32(aval)
    n = len(arp) - 1
    zci, zval = _i32(zci).copy(), _f32(zval).copy()
    rc = _load().oracle_embed_epoch(n, arp.ctypes.data, aci.ctypes.data, aval.ctypes.data, d, k, zci.ctypes.data,
                                    zval.ctypes.data, float(lr), batch, row_begin, n if row_end is None else row_end)
    if rc:
        raise ValueError("embed_epoch: bad k, batch or row range")
    return zci, zval


def column_slice(arp, aci, aval, c0: int, c1: int):
    """Columns [c0, c1) of A with their column ids (a column tile, Sec. III-B).
    Returns (rp int64, ci int32, val float64 or None)."""
    arp, aci = _i32(arp), _i32(aci)
    av = None if aval is None else _f64(aval)
    n = len(arp) - 1
    rp = np.empty(n + 1, dtype=np.int64)
    nnz = _load().oracle_column_slice(n, arp.ctypes.data, aci.ctypes.data, _ptr(av), c0, c1, rp.ctypes.data,
                                      None, None)
    ci = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    _load().oracle_column_slice(n, arp.ctypes.data, aci.ctypes.data, _ptr(av), c0, c1, rp.ctypes.data,
                                ci.ctypes.data, val.ctypes.data)
    return rp, ci, (val if av is not None else None)


def merge_rows(parts):
    """Sum of n-row CSR matrices given as [(rp, ci, val), ...], row by row, the
    parts added in order in FP64 (the Merge of Algorithm 2).
    Returns (rp int64, ci int32, val float64)."""
    if not parts:
        raise ValueError("merge_rows needs at least one part")
    keep = [(_i32(rp), _i32(ci), _f64(v)) for rp, ci, v in parts]
    n = len(keep[0][0]) - 1
    arr = lambda xs: (ctypes.c_void_p * len(xs))(*[x.ctypes.data for x in xs])
    h = _load().oracle_merge_rows(n, len(keep), arr([k[0] for k in keep]), arr([k[1] for k in keep]),
                                  arr([k[2] for k in keep]))
    return _take(h, True)
