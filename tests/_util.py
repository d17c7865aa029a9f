"""Small test-only helpers: random tiny CSR inputs and dense views."""
from __future__ import annotations

import numpy as np

from synth import Csr


def random_csr(rng: np.random.Generator, nrows: int, ncols: int, density: float, kind: str = "uniform",
               empty_rows: float = 0.0, dense_rows: int = 0) -> Csr:
    """Tiny random CSR with sorted unique columns (test inputs only)."""
    pat = rng.random((nrows, ncols)) < density
    if empty_rows > 0:
        pat[rng.random(nrows) < empty_rows, :] = False
    for r in rng.choice(nrows, size=min(dense_rows, nrows), replace=False) if dense_rows else []:
        pat[r, :] = True
    rp = np.zeros(nrows + 1, dtype=np.int32)
    rp[1:] = np.cumsum(pat.sum(axis=1))
    ci = np.nonzero(pat)[1].astype(np.int32)
    nnz = int(rp[-1])
    if kind == "uniform":
        val = ((rng.integers(0, 2**24, size=nnz) + 1) * 2.0**-24).astype(np.float32)
    elif kind == "normal":
        val = rng.standard_normal(nnz).astype(np.float32)
    elif kind == "int":
        val = rng.integers(-8, 9, size=nnz).astype(np.float32)
    else:
        raise ValueError(kind)
    return Csr(nrows, ncols, rp, ci, val)


def dense(m: Csr, dtype=np.float64) -> np.ndarray:
    out = np.zeros((m.nrows, m.ncols), dtype=dtype)
    rows = np.repeat(np.arange(m.nrows), np.diff(m.rp))
    if m.val is None:
        out[rows, m.ci] = 1
    else:
        out[rows, m.ci] = m.val.astype(dtype)
    return out


def pattern(m: Csr) -> np.ndarray:
    out = np.zeros((m.nrows, m.ncols), dtype=np.int64)
    rows = np.repeat(np.arange(m.nrows), np.diff(m.rp))
    out[rows, m.ci] = 1
    return out


def csr_from_dense_pattern(pat: np.ndarray, vals: np.ndarray | None = None) -> Csr:
    nrows, ncols = pat.shape
    rp = np.zeros(nrows + 1, dtype=np.int32)
    rp[1:] = np.cumsum((pat != 0).sum(axis=1))
    r, c = np.nonzero(pat)
    val = None if vals is None else vals[r, c].astype(np.float32)
    return Csr(nrows, ncols, rp, c.astype(np.int32), val)


def rows_of(rp: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))
