"""Helpers shared by the GPU parity tests (comparison against the oracle)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

# FP32 plus-times tolerance: relative 1e-5 of the FP64 oracle value on
# non-negative data; on signed data relative to sum |a||b| of the entry's
# terms (plain relative error is undefined under cancellation).
RTOL = 1e-5


def note(msg: str):
    """Name the case on stdout (flushed) before a GPU step."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"


def to_dev(m, dtype=torch.float32, with_values=True):
    from paper_2408_11988_amd import DeviceCsr

    return DeviceCsr.from_host(m, dtype=dtype, with_values=with_values)


def abs_csr(m):
    from synth import Csr

    return Csr(m.nrows, m.ncols, m.rp, m.ci, np.abs(m.val))


def compare_f32(a, b, C, rows=None, threads=8, signed=False, ref=None):
    """Structure bit-exact, values within RTOL of the FP64 oracle. With `rows`,
    only those rows are compared (C is the full GPU result). `ref` is the
    oracle's (rp, ci, val) for all rows when already computed. Returns the
    fraction of values equal to the oracle rounded to FP32."""
    g_rp, g_ci, g_val = C.to_host()
    if ref is not None:
        assert rows is None and not signed
        rp, ci, val = ref
    else:
        rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, rows=rows, threads=threads)
    if signed:
        _, _, scale = oracle.spgemm(a.rp, a.ci, np.abs(a.val), b.rp, b.ci, np.abs(b.val), rows=rows, threads=threads)
    else:
        scale = np.abs(val)
    if rows is None:
        assert np.array_equal(g_rp.astype(np.int64), rp), "row pointers differ"
        assert np.array_equal(g_ci, ci), "column indices differ"
        gv = g_val.astype(np.float64)
    else:
        gcols, gvals = [], []
        for t, i in enumerate(rows):
            seg = slice(int(g_rp[i]), int(g_rp[i + 1]))
            assert g_rp[i + 1] - g_rp[i] == rp[t + 1] - rp[t], f"row {i}: nnz differs"
            gcols.append(g_ci[seg])
            gvals.append(g_val[seg])
        gc = np.concatenate(gcols) if gcols else np.zeros(0, np.int32)
        assert np.array_equal(gc, ci), "column indices differ on sampled rows"
        gv = (np.concatenate(gvals) if gvals else np.zeros(0, np.float32)).astype(np.float64)
    err = np.abs(gv - val)
    bad = err > RTOL * scale
    assert not bad.any(), f"{bad.sum()} values outside tolerance; worst rel {np.max(err / np.maximum(scale, 1e-300))}"
    return float(np.mean(gv == val.astype(np.float32).astype(np.float64))) if len(val) else 1.0


def same_structure_close_values(c1, c2):
    """Two GPU results of one product: identical structure, values within RTOL
    of each other (FP64 sums in another order may round to a neighbouring
    FP32 value). Returns the fraction of bit-identical values."""
    r1, i1, v1 = c1.to_host()
    r2, i2, v2 = c2.to_host()
    assert np.array_equal(r1, r2), "row pointers differ"
    assert np.array_equal(i1, i2), "column indices differ"
    x, y = v1.astype(np.float64), v2.astype(np.float64)
    assert np.all(np.abs(x - y) <= RTOL * np.maximum(np.abs(x), np.abs(y))), "values differ beyond the tolerance"
    return float(np.mean(v1 == v2)) if len(v1) else 1.0


def compare_int(a, b, C):
    g_rp, g_ci, g_val = C.to_host()
    rp, ci, val = oracle.spgemm_int(a.rp, a.ci, a.val.astype(np.int64), b.rp, b.ci, b.val.astype(np.int64))
    assert np.array_equal(g_rp.astype(np.int64), rp)
    assert np.array_equal(g_ci, ci)
    assert np.array_equal(g_val.astype(np.int64), val)


def compare_bool(a, b, C, mask=None):
    g_rp, g_ci, _ = C.to_host()
    if mask is None:
        rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci)
    else:
        rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci, mask.rp, mask.ci)
    assert np.array_equal(g_rp.astype(np.int64), rp)
    assert np.array_equal(g_ci, ci)
