"""Pins of the column-tile and merge oracles (Sec. III-B / III-C, Algorithm 2),
CPU only: dense brute force for the slice and the merge, the union of the
parts' patterns for the merged structure, exact dyadic sums, and the tiling
identity sum_t A(:, tile t) B = A B."""
import numpy as np
import pytest

import oracle
from tests._util import dense, random_csr, rows_of


def _dense_of(rp, ci, val, n, m):
    out = np.zeros((n, m))
    out[rows_of(rp), ci] = val
    return out


def slice_matches_dense(seed=0):
    rng = np.random.default_rng(seed)
    ok = True
    for c0, c1 in ((0, 40), (5, 17), (17, 17), (0, 1), (39, 40), (30, 45)):
        a = random_csr(rng, 35, 40, 0.25, empty_rows=0.2)
        rp, ci, val = oracle.column_slice(a.rp, a.ci, a.val, c0, c1)
        want = dense(a).copy()
        want[:, :max(c0, 0)] = 0
        want[:, min(c1, 40):] = 0
        mask = np.zeros(40, bool)
        mask[max(c0, 0):min(c1, 40)] = True
        ok &= bool(np.array_equal(_dense_of(rp, ci, val, 35, 40), want))
        ok &= int(rp[-1]) == int(mask[a.ci].sum())  # every entry in range, explicit zeros included
    return ok


def merge_matches_dense(seed=1):
    rng = np.random.default_rng(seed)
    ok = True
    for count in (1, 2, 5):
        n, d = 25, 12
        parts = [random_csr(rng, n, d, 0.3, kind="normal", empty_rows=0.3) for _ in range(count)]
        rp, ci, val = oracle.merge_rows([(p.rp, p.ci, p.val) for p in parts])
        ok &= bool(np.allclose(_dense_of(rp, ci, val, n, d), sum(dense(p) for p in parts), rtol=1e-14, atol=1e-14))
        union = np.zeros((n, d), bool)
        for p in parts:
            union[rows_of(p.rp), p.ci] = True
        got = np.zeros((n, d), bool)
        got[rows_of(rp), ci] = True
        ok &= bool(np.array_equal(got, union)) and bool(np.all(np.diff(ci)[np.diff(rows_of(rp)) == 0] > 0))
    return ok


def test_column_slice_matches_dense():
    assert slice_matches_dense()


def test_merge_matches_dense_sum_and_union_pattern():
    assert merge_matches_dense()


def test_merge_is_exact_on_a_dyadic_grid():
    rng = np.random.default_rng(2)
    n, d = 30, 16
    parts = []
    for _ in range(4):
        p = random_csr(rng, n, d, 0.35)
        p.val = (rng.integers(-64, 65, p.nnz) / 8.0).astype(np.float32)
        parts.append(p)
    rp, ci, val = oracle.merge_rows([(p.rp, p.ci, p.val) for p in parts])
    assert np.array_equal(_dense_of(rp, ci, val, n, d), sum(dense(p) for p in parts))


def test_tiling_identity():
    """sum over column tiles of A(:, tile) B, merged, equals A B (Algorithm 2's
    tile-by-tile computation followed by Merge)."""
    rng = np.random.default_rng(3)
    n, d = 60, 20
    a = random_csr(rng, n, n, 0.12, kind="normal")
    b = random_csr(rng, n, d, 0.3, kind="normal")
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    for tiles in (1, 2, 7, n):
        edges = np.linspace(0, n, tiles + 1).astype(int)
        parts = []
        for t in range(tiles):
            srp, sci, sval = oracle.column_slice(a.rp, a.ci, a.val, int(edges[t]), int(edges[t + 1]))
            parts.append(oracle.spgemm(srp.astype(np.int32), sci, sval, b.rp, b.ci, b.val))
        mrp, mci, mval = oracle.merge_rows(parts)
        assert np.array_equal(mrp, rp) and np.array_equal(mci, ci)
        assert np.allclose(mval, val, rtol=1e-12, atol=1e-12)


def test_merge_needs_a_part():
    with pytest.raises(ValueError):
        oracle.merge_rows([])
