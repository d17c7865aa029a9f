"""GPU parity of the column tiles, the merge of partial outputs and the tiled
multiply (Sec. III-B, III-C, Algorithm 2) against the oracle.

The slice copies entries and the merge adds the same FP32 values in the same
order (parts in order, FP64, rounded once) as the oracle, so both are compared
bit for bit. The tiled multiply rounds each tile's partial values to FP32
before the merge: its error is at most 2 * 2^-24 * sum |a||b| per entry, well
inside the 1e-5 tolerance of the plain multiply, and its pattern equals the
plain product's.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import random_csr
from tests.gpu_util import compare_f32, note, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_column_slice_bit_exact():
    import paper_2408_11988_amd as tss

    rng = np.random.default_rng(900)
    a = random_csr(rng, 500, 700, 0.02, kind="normal", empty_rows=0.2, dense_rows=2)
    A = to_dev(a)
    for c0, c1 in ((0, 700), (0, 1), (13, 250), (250, 250), (699, 700), (600, 2000)):
        note(f"column slice [{c0}, {c1})")
        S = tss.column_slice(A, c0, c1)
        rp, ci, val = oracle.column_slice(a.rp, a.ci, a.val, c0, c1)
        g_rp, g_ci, g_val = S.to_host()
        assert np.array_equal(g_rp.astype(np.int64), rp) and np.array_equal(g_ci, ci)
        assert np.array_equal(g_val.astype(np.float64), val)


@pytest.mark.parametrize("count,d", [(1, 64), (2, 1), (3, 31), (5, 128), (8, 1000), (64, 1024)])
def test_merge_bit_exact(count, d):
    import paper_2408_11988_amd as tss

    rng = np.random.default_rng(1000 + count * 7 + d)
    n = 300
    parts = [random_csr(rng, n, d, min(0.5, 6.0 / d + 0.02), kind="normal", empty_rows=0.3) for _ in range(count)]
    note(f"merge count={count} d={d}")
    M = tss.merge_rows([to_dev(p) for p in parts])
    rp, ci, val = oracle.merge_rows([(p.rp, p.ci, p.val) for p in parts])
    g_rp, g_ci, g_val = M.to_host()
    assert np.array_equal(g_rp.astype(np.int64), rp) and np.array_equal(g_ci, ci)
    assert np.array_equal(g_val, val.astype(np.float32))


def test_merge_errors():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd import _lib

    rng = np.random.default_rng(5)
    p = to_dev(random_csr(rng, 50, 40, 0.1))
    note("merge argument errors")
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.merge_rows([p] * 65)
    assert e.value.code == _lib.ERR_UNSUPPORTED
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.merge_rows([to_dev(random_csr(rng, 50, 1030, 0.01))])
    assert e.value.code == _lib.ERR_UNSUPPORTED
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.merge_rows([p, to_dev(random_csr(rng, 50, 41, 0.1))])
    assert e.value.code == _lib.ERR_INVALID_ARG


@pytest.mark.parametrize("tiles", [1, 2, 7, 33])
def test_tiled_spgemm_matches_oracle(tiles):
    import paper_2408_11988_amd as tss

    a, b = synth.workload_er_small()
    note(f"tiled spgemm ER 4096 x 64, {tiles} tiles")
    C = tss.tiled_spgemm(to_dev(a), to_dev(b), tiles)
    compare_f32(a, b, C)


def test_tiled_spgemm_rmat20_sampled_rows():
    """The bench configuration (R-MAT 20 x 128) in 8 column tiles: the 24
    heaviest rows and 2000 random rows against the oracle."""
    import paper_2408_11988_amd as tss

    a, b = synth.workload_rmat_plain(scale=20, d=128)
    note("tiled spgemm R-MAT 20 x 128, 8 tiles")
    C = tss.tiled_spgemm(to_dev(a), to_dev(b), 8)
    torch.cuda.synchronize()
    deg = np.diff(a.rp)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([np.argsort(deg)[-24:], rng.choice(a.nrows, 2000, replace=False)]))
    compare_f32(a, b, C, rows=rows.astype(np.int32), threads=16)
    assert C.nnz == 53141923
