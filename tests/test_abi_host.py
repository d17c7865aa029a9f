"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/tsspgemm.h, and rejects bad arguments with error codes
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsspgemm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsspgemm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2408_11988_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2408_11988_amd import build

        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2408_11988_amd import _lib

    assert set(names) == set(_lib.EXPORTED)


def test_bitmap_words(lib):
    assert [lib.tsspgemm_bitmap_words(d) for d in (0, 1, 32, 33, 64, 65, 96, 128, 200, 512, 1024)] == \
        [1, 1, 1, 2, 2, 4, 4, 4, 8, 16, 32]


def test_version(lib):
    assert lib.tsspgemm_version().startswith(b"tsspgemm")


def _desc(nrows, ncols, nnz, ptr=0x1000):
    from paper_2408_11988_amd import _lib

    return _lib.CsrDesc(nrows, ncols, nnz, ptr, ptr, ptr)


def _symbolic(lib, A, B, sr=0, rowptr=0x1000, tune=None):
    plan = ctypes.c_void_p(None)
    nnz = ctypes.c_int64(-1)
    rc = lib.tsspgemm_symbolic(ctypes.byref(A) if A is not None else None, ctypes.byref(B) if B is not None else None,
                               sr, None, ctypes.byref(tune) if tune is not None else None, rowptr, ctypes.byref(nnz),
                               ctypes.byref(plan), None)
    return rc, plan


def test_argument_errors_without_device(lib):
    from paper_2408_11988_amd import _lib

    rc, plan = _symbolic(lib, None, _desc(4, 2, 0))
    assert rc == _lib.ERR_INVALID_ARG and not plan.value
    assert b"NULL" in lib.tsspgemm_last_error()
    rc, _ = _symbolic(lib, _desc(4, 5, 0), _desc(5, 2, 0))  # A not square
    assert rc == _lib.ERR_INVALID_ARG and b"square" in lib.tsspgemm_last_error()
    rc, _ = _symbolic(lib, _desc(4, 4, 0), _desc(5, 2, 0))  # inner dimensions differ
    assert rc == _lib.ERR_INVALID_ARG
    rc, _ = _symbolic(lib, _desc(4, 4, 0), _desc(4, 2, 0), sr=7)
    assert rc == _lib.ERR_INVALID_ARG
    rc, _ = _symbolic(lib, _desc(4, 4, 0), _desc(4, 2, 0), rowptr=None)
    assert rc == _lib.ERR_INVALID_ARG
    rc, _ = _symbolic(lib, _desc(-1, -1, 0), _desc(4, 2, 0))
    assert rc == _lib.ERR_INVALID_ARG
    rc, _ = _symbolic(lib, _desc(4, 4, 1 << 40), _desc(4, 2, 0))
    assert rc == _lib.ERR_OVERFLOW
    rc, plan = _symbolic(lib, _desc(4, 4, 0), _desc(4, 2, 0), tune=_lib.Tuning(0, 0, 0, 0, 9, 0, 0))
    assert rc == _lib.ERR_INVALID_ARG and b"accumulator" in lib.tsspgemm_last_error() and not plan.value
    rc, _ = _symbolic(lib, _desc(4, 4, 0), _desc(4, 2048, 0), tune=_lib.Tuning(0, 0, 0, 0, 1, 0, 0))
    assert rc == _lib.ERR_UNSUPPORTED  # the LDS strip needs d <= 1024
    bad = _lib.CsrDesc(4, 4, 3, 0x1000, None, 0x1000)  # nnz > 0 but no column array
    rc, _ = _symbolic(lib, bad, _desc(4, 2, 0))
    assert rc == _lib.ERR_INVALID_ARG
    # numeric without a plan
    a, b = _desc(4, 4, 0), _desc(4, 2, 0)
    assert lib.tsspgemm_numeric(None, ctypes.byref(a), ctypes.byref(b), None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.tsspgemm_plan_stats(None, None, None, None, None, None, None) == _lib.ERR_INVALID_ARG
    lib.tsspgemm_plan_destroy(None)  # no-op


def test_python_errors_are_raised():
    from paper_2408_11988_amd import _lib

    with pytest.raises(_lib.TSSpGEMMError) as e:
        _lib.check(_lib.ERR_UNSUPPORTED, "where")
    assert e.value.code == _lib.ERR_UNSUPPORTED and "UNSUPPORTED" in str(e.value)


def test_argument_errors_of_the_extra_entry_points(lib):
    """SpMM, the embedding epoch, column tiles and the merge reject bad
    arguments on the host, before any device work."""
    from paper_2408_11988_amd import _lib

    p = ctypes.c_void_p(0x1000)
    a = _desc(4, 4, 2)
    rect = _desc(4, 5, 2)
    # spmm
    assert lib.tsspgemm_spmm(ctypes.byref(rect), p, 8, 8, p, 8, None) == _lib.ERR_INVALID_ARG
    assert lib.tsspgemm_spmm(ctypes.byref(a), p, 8, 4, p, 8, None) == _lib.ERR_INVALID_ARG  # ldb < d
    assert lib.tsspgemm_spmm(ctypes.byref(a), p, 2000, 2000, p, 2000, None) == _lib.ERR_UNSUPPORTED
    # embedding epoch
    emb = lambda d, k, b, r0, r1: lib.tsspgemm_embed_epoch(ctypes.byref(a), d, k, p, p, 0.1, b, r0, r1, None)
    assert emb(8, 9, 4, 0, 4) == _lib.ERR_INVALID_ARG    # k > d
    assert emb(8, 0, 4, 0, 4) == _lib.ERR_INVALID_ARG    # k < 1
    assert emb(8, 4, 0, 0, 4) == _lib.ERR_INVALID_ARG    # batch < 1
    assert emb(8, 4, 2, 3, 2) == _lib.ERR_INVALID_ARG    # row_begin > row_end
    assert emb(8, 4, 2, 0, 5) == _lib.ERR_INVALID_ARG    # row_end > n
    assert emb(2048, 4, 2, 0, 4) == _lib.ERR_UNSUPPORTED  # d > 1024
    assert emb(8, 4, 2, 2, 2) == _lib.OK                 # empty range: nothing to do
    assert lib.tsspgemm_embed_epoch(ctypes.byref(rect), 8, 4, p, p, 0.1, 2, 0, 4, None) == _lib.ERR_INVALID_ARG
    # column tiles
    nnz = ctypes.c_int64(0)
    assert lib.tsspgemm_column_slice_count(ctypes.byref(a), 3, 2, p, ctypes.byref(nnz), None) == _lib.ERR_INVALID_ARG
    assert lib.tsspgemm_column_slice_count(ctypes.byref(a), 0, 2, None, ctypes.byref(nnz), None) == _lib.ERR_INVALID_ARG
    assert lib.tsspgemm_column_slice_fill(ctypes.byref(a), -1, 2, p, p, p, None) == _lib.ERR_INVALID_ARG
    # merge
    two = (_lib.CsrDesc * 2)(_desc(4, 8, 2), _desc(4, 9, 2))
    assert lib.tsspgemm_merge_count(0, two, p, ctypes.byref(nnz), None) == _lib.ERR_INVALID_ARG
    assert lib.tsspgemm_merge_count(65, two, p, ctypes.byref(nnz), None) == _lib.ERR_UNSUPPORTED
    assert lib.tsspgemm_merge_count(2, two, p, ctypes.byref(nnz), None) == _lib.ERR_INVALID_ARG  # shapes differ
    wide = (_lib.CsrDesc * 1)(_desc(4, 2048, 2))
    assert lib.tsspgemm_merge_values(1, wide, p, p, p, None) == _lib.ERR_UNSUPPORTED
    # batched plan: an instance with d > 1024 (the batch has no hash accumulator)
    batch = ctypes.c_void_p(None)
    pool, rps = ctypes.c_int64(0), ctypes.c_int64(0)
    As = (_lib.CsrDesc * 2)(_desc(4, 4, 2), _desc(4, 4, 2))
    Bs = (_lib.CsrDesc * 2)(_desc(4, 64, 2), _desc(4, 2048, 2))
    rc = lib.tsspgemm_batched_plan(2, As, Bs, None, ctypes.byref(batch), ctypes.byref(pool), ctypes.byref(rps), None)
    assert rc == _lib.ERR_UNSUPPORTED and b"d > 1024" in lib.tsspgemm_last_error() and not batch.value
    Bs = (_lib.CsrDesc * 2)(_desc(4, 64, 2), _desc(5, 64, 2))  # B's rows differ from A's columns
    rc = lib.tsspgemm_batched_plan(2, As, Bs, None, ctypes.byref(batch), ctypes.byref(pool), ctypes.byref(rps), None)
    assert rc == _lib.ERR_INVALID_ARG and not batch.value


def test_tiled_spgemm_rejects_tile_counts_outside_the_merge_limit():
    import paper_2408_11988_amd as tss

    for tiles in (0, 65):
        with pytest.raises(ValueError):
            tss.tiled_spgemm(None, None, tiles)
