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
