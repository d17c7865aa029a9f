"""The allocation-free SpMM entry point (tsspgemm_spmm_noalloc): the same
result as tsspgemm_spmm (same kernels, same order of addition, so bit for
bit) and within the tolerance of the oracle, on two calls in a row whose
second input is smaller (the shared per-GPU workspace keeps the first call's
contents), and a clear CAPACITY error beyond the workspace's size."""
import numpy as np
import pytest
import torch

import oracle
from tests._util import random_csr
from tests.gpu_util import RTOL, note, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dense_b(rng, n, d):
    return rng.random((n, d), dtype=np.float32)


def _oracle_dense(a, bd):
    """A B with dense B through the oracle's plus-times product (B as CSR
    with every entry stored)."""
    n, d = bd.shape
    brp = (np.arange(n + 1) * d).astype(np.int32)
    bci = np.tile(np.arange(d, dtype=np.int32), n)
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, brp, bci, bd.ravel().astype(np.float64), threads=8)
    out = np.zeros((n, d))
    rows = np.repeat(np.arange(n), np.diff(rp))
    out[rows, ci] = val
    return out


def test_noalloc_matches_spmm_twice_then_smaller():
    import paper_2408_11988_amd as tss

    rng = np.random.default_rng(77)
    # first call: rows long enough to be cut into several chunks (partial rows
    # in the scratch array); second call: a smaller product on the same array
    cases = [(3000, 96, 0.02, 6), (700, 40, 0.01, 2)]
    for n, d, dens, dense_rows in cases:
        a = random_csr(rng, n, n, dens, empty_rows=0.1, dense_rows=dense_rows)
        bd = _dense_b(rng, n, d)
        A = to_dev(a)
        B = torch.from_numpy(bd).cuda()
        note(f"spmm_noalloc n={n} d={d} nnzA={a.nnz}")
        C = torch.full((n, d), float("nan"), dtype=torch.float32, device="cuda")
        tss.spmm_noalloc(A, B, C)
        ref = tss.spmm(A, B)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy()), "noalloc differs from tsspgemm_spmm"
        exact = _oracle_dense(a, bd)
        assert np.all(np.abs(got.astype(np.float64) - exact) <= RTOL * np.abs(exact))


def test_noalloc_capacity_error():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd import _lib

    # nnz(A) * d / 8 well above the 64 MiB array: rejected before any launch
    n, d = 1 << 16, 1024
    per_row = 16
    rp = torch.arange(0, (n + 1) * per_row, per_row, dtype=torch.int32, device="cuda")
    ci = (torch.arange(n * per_row, device="cuda", dtype=torch.int64) % n).to(torch.int32)
    ci = ci.view(n, per_row).sort(dim=1).values.reshape(-1).contiguous()
    A = tss.DeviceCsr(n, n, rp, ci, torch.ones(n * per_row, dtype=torch.float32, device="cuda"))
    B = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    C = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    note("spmm_noalloc beyond the scratch size")
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.spmm_noalloc(A, B, C)
    assert e.value.code == _lib.ERR_CAPACITY and "scratch" in str(e.value)
