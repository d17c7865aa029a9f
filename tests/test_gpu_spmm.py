"""GPU parity of the dense-B SpMM (C = A B, B and C dense) against the oracle.

The oracle multiplies by B given as a CSR matrix that stores every entry of
B, zeros included, so its output rows are dense where A's row has an entry.
Values: |gpu - oracle| <= 1e-5 * sum |a| |b| (signed inputs); rows of A
without entries must be exactly 0.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import random_csr
from tests.gpu_util import RTOL, note, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dense_as_csr(b):
    n, d = b.shape
    rp = (np.arange(n + 1, dtype=np.int64) * d).astype(np.int32)
    ci = np.tile(np.arange(d, dtype=np.int32), n)
    return rp, ci, b.ravel().astype(np.float32)


def _check(a, b, C):
    n, d = b.shape
    brp, bci, bval = _dense_as_csr(b)
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, brp, bci, bval, threads=8)
    _, _, scale = oracle.spgemm(a.rp, a.ci, np.abs(a.val), brp, bci, np.abs(bval), threads=8)
    ref = np.zeros((n, d))
    sc = np.zeros((n, d))
    rows = np.repeat(np.arange(n), np.diff(rp))
    ref[rows, ci] = val
    sc[rows, ci] = scale
    got = C.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    assert np.all(err <= RTOL * sc), f"worst {np.max(err / np.maximum(sc, 1e-300))}"
    empty = np.diff(a.rp) == 0
    assert np.all(got[empty] == 0.0)


@pytest.mark.parametrize("d", [1, 3, 4, 64, 128, 130, 256, 1000, 1024])
def test_spmm_random(d):
    import paper_2408_11988_amd as tss

    rng = np.random.default_rng(5000 + d)
    n = 700
    a = random_csr(rng, n, n, 0.01, kind="normal", empty_rows=0.2, dense_rows=2)  # dense rows: > 512 entries
    b = rng.standard_normal((n, d)).astype(np.float32)
    b[rng.random((n, d)) < 0.5] = 0.0
    note(f"spmm n={n} d={d} nnzA={a.nnz} longest row={np.diff(a.rp).max()}")
    C = tss.spmm(to_dev(a), torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    _check(a, b, C)


def test_spmm_strided_and_edge_cases():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd import _lib

    rng = np.random.default_rng(77)
    n, d = 300, 96
    a = random_csr(rng, n, n, 0.05, dense_rows=1)
    wide = rng.random((n, d + 8)).astype(np.float32)
    Bw = torch.from_numpy(wide).cuda()
    note("spmm with ldb > d (16-byte lane path)")
    C = tss.spmm(to_dev(a), Bw[:, :d])
    _check(a, wide[:, :d].copy(), C)
    note("spmm with a column offset of 2 (8-byte lane path)")
    C = tss.spmm(to_dev(a), Bw[:, 2:d + 2])
    _check(a, wide[:, 2:d + 2].copy(), C)
    note("spmm with an odd column offset (scalar path)")
    C = tss.spmm(to_dev(a), Bw[:, 1:d + 1])
    _check(a, wide[:, 1:d + 1].copy(), C)
    note("spmm, A without entries")
    ea = synth.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    C = tss.spmm(to_dev(ea), Bw[:, :d])
    assert torch.count_nonzero(C).item() == 0
    note("spmm, d > 1024")
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.spmm(to_dev(a), torch.zeros((n, 1040), device="cuda"))
    assert e.value.code == _lib.ERR_UNSUPPORTED


def test_spmm_rmat16_equals_spgemm_on_dense_b():
    """R-MAT 16 x 128: the SpMM result equals the TS-SpGEMM result for the
    same B stored sparse (where B has entries; 0 elsewhere)."""
    import paper_2408_11988_amd as tss

    a, b = synth.workload_rmat_plain(scale=16, d=128)
    A, Bs = to_dev(a), to_dev(b)
    dense = np.zeros((b.nrows, b.ncols), np.float32)
    dense[np.repeat(np.arange(b.nrows), np.diff(b.rp)), b.ci] = b.val
    note(f"R-MAT 16 spmm vs spgemm nnzA={a.nnz}")
    C = tss.spmm(A, torch.from_numpy(dense).cuda())
    S = tss.spgemm(A, Bs)
    rp, ci, val = S.to_host()
    ref = np.zeros_like(dense)
    ref[np.repeat(np.arange(a.nrows), np.diff(rp)), ci] = val
    got = C.cpu().numpy()
    rel = np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), 1e-30)
    assert np.all((ref == 0) == (got == 0)) and rel.max() <= 2 * RTOL


def test_spmm_on_two_streams():
    """Calls on two streams share the device's workspace; the library orders
    them on the device, so every result still matches the oracle."""
    import paper_2408_11988_amd as tss

    rng = np.random.default_rng(77)
    probs = []
    for n, d in ((3000, 96), (2500, 130)):
        a = random_csr(rng, n, n, 0.004, kind="normal", empty_rows=0.1, dense_rows=3)
        b = rng.standard_normal((n, d)).astype(np.float32)
        probs.append((a, b, to_dev(a), torch.from_numpy(b).cuda()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    note("spmm on two streams, 4 rounds")
    outs = [[], []]
    for _ in range(4):
        for t, (s, (_, _, A, B)) in enumerate(zip(streams, probs)):
            with torch.cuda.stream(s):
                outs[t].append(tss.spmm(A, B))
    torch.cuda.synchronize()
    for t, (a, b, _, _) in enumerate(probs):
        for C in outs[t]:
            _check(a, b, C)
