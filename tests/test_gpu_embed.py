"""GPU parity of the sparse-embedding update (Sec. IV-B) against the oracle.

Both sides round u = z + lr F (FP64) once to FP32 and select on those FP32
values. In the first minibatch both start from the same Z and their FP64
sums differ only in order, so every value is within one FP32 ulp of the
oracle's. Later minibatches read rows that earlier ones rounded, so those
differences carry forward: there a value may differ by one ulp plus 2^-20 of
its row's largest magnitude. The selected columns must be identical
everywhere. Cases run whole minibatch schedules, at sizes that span several
workgroups, all lane-group shapes of the kernel and a ragged last minibatch.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import note, require_gpu

pytestmark = pytest.mark.gpu

LR = float(np.float32(0.02))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _graph(n_scale, ef, ns, seed):
    g = synth.rmat(n_scale, ef, seed)
    return synth.signed_graph(g, synth.negatives(g, ns, seed))


def _run_gpu(a, zci, zval, d, k, lr, batch, r0=0, r1=None):
    import paper_2408_11988_amd as tss

    A = tss.DeviceCsr.from_host(a)
    ci = torch.from_numpy(zci).cuda()
    val = torch.from_numpy(zval).cuda()
    tss.embed_epoch(A, ci, val, d, k, lr, batch, r0, r1)
    torch.cuda.synchronize()
    return ci.cpu().numpy(), val.cpu().numpy()


def _assert_same(got, want, k, what, first=None):
    """Columns identical; values within 1 ulp in the rows of the first
    minibatch (`first` = (r0, r1), default: every row) and within
    1 ulp + 2^-20 * (row's largest |value|) elsewhere."""
    gci, gval = got
    wci, wval = want
    rows_bad = np.nonzero((gci != wci).reshape(-1, k).any(axis=1))[0]
    assert len(rows_bad) == 0, f"{what}: selected columns differ in rows {rows_bad[:10]}"
    n = len(wval) // k
    w = wval.astype(np.float64).reshape(n, k)
    ulp = np.spacing(np.abs(wval).astype(np.float32)).astype(np.float64).reshape(n, k)
    err = np.abs(gval.astype(np.float64).reshape(n, k) - w)
    r0, r1 = first if first is not None else (0, n)
    strict = np.zeros(n, bool)
    strict[r0:r1] = True
    assert np.all(err[strict] <= ulp[strict]), f"{what}: first minibatch, worst {np.max(err[strict] / ulp[strict])} ulp"
    tol = ulp + 2.0 ** -20 * np.abs(w).max(axis=1, keepdims=True)
    assert np.all(err <= tol), f"{what}: worst error {np.max(err / tol)} of the tolerance"


# (d, k): lane groups of 8, 16, 32 and 64 lanes, and 2, 4, 8, 16 entries per lane
SHAPES = [(16, 3), (64, 13), (128, 26), (128, 64), (200, 100), (512, 200), (1024, 300), (1024, 1024), (1, 1)]


@pytest.mark.parametrize("d,k", SHAPES)
def test_embed_epoch_matches_oracle(d, k):
    a = _graph(9, 6, 4, 4000 + d + k)
    zci, zval = synth.embed_init(a.nrows, d, k, 4100 + d + k)
    for batch in (37, a.nrows):
        note(f"embed n={a.nrows} nnzA={a.nnz} d={d} k={k} batch={batch}")
        got = _run_gpu(a, zci, zval, d, k, LR, batch)
        want = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, LR, batch)
        _assert_same(got, want, k, f"d={d} k={k} batch={batch}", first=(0, batch))


def test_embed_batch_of_one_row_and_row_range():
    d, k = 64, 10
    a = _graph(8, 6, 3, 4200)
    zci, zval = synth.embed_init(a.nrows, d, k, 4201)
    note("embed batch=1 (one launch per row)")
    got = _run_gpu(a, zci, zval, d, k, 0.5, 1)
    _assert_same(got, oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, 0.5, 1), k, "batch=1", first=(0, 1))
    for r0, r1, b in ((17, 200, 23), (0, 64, 64), (100, 101, 5)):
        note(f"embed rows [{r0}, {r1}) batch={b}")
        got = _run_gpu(a, zci, zval, d, k, 0.3, b, r0, r1)
        want = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, 0.3, b, r0, r1)
        _assert_same(got, want, k, f"rows [{r0},{r1})", first=(r0, min(r1, r0 + b)))
        outside = np.ones(a.nrows, bool)
        outside[r0:r1] = False
        assert np.array_equal(got[0].reshape(-1, k)[outside], zci.reshape(-1, k)[outside])


def test_embed_edge_cases():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd import _lib

    d, k, n = 32, 8, 300
    zci, zval = synth.embed_init(n, d, k, 4300)
    empty = synth.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    note("embed with no edges: rows keep their entries")
    got = _run_gpu(empty, zci, zval, d, k, 0.5, 16)
    assert np.array_equal(got[0], zci) and np.array_equal(got[1], zval)
    a = _graph(8, 4, 2, 4301)
    a0 = synth.Csr(a.nrows, a.ncols, a.rp, a.ci, np.zeros(a.nnz, np.float32))
    zci, zval = synth.embed_init(a.nrows, d, k, 4302)
    note("embed with zero weights and with lr = 0")
    for m, lr in ((a0, 0.5), (a, 0.0)):
        got = _run_gpu(m, zci, zval, d, k, lr, 16)
        assert np.array_equal(got[0], zci) and np.array_equal(got[1], zval)
    note("embed with ties: repeated magnitudes, zeros in the initial rows")
    tz = zval.copy()
    tz[::3] = 0.0
    tz[1::3] = np.sign(tz[1::3]) * np.float32(0.25)
    got = _run_gpu(a, zci, tz, d, k, 0.05, 9)
    _assert_same(got, oracle.embed_epoch(a.rp, a.ci, a.val, zci, tz, d, k, 0.05, 9), k, "ties", first=(0, 9))
    A = tss.DeviceCsr.from_host(a)
    ci = torch.from_numpy(zci).cuda()
    val = torch.from_numpy(zval).cuda()
    note("embed argument errors")
    for args, code in (((d, d + 1, 0.1, 4), _lib.ERR_INVALID_ARG), ((d, k, 0.1, 0), _lib.ERR_INVALID_ARG),
                       ((2048, k, 0.1, 4), _lib.ERR_UNSUPPORTED)):
        with pytest.raises(_lib.TSSpGEMMError) as e:
            if args[1] != k:
                tss.embed_epoch(A, torch.zeros(a.nrows * args[1], dtype=torch.int32, device="cuda"),
                                torch.zeros(a.nrows * args[1], device="cuda"), *args)
            else:
                tss.embed_epoch(A, ci, val, *args)
        assert e.value.code == code


def test_embed_full_workload_epoch_and_determinism():
    """The benchmarked workload (R-MAT 17, edge factor 8, 5 negative samples,
    d = 128 at 80% sparsity) for a whole epoch of 256-row minibatches and of
    two half-size minibatches, against the oracle, twice (bit-identical)."""
    a, zci, zval, k = synth.workload_embed_step()
    d = 128
    for batch in (256, (a.nrows + 1) // 2):
        note(f"embed full workload n={a.nrows} nnzA={a.nnz} k={k} batch={batch}")
        got = _run_gpu(a, zci, zval, d, k, LR, batch)
        again = _run_gpu(a, zci, zval, d, k, LR, batch)
        assert np.array_equal(got[0], again[0]) and np.array_equal(got[1].view(np.int32), again[1].view(np.int32))
        want = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, LR, batch)
        _assert_same(got, want, k, f"full workload batch={batch}", first=(0, batch))


def test_embed_epoch_in_a_graph_replays():
    """One epoch captured into a HIP graph (torch.cuda.CUDAGraph), replayed
    three times on fresh copies of Z, with eager work in between."""
    import paper_2408_11988_amd as tss

    d, k, batch = 128, 26, 64
    a = _graph(10, 6, 5, 4400)
    zci, zval = synth.embed_init(a.nrows, d, k, 4401)
    A = tss.DeviceCsr.from_host(a)
    ci0 = torch.from_numpy(zci).cuda()
    val0 = torch.from_numpy(zval).cuda()
    ci = ci0.clone()
    val = val0.clone()
    want = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, LR, batch)
    note("embed warm-up, then capture")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tss.embed_epoch(A, ci, val, d, k, LR, batch)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    ci.copy_(ci0)
    val.copy_(val0)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        tss.embed_epoch(A, ci, val, d, k, LR, batch)
    for rep in range(3):
        ci.copy_(ci0)
        val.copy_(val0)
        _ = (val0 * 2).sum().item()  # eager work between replays
        note(f"embed graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        _assert_same((ci.cpu().numpy(), val.cpu().numpy()), want, k, f"graph replay {rep}", first=(0, batch))
