"""GPU multi-source BFS (Algorithm 3 by masked Boolean TS-SpGEMM) against the
oracle's queue BFS (independent algorithm) and Algorithm 3 frontier counts.
Levels are integers: compared exactly."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import csr_from_dense_pattern, random_csr
from tests.gpu_util import note, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _bfs(a, srcs):
    import paper_2408_11988_amd as tss

    A = to_dev(a, with_values=False)
    lev, fn = tss.msbfs(A, torch.from_numpy(np.ascontiguousarray(srcs, dtype=np.int32)).cuda())
    torch.cuda.synchronize()
    return lev.cpu().numpy(), fn


def _sym(n, edges):
    pat = np.zeros((n, n), dtype=np.int64)
    for u, v in edges:
        pat[u, v] = pat[v, u] = 1
    return csr_from_dense_pattern(pat)


def test_closed_forms():
    n = 40
    path = _sym(n, [(i, i + 1) for i in range(n - 1)])
    srcs = np.array([0, 13, 39], np.int32)
    note("path graph")
    lev, fn = _bfs(path, srcs)
    assert np.array_equal(lev, np.abs(np.arange(n)[:, None] - srcs[None, :]))
    w, h = 9, 6
    grid = _sym(w * h, [(y * w + x, y * w + x + 1) for y in range(h) for x in range(w - 1)] +
                [(y * w + x, (y + 1) * w + x) for y in range(h - 1) for x in range(w)])
    s = np.array([0, 22, 53, 8], np.int32)
    ys, xs = np.divmod(np.arange(w * h), w)
    sy, sx = np.divmod(s, w)
    note("2-D grid")
    lev, _ = _bfs(grid, s)
    assert np.array_equal(lev, np.abs(ys[:, None] - sy[None, :]) + np.abs(xs[:, None] - sx[None, :]))
    two = _sym(10, [(0, 1), (1, 2), (5, 6)])
    note("two components + isolated vertices")
    lev, fn = _bfs(two, np.array([0, 5, 9], np.int32))
    assert list(lev[:, 0]) == [0, 1, 2, -1, -1, -1, -1, -1, -1, -1]
    assert list(lev[:, 1]) == [-1, -1, -1, -1, -1, 0, 1, -1, -1, -1]
    assert list(lev[:, 2]) == [-1] * 9 + [0]


@pytest.mark.parametrize("d", [1, 7, 32, 33, 64, 100])
def test_directed_random_vs_queue_bfs(d):
    rng = np.random.default_rng(700 + d)
    n = 500
    a = random_csr(rng, n, n, 0.004)  # not symmetric: A F direction matters
    srcs = rng.choice(n, size=d, replace=False).astype(np.int32)
    note(f"directed random n={n} d={d}")
    lev, fn = _bfs(a, srcs)
    assert np.array_equal(lev, oracle.bfs_queue(a.rp, a.ci, srcs))
    lev3, fn3 = oracle.msbfs(a.rp, a.ci, srcs)
    assert np.array_equal(lev, lev3) and list(fn) == list(fn3)


@pytest.mark.parametrize("scale,d", [(10, 64), (12, 512), (14, 256), (16, 512)])
def test_rmat_vs_queue_bfs(scale, d):
    a, srcs = synth.workload_bfs(scale=scale, d=d)
    note(f"R-MAT scale {scale} d={d} nnz={a.nnz}")
    lev, fn = _bfs(a, srcs)
    ref = oracle.bfs_queue(a.rp, a.ci, srcs, threads=16)
    assert np.array_equal(lev, ref)
    counts = [int((ref == t).sum()) for t in range(1, len(fn) + 1)]
    assert list(fn) == counts and fn[-1] == 0
    if scale <= 12:
        _, fn3 = oracle.msbfs(a.rp, a.ci, srcs)
        assert list(fn) == list(fn3)


@pytest.fixture(scope="module")
def rmat22_levels():
    """The full-size BFS workload (R-MAT scale 22, 512 sources) run once on the
    GPU; its levels are kept on the host for the checks below."""
    import paper_2408_11988_amd as tss

    a, srcs = synth.workload_bfs(scale=22, d=512)
    note(f"R-MAT 22 d=512 nnz={a.nnz}")
    A = to_dev(a, with_values=False)
    lev, fn = tss.msbfs(A, torch.from_numpy(srcs).cuda())
    torch.cuda.synchronize()
    per_level = [int((lev == t).sum()) for t in range(0, len(fn) + 1)]
    host = lev.cpu().numpy()
    del lev, A
    torch.cuda.empty_cache()
    return a, srcs, host, fn, per_level


def test_rmat_scale22_d512_invariants(rmat22_levels):
    """Every column: sources at level 0, and the per-iteration frontier sizes
    equal the level histogram (Algorithm 3)."""
    a, srcs, lev, fn, per_level = rmat22_levels
    d = len(srcs)
    assert np.all(lev[srcs, np.arange(d)] == 0)
    assert per_level[0] == d  # level 0: the sources
    assert per_level[1:len(fn)] == list(fn[:-1]) and fn[-1] == 0 and per_level[len(fn)] == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("part", range(4))
def test_rmat_scale22_d512_full(part, rmat22_levels):
    """Full-size workload: the levels of every source (128 per part) compared
    exactly with the oracle's queue BFS."""
    a, srcs, lev, fn, _ = rmat22_levels
    cols = np.arange(part * 128, (part + 1) * 128)
    note(f"queue BFS on sources {cols[0]}..{cols[-1]}")
    ref = oracle.bfs_queue(a.rp, a.ci, srcs[cols], threads=16)
    assert np.array_equal(lev[:, cols], ref)


def test_bad_source_is_an_error():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd import _lib

    a = _sym(8, [(0, 1), (1, 2)])
    note("source out of range")
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.msbfs(to_dev(a, with_values=False), torch.tensor([1, 8], dtype=torch.int32, device="cuda"))
    assert e.value.code == _lib.ERR_INVALID_ARG


def test_workspace_reused_across_calls():
    """The device's BFS workspace is kept between calls: a deeper search on a
    larger graph, then a shallow one on a smaller graph with another d (the
    kept frontiers are longer than needed), then the first again, each
    matching the queue BFS exactly."""
    rng = np.random.default_rng(1700)
    n1 = 3000
    path = _sym(n1, [(i, i + 1) for i in range(n1 - 1)] + [(i, i + 3) for i in range(0, n1 - 3, 7)])
    s1 = rng.choice(n1, size=64, replace=False).astype(np.int32)
    pat = rng.random((500, 500)) < 0.01
    small = csr_from_dense_pattern((pat | pat.T).astype(np.int64))
    s2 = rng.choice(500, size=200, replace=False).astype(np.int32)
    for a, s in ((path, s1), (small, s2), (path, s1)):
        note(f"msbfs n={a.nrows} d={len(s)}")
        lev, fn = _bfs(a, s)
        assert np.array_equal(lev, oracle.bfs_queue(a.rp, a.ci, s))
