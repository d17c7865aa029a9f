"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

The paper prints no worked example with values (its toy examples live in the
figures), so every pin here is a closed form, an invariant, dense brute force
on tiny inputs, or an independent library routine (numpy, scipy, networkx).
Each is chosen so that a plausible oracle mistake -- a dropped term, a wrong
index, a transposed operand, a missing mask -- fails at least one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests._util import csr_from_dense_pattern, dense, pattern, random_csr, rows_of

SEEDS = list(range(12))


def _oracle_dense(a, b):
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    out = np.zeros((a.nrows, b.ncols))
    pat = np.zeros((a.nrows, b.ncols), dtype=np.int64)
    r = rows_of(rp)
    out[r, ci] = val
    pat[r, ci] = 1
    return rp, ci, val, out, pat


# ---------------------------------------------------------------- Eq. (1): plus-times

@pytest.mark.parametrize("seed", SEEDS)
def test_plus_times_matches_dense_brute_force(seed):
    """Eq. (1) against an FP64 dense product; structure against the integer
    count product (entries with at least one contributing term)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    d = int(rng.choice([1, 3, 16, 33]))
    a = random_csr(rng, n, n, rng.uniform(0.02, 0.4), empty_rows=0.2, dense_rows=int(rng.integers(0, 2)))
    b = random_csr(rng, n, d, rng.uniform(0.05, 0.6), empty_rows=0.2)
    rp, ci, val, out, pat = _oracle_dense(a, b)
    count = pattern(a) @ pattern(b)
    assert np.array_equal(pat, (count > 0).astype(np.int64))
    np.testing.assert_allclose(out, dense(a) @ dense(b), rtol=1e-13, atol=0)
    # rows sorted, unique
    for i in range(n):
        seg = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_structural_zero_is_kept():
    """A numerically cancelling sum still occupies C's pattern (structural product)."""
    a = csr_from_dense_pattern(np.array([[1, 1]]), np.array([[1.0, -1.0]]))
    a.ncols = 2
    b = csr_from_dense_pattern(np.array([[1], [1]]), np.array([[2.0], [2.0]]))
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    assert list(rp) == [0, 1] and list(ci) == [0] and val[0] == 0.0


def test_products_are_exact_in_fp64():
    """FP32 x FP32 products are exact in FP64: a single-term entry equals the
    exact product (checked with Python's arbitrary-precision fractions)."""
    from fractions import Fraction

    rng = np.random.default_rng(7)
    x = rng.random(64).astype(np.float32)
    y = rng.random(64).astype(np.float32)
    n = 64
    a = synth.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), x)
    b = synth.Csr(n, 1, np.arange(n + 1, dtype=np.int32), np.zeros(n, dtype=np.int32), y)
    _, _, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    for t in range(n):
        assert Fraction(float(val[t])) == Fraction(float(x[t])) * Fraction(float(y[t]))


@pytest.mark.parametrize("seed", SEEDS[:6])
def test_integer_semiring_exact(seed):
    rng = np.random.default_rng(100 + seed)
    n, d = int(rng.integers(2, 50)), int(rng.choice([5, 32, 64]))
    a = random_csr(rng, n, n, 0.2, kind="int")
    b = random_csr(rng, n, d, 0.3, kind="int")
    rp, ci, val = oracle.spgemm_int(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    ref = dense(a, np.int64) @ dense(b, np.int64)
    got = np.zeros_like(ref)
    got[rows_of(rp), ci] = val
    assert np.array_equal(got, ref)
    assert np.array_equal((pattern(a) @ pattern(b) > 0), np.isin(np.arange(n * d), rows_of(rp) * d + ci).reshape(n, d))


# ---------------------------------------------------------------- closed forms

def test_identity_gives_b():
    rng = np.random.default_rng(3)
    n, d = 50, 17
    eye = synth.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    b = random_csr(rng, n, d, 0.3, empty_rows=0.1)
    rp, ci, val = oracle.spgemm(eye.rp, eye.ci, eye.val, b.rp, b.ci, b.val)
    assert np.array_equal(rp, b.rp) and np.array_equal(ci, b.ci) and np.array_equal(val, b.val.astype(np.float64))


def test_permutation_permutes_rows():
    rng = np.random.default_rng(4)
    n, d = 40, 9
    perm = rng.permutation(n).astype(np.int32)
    a = synth.Csr(n, n, np.arange(n + 1, dtype=np.int32), perm, np.ones(n, np.float32))
    b = random_csr(rng, n, d, 0.4)
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    for i in range(n):
        k = perm[i]
        assert np.array_equal(ci[rp[i]:rp[i + 1]], b.ci[b.rp[k]:b.rp[k + 1]])
        assert np.array_equal(val[rp[i]:rp[i + 1]], b.val[b.rp[k]:b.rp[k + 1]].astype(np.float64))


def test_one_hot_columns_select_columns_of_a():
    """B with a single 1 per column j at row r_j: C(:,j) = A(:, r_j)."""
    rng = np.random.default_rng(5)
    n, d = 30, 6
    a = random_csr(rng, n, n, 0.2)
    r = rng.choice(n, size=d, replace=False)
    bd = np.zeros((n, d))
    bd[r, np.arange(d)] = 1.0
    b = csr_from_dense_pattern(bd, bd)
    _, _, _, out, _ = _oracle_dense(a, b)
    assert np.array_equal(out, dense(a)[:, r])


def test_d1_is_sparse_matrix_sparse_vector():
    rng = np.random.default_rng(6)
    n = 60
    a = random_csr(rng, n, n, 0.1)
    b = random_csr(rng, n, 1, 0.3)
    _, _, _, out, _ = _oracle_dense(a, b)
    ref = sp.csr_matrix((a.val.astype(np.float64), a.ci, a.rp), shape=(n, n)) @ dense(b)[:, 0]
    np.testing.assert_allclose(out[:, 0], ref, rtol=1e-13)


def test_empty_inputs():
    n, d = 8, 4
    a = synth.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    rng = np.random.default_rng(1)
    b = random_csr(rng, n, d, 0.5)
    rp, ci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    assert rp[-1] == 0
    a2 = random_csr(rng, n, n, 0.5)
    b0 = synth.Csr(n, d, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    rp, ci, _ = oracle.spgemm(a2.rp, a2.ci, a2.val, b0.rp, b0.ci, b0.val)
    assert rp[-1] == 0


def test_dense_row_gives_union_of_b_rows():
    rng = np.random.default_rng(8)
    n, d = 25, 40
    pa = np.zeros((n, n), dtype=np.int64)
    pa[3, :] = 1
    a = csr_from_dense_pattern(pa, np.ones((n, n)))
    b = random_csr(rng, n, d, 0.1)
    rp, ci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    assert np.array_equal(ci[rp[3]:rp[4]], np.unique(b.ci))


# ---------------------------------------------------------------- Sec. II-A flops

@pytest.mark.parametrize("seed", SEEDS[:4])
def test_flops_definition_and_bounds(seed):
    rng = np.random.default_rng(200 + seed)
    n, d = 45, 20
    a = random_csr(rng, n, n, 0.15, empty_rows=0.2)
    b = random_csr(rng, n, d, 0.3)
    f = oracle.row_flops(a.rp, a.ci, b.rp)
    count = pattern(a) @ pattern(b)
    assert np.array_equal(f, count.sum(axis=1))  # every product A(i,k)B(k,j) counted once
    rp, _, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    assert np.all(np.diff(rp) <= np.minimum(d, f))
    assert np.all((np.diff(rp) == 0) == (f == 0))


# ---------------------------------------------------------------- library cross-check

def test_scipy_medium_size():
    """ER 4096 x 4096 times 4096 x 64 (positive values, no cancellation):
    scipy's float64 product gives the same pattern and values."""
    a, b = synth.workload_er_small()
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    sa = sp.csr_matrix((a.val.astype(np.float64), a.ci, a.rp), shape=(a.nrows, a.ncols))
    sb = sp.csr_matrix((b.val.astype(np.float64), b.ci, b.rp), shape=(b.nrows, b.ncols))
    sc = (sa @ sb).tocsr()
    sc.sort_indices()
    assert np.array_equal(rp, sc.indptr) and np.array_equal(ci, sc.indices)
    np.testing.assert_allclose(val, sc.data, rtol=1e-13)


# ---------------------------------------------------------------- (AND, OR) and masks

@pytest.mark.parametrize("seed", SEEDS[:6])
def test_boolean_and_complement_mask(seed):
    rng = np.random.default_rng(300 + seed)
    n, d = int(rng.integers(2, 40)), int(rng.choice([1, 8, 70]))
    a = random_csr(rng, n, n, 0.15)
    b = random_csr(rng, n, d, 0.2)
    m = random_csr(rng, n, d, 0.4)
    rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci)
    ref = (pattern(a) @ pattern(b)) > 0
    got = np.zeros((n, d), bool)
    got[rows_of(rp), ci] = True
    assert np.array_equal(got, ref)
    rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci, m.rp, m.ci)
    got = np.zeros((n, d), bool)
    got[rows_of(rp), ci] = True
    assert np.array_equal(got, ref & ~(pattern(m) > 0))


def test_row_subset_matches_full():
    a, b = synth.workload_er_small()
    rows = np.array([0, 17, 4095, 2048, 5], dtype=np.int32)
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    srp, sci, sval = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, rows=rows)
    for t, i in enumerate(rows):
        assert np.array_equal(sci[srp[t]:srp[t + 1]], ci[rp[i]:rp[i + 1]])
        assert np.array_equal(sval[srp[t]:srp[t + 1]], val[rp[i]:rp[i + 1]])
    rp8, ci8, val8 = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, threads=4)
    assert np.array_equal(rp8, rp) and np.array_equal(ci8, ci) and np.array_equal(val8, val)


# ---------------------------------------------------------------- transpose

def test_transpose_matches_scipy():
    rng = np.random.default_rng(11)
    a = random_csr(rng, 70, 50, 0.1, empty_rows=0.2)
    trp, tci, perm = oracle.transpose(a.rp, a.ci, 50)
    st = sp.csr_matrix((np.arange(a.nnz), a.ci, a.rp), shape=(70, 50)).T.tocsr()
    st.sort_indices()
    assert np.array_equal(trp, st.indptr) and np.array_equal(tci, st.indices)
    assert np.array_equal(perm, st.data)


# ---------------------------------------------------------------- Algorithm 3 / BFS

def _nx_levels(a, srcs):
    import networkx as nx

    g = nx.DiGraph()
    g.add_nodes_from(range(a.nrows))
    r = rows_of(a.rp)
    g.add_edges_from(zip(a.ci.tolist(), r.tolist()))  # k -> i when A(i,k) != 0
    lev = -np.ones((a.nrows, len(srcs)), dtype=np.int32)
    for j, s in enumerate(srcs):
        for v, l in nx.single_source_shortest_path_length(g, int(s)).items():
            lev[v, j] = l
    return lev


@pytest.mark.parametrize("seed", SEEDS[:5])
def test_queue_bfs_matches_networkx_directed(seed):
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(5, 80))
    a = random_csr(rng, n, n, rng.uniform(0.01, 0.1))  # not symmetric: direction matters
    srcs = rng.choice(n, size=min(n, 7), replace=False).astype(np.int32)
    assert np.array_equal(oracle.bfs_queue(a.rp, a.ci, srcs), _nx_levels(a, srcs))


def _sym_csr(n, edges):
    pat = np.zeros((n, n), dtype=np.int64)
    for u, v in edges:
        pat[u, v] = pat[v, u] = 1
    return csr_from_dense_pattern(pat)


def test_bfs_closed_forms():
    n = 30
    path = _sym_csr(n, [(i, i + 1) for i in range(n - 1)])
    srcs = np.array([0, 7, 29], dtype=np.int32)
    exp = np.abs(np.arange(n)[:, None] - srcs[None, :])
    for f in (lambda: oracle.msbfs(path.rp, path.ci, srcs)[0], lambda: oracle.bfs_queue(path.rp, path.ci, srcs)):
        assert np.array_equal(f(), exp)
    cyc = _sym_csr(n, [(i, (i + 1) % n) for i in range(n)])
    dd = np.abs(np.arange(n)[:, None] - srcs[None, :])
    assert np.array_equal(oracle.msbfs(cyc.rp, cyc.ci, srcs)[0], np.minimum(dd, n - dd))
    star = _sym_csr(n, [(0, i) for i in range(1, n)])
    lev = oracle.msbfs(star.rp, star.ci, np.array([0, 5], np.int32))[0]
    assert np.array_equal(lev[:, 0], np.r_[0, np.ones(n - 1, int)])
    exp5 = np.full(n, 2)
    exp5[0], exp5[5] = 1, 0
    assert np.array_equal(lev[:, 1], exp5)
    w, h = 7, 5
    grid = _sym_csr(w * h, [(y * w + x, y * w + x + 1) for y in range(h) for x in range(w - 1)] +
                    [(y * w + x, (y + 1) * w + x) for y in range(h - 1) for x in range(w)])
    s = np.array([0, 12, 34], np.int32)
    ys, xs = np.divmod(np.arange(w * h), w)
    sy, sx = np.divmod(s, w)
    man = np.abs(ys[:, None] - sy[None, :]) + np.abs(xs[:, None] - sx[None, :])
    assert np.array_equal(oracle.msbfs(grid.rp, grid.ci, s)[0], man)
    comp = _sym_csr(12, [(i, j) for i in range(12) for j in range(i + 1, 12)])
    lev = oracle.msbfs(comp.rp, comp.ci, np.array([3], np.int32))[0][:, 0]
    assert lev[3] == 0 and np.all(np.delete(lev, 3) == 1)
    # unreachable vertices: two components
    two = _sym_csr(10, [(0, 1), (1, 2), (5, 6)])
    lev = oracle.msbfs(two.rp, two.ci, np.array([0, 5], np.int32))[0]
    assert list(lev[:, 0]) == [0, 1, 2, -1, -1, -1, -1, -1, -1, -1]
    assert list(lev[:, 1]) == [-1, -1, -1, -1, -1, 0, 1, -1, -1, -1]


@pytest.mark.parametrize("scale", [6, 9, 11])
def test_algorithm3_matches_queue_bfs_and_invariants(scale):
    a, srcs = synth.workload_bfs(scale=scale, d=32)
    lev3, fnnz, fflops = oracle.msbfs(a.rp, a.ci, srcs, return_flops=True)
    levq = oracle.bfs_queue(a.rp, a.ci, srcs, threads=4)
    assert np.array_equal(lev3, levq)
    # sum over iterations of nnz(F) = sum over sources of (|reach(s)| - 1)
    assert fnnz.sum() == (levq >= 0).sum() - len(srcs)
    # Sec. II-A flops summed over the iterations of Algorithm 3: every reached
    # (v, s) is in exactly one multiplied frontier, and F(v, s) meets every
    # stored A(i, v), so sum_t flops(A F_t) = sum_s sum_{v in reach(s)} deg(v)
    # with deg(v) the entries of column v of A (reach from the queue BFS)
    deg = np.bincount(a.ci, minlength=a.nrows).astype(np.int64)
    assert len(fflops) == len(fnnz) and fflops[-1] > 0
    assert int(fflops.sum()) == int((deg[:, None] * (levq >= 0)).sum())
    # per-iteration frontier sizes are the level histogram
    for t, f in enumerate(fnnz, start=1):
        assert f == (levq == t).sum()
    assert (levq == len(fnnz) + 1).sum() == 0


# ---------------------------------------------------------------- gradients

def _loss(a, aval, b, bval, w_dense):
    rp, ci, val = oracle.spgemm(a.rp, a.ci, aval, b.rp, b.ci, bval)
    return float(np.dot(val, w_dense[rows_of(rp), ci]))


@pytest.mark.parametrize("seed", SEEDS[:4])
def test_gradients_dense_closed_form(seed):
    rng = np.random.default_rng(500 + seed)
    n, d = int(rng.integers(3, 30)), int(rng.choice([4, 16]))
    a = random_csr(rng, n, n, 0.2, kind="normal")
    b = random_csr(rng, n, d, 0.3, kind="normal")
    rp, ci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    w = rng.standard_normal((n, d))
    g = w[rows_of(rp), ci]
    gd = np.zeros((n, d))
    gd[rows_of(rp), ci] = g
    ga = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, b.val, rp, ci, g)
    gb = oracle.grad_b(a.rp, a.ci, a.val, b.rp, b.ci, rp, ci, g)
    ref_a = (gd @ dense(b).T)[rows_of(a.rp), a.ci]
    ref_b = (dense(a).T @ gd)[rows_of(b.rp), b.ci]
    np.testing.assert_allclose(ga, ref_a, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gb, ref_b, rtol=1e-12, atol=1e-12)
    # sampled forms agree with the full ones
    rows = np.array(sorted(rng.choice(n, size=min(n, 5), replace=False)), np.int32)
    sel_a = np.concatenate([np.arange(a.rp[i], a.rp[i + 1]) for i in rows])
    np.testing.assert_array_equal(oracle.grad_a_rows(a.rp, a.ci, b.rp, b.ci, b.val, rp, ci, g, rows), ga[sel_a])
    sel_b = np.concatenate([np.arange(b.rp[k], b.rp[k + 1]) for k in rows])
    np.testing.assert_allclose(oracle.grad_b_rows(a.rp, a.ci, a.val, b.rp, b.ci, rp, ci, g, rows), gb[sel_b],
                               rtol=1e-14, atol=1e-14)


def test_gradients_central_differences_are_exact():
    """L is linear in each single entry, so a central difference with h = 2^-10
    equals the partial derivative up to FP64 rounding (loss of size ~1e2)."""
    a, b = synth.workload_embedding(scale=8, d=16, density=0.2)
    rp, ci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    rng = np.random.default_rng(9)
    w = rng.standard_normal((a.nrows, b.ncols))
    g = w[rows_of(rp), ci]
    ga = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, b.val, rp, ci, g)
    gb = oracle.grad_b(a.rp, a.ci, a.val, b.rp, b.ci, rp, ci, g)
    h = 2.0**-10
    av0, bv0 = a.val.astype(np.float64), b.val.astype(np.float64)
    for p in rng.choice(a.nnz, size=24, replace=False):
        ap, am = av0.copy(), av0.copy()
        ap[p] += h
        am[p] -= h
        fd = (_loss(a, ap, b, bv0, w) - _loss(a, am, b, bv0, w)) / (2 * h)
        assert abs(fd - ga[p]) <= 1e-9 * (1 + abs(ga[p]))
    for q in rng.choice(b.nnz, size=24, replace=False):
        bp, bm = bv0.copy(), bv0.copy()
        bp[q] += h
        bm[q] -= h
        fd = (_loss(a, av0, b, bp, w) - _loss(a, av0, b, bm, w)) / (2 * h)
        assert abs(fd - gb[q]) <= 1e-9 * (1 + abs(gb[q]))
    # directional derivative along random (U, V): exact up to the quadratic term,
    # which central differences cancel for a bilinear form
    u = rng.standard_normal(a.nnz)
    v = rng.standard_normal(b.nnz)
    fd = (_loss(a, av0 + h * u, b, bv0 + h * v, w) - _loss(a, av0 - h * u, b, bv0 - h * v, w)) / (2 * h)
    assert abs(fd - (ga @ u + gb @ v)) <= 1e-8 * (1 + abs(fd))
