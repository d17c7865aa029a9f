"""Statistical checks of the seeded generators (their exact output is not
pinned by anything outside this repository; see tests/golden for drift)."""
import math

import numpy as np

import synth


def test_er_row_counts_and_determinism():
    a = synth.er(4096, 8, 11)
    deg = np.diff(a.rp)
    # 8 draws from 4096 columns: expected unique 4096 (1 - (1 - 1/4096)^8) ~ 7.993
    assert abs(deg.mean() - 4096 * (1 - (1 - 1 / 4096) ** 8)) < 0.02
    assert np.all(np.diff(a.ci[a.rp[0]:a.rp[1]]) > 0)
    b = synth.er(4096, 8, 11)
    assert np.array_equal(a.ci, b.ci)


def test_bernoulli_density():
    b = synth.b_bernoulli(20000, 64, 0.1, 5)
    assert abs(b.nnz / (20000 * 64) - 0.1) < 0.002
    for i in (0, 7, 19999):
        seg = b.ci[b.rp[i]:b.rp[i + 1]]
        assert np.all(np.diff(seg) > 0) and (len(seg) == 0 or seg.max() < 64)


def test_poisson_rows():
    b = synth.b_poisson(50000, 128, 25.6, 6)
    deg = np.diff(b.rp)
    assert abs(deg.mean() - 25.6) < 0.1 and abs(deg.var() - 25.6) < 1.0
    assert np.all(np.diff(b.ci[b.rp[3]:b.rp[4]]) > 0)


def test_rmat_structure():
    a = synth.rmat(12, 16, 3)
    n = 4096
    rows = np.repeat(np.arange(n), np.diff(a.rp))
    assert np.all(a.ci != rows)  # no self-loops
    # symmetric pattern
    key = rows.astype(np.int64) * n + a.ci
    keyt = a.ci.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(key), np.sort(keyt))
    # top-level quadrant frequencies of an undirected R-MAT: (0,0) ~ a, off-diagonal ~ b + c, (1,1) ~ d
    top_r, top_c = rows >= n // 2, a.ci >= n // 2
    f00 = np.mean(~top_r & ~top_c)
    f11 = np.mean(top_r & top_c)
    assert abs(f00 - 0.57) < 0.05 and abs(f11 - 0.05) < 0.03


def test_values_are_fp32_grid_and_keyed_by_position():
    a = synth.er(256, 4, 9)
    v = synth.values(a, "uniform", 9, synth.S_AVAL)
    assert v.min() > 0 and v.max() <= 1
    assert np.all((v.astype(np.float64) * 2**24) == np.round(v.astype(np.float64) * 2**24))
    n = synth.values(a, "normal", 9, synth.S_AVAL)
    assert abs(n.mean()) < 0.1 and abs(n.std() - 1) < 0.1


def test_sources_distinct_non_isolated():
    a = synth.rmat(10, 16, 1)
    s = synth.sources(a, 64, 2)
    assert len(set(s.tolist())) == 64
    assert np.all(a.rp[s + 1] > a.rp[s])


def test_batched_params_ranges():
    ps = synth.batched_params()
    assert len(ps) == 64
    for p in ps:
        assert 2**14 <= p["n"] <= 2**18 and p["d"] in (32, 64, 128, 256) and 4 <= p["k"] <= 32
        assert 0.01 <= p["density"] <= 0.5 and p["kind"] in ("er", "rmat")
    assert math.isclose(np.mean([p["kind"] == "er" for p in ps]), 0.5, abs_tol=0.2)


def test_negatives_and_signed_graph():
    g = synth.rmat(9, 8, 123)
    neg = synth.negatives(g, 5, 123)
    a = synth.signed_graph(g, neg)
    assert a.nnz == g.nnz + neg.nnz
    for i in range(g.nrows):
        nb = set(g.ci[g.rp[i]:g.rp[i + 1]].tolist())
        ng = neg.ci[neg.rp[i]:neg.rp[i + 1]]
        assert len(set(ng.tolist())) == len(ng) and i not in ng and not (nb & set(ng.tolist()))
        assert len(ng) == min(5, g.nrows - 1 - len(nb))
        row = a.ci[a.rp[i]:a.rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        sgn = a.val[a.rp[i]:a.rp[i + 1]]
        assert set(row[sgn > 0].tolist()) == nb and set(row[sgn < 0].tolist()) == set(ng.tolist())
    again = synth.negatives(g, 5, 123)
    assert np.array_equal(again.ci, neg.ci)


def test_embed_init_rows():
    n, d, k = 500, 64, 13
    ci, val = synth.embed_init(n, d, k, 9)
    rows = ci.reshape(n, k)
    assert np.all(np.diff(rows, axis=1) > 0) and rows.min() >= 0 and rows.max() < d
    assert np.all(val != 0) and abs(float(np.std(val)) * np.sqrt(k) - 1.0) < 0.05
    ci2, val2 = synth.embed_init(n, d, k, 9)
    assert np.array_equal(ci, ci2) and np.array_equal(val, val2)
