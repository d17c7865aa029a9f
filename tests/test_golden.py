"""Regression fixtures (see tests/golden/README.md): the generators must still
draw the stored inputs and the oracle must still produce the stored outputs."""
import os

import numpy as np

import oracle
import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        head, body = line.split(":", 1)
        key, kind, n = head.split()
        vals = body.split()
        assert len(vals) == int(n)
        out[key] = np.array([int(v) for v in vals], np.int64) if kind == "i" else \
            np.array([float.fromhex(v) for v in vals], np.float64)
    return out


def test_spgemm_fixture():
    g = _read("spgemm_er12_d5.txt")
    seed = 20240811
    a = synth.er(12, 3, seed)
    b = synth.b_bernoulli(12, 5, 0.4, seed)
    assert np.array_equal(a.rp, g["a_rp"]) and np.array_equal(a.ci, g["a_ci"])
    assert np.array_equal(synth.values(a, "uniform", seed, synth.S_AVAL), g["a_val"].astype(np.float32))
    assert np.array_equal(b.rp, g["b_rp"]) and np.array_equal(b.ci, g["b_ci"])
    rp, ci, val = oracle.spgemm(g["a_rp"], g["a_ci"], g["a_val"], g["b_rp"], g["b_ci"], g["b_val"])
    assert np.array_equal(rp, g["c_rp"]) and np.array_equal(ci, g["c_ci"]) and np.array_equal(val, g["c_val"])


def test_msbfs_fixture():
    g = _read("msbfs_rmat6_d4.txt")
    a, srcs = synth.workload_bfs(scale=6, d=4, seed=20240812)
    assert np.array_equal(a.rp, g["a_rp"]) and np.array_equal(srcs, g["sources"])
    lev, fnnz = oracle.msbfs(g["a_rp"], g["a_ci"], g["sources"])
    assert np.array_equal(lev.ravel(), g["levels"]) and np.array_equal(fnnz, g["frontier_nnz"])


def test_grad_fixture():
    g = _read("grad_rmat4_d8.txt")
    rp, ci, _ = oracle.spgemm(g["a_rp"], g["a_ci"], g["a_val"], g["b_rp"], g["b_ci"], g["b_val"])
    ga = oracle.grad_a(g["a_rp"], g["a_ci"], g["b_rp"], g["b_ci"], g["b_val"], rp, ci, g["g"])
    gb = oracle.grad_b(g["a_rp"], g["a_ci"], g["a_val"], g["b_rp"], g["b_ci"], rp, ci, g["g"])
    assert np.array_equal(ga, g["grad_a"]) and np.array_equal(gb, g["grad_b"])
