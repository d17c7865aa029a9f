"""Pins of the sparse-embedding oracle (Sec. IV-B), CPU only.

The force on a row is checked against torch autograd of the log-likelihood
whose gradient it is by definition (sum over neighbours of log sig(z_i . z_j)
plus sum over negative samples of log sig(-z_i . z_j)), the whole update
against a hand-computed case with exact binary values, the re-sparsification
against the defining property of a top-k selection, and the minibatch
schedule against a literal composition of single-row updates.
"""
import numpy as np
import pytest
import torch

import oracle
import synth


def _small_graph(seed, n=40, d=16, k=5, ns=3, ef=4):
    g = synth.er(n, ef, seed)
    a = synth.signed_graph(g, synth.negatives(g, ns, seed))
    zci, zval = synth.embed_init(n, d, k, seed)
    return a, zci, zval


def _dense_rows(zci, zval, n, d, k):
    z = np.zeros((n, d))
    z[np.repeat(np.arange(n), k), zci] = zval
    return z


def force_is_loglik_gradient(seed=3):
    """Pin: F_i equals d/dz_i of sum log sig(+-z_i . z_j) (torch autograd, FP64)."""
    n, d, k = 40, 16, 5
    a, zci, zval = _small_graph(seed, n, d, k)
    Z = torch.from_numpy(_dense_rows(zci, zval, n, d, k))
    ok = True
    for i in range(n):
        lo, hi = a.rp[i], a.rp[i + 1]
        if hi == lo:
            continue
        zi = Z[i].clone().requires_grad_(True)
        js = torch.from_numpy(a.ci[lo:hi].astype(np.int64))
        sgn = torch.from_numpy(a.val[lo:hi].astype(np.float64))
        loss = torch.nn.functional.logsigmoid(sgn * (Z[js] @ zi)).sum()
        loss.backward()
        F = oracle.embed_force(a.rp, a.ci, a.val, zci, zval, d, k, i)
        ok &= bool(np.allclose(F, zi.grad.numpy(), rtol=1e-12, atol=1e-14))
    return ok


def closed_form_holds():
    """Pin: mutually orthogonal rows (every z_i . z_j = 0, so sig = 1/2) and
    lr = 1/2 make every value exact in binary; the expected rows are worked
    out by hand."""
    d, k = 4, 2
    rp = np.array([0, 2, 3, 4], np.int32)
    ci = np.array([1, 2, 0, 1], np.int32)
    val = np.array([1, -1, 1, -1], np.float32)  # row 0: +z1, -z2; row 1: +z0; row 2: -z1
    zci = np.array([0, 1, 2, 3, 2, 3], np.int32)
    zval = np.array([1.0, 0.5, 2.0, -1.0, 1.0, 2.0], np.float32)
    # row 0: F = (z1 - z2) / 2 = (0, 0, 0.5, -1.5);  u = (1, 0.5, 0.25, -0.75) -> cols 0, 3
    # row 1: F = z0 / 2 = (0.5, 0.25, 0, 0);        u = (0.25, 0.125, 2, -1)  -> cols 2, 3
    # row 2: F = -z1 / 2 = (0, 0, -1, 0.5);         u = (0, 0, 0.5, 2.25)     -> cols 2, 3
    want_ci = np.array([0, 3, 2, 3, 2, 3], np.int32)
    want_val = np.array([1.0, -0.75, 2.0, -1.0, 0.5, 2.25], np.float32)
    got_ci, got_val = oracle.embed_epoch(rp, ci, val, zci, zval, d, k, 0.5, batch=3)
    return bool(np.array_equal(got_ci, want_ci) and np.array_equal(got_val, want_val))


def topk_property_holds(seed=5):
    """Pin: the selection keeps exactly k columns, sorted; every kept |u| is
    >= every dropped |u|; at equal |u| a kept column is lower than a dropped
    one; kept values are fp32(z + lr F)."""
    rng = np.random.default_rng(seed)
    ok = True
    for trial in range(40):
        d = int(rng.integers(1, 40))
        k = int(rng.integers(1, d + 1))
        zi = rng.choice([0.0, 0.5, -0.5, 1.0, -2.0], size=d) if trial % 2 else rng.standard_normal(d)
        F = np.zeros(d) if trial % 3 == 0 else rng.standard_normal(d)
        lr = 0.25
        u = (zi + lr * F).astype(np.float32)
        ci, val = oracle.embed_select(zi, F, lr, k)
        ok &= len(ci) == k and bool(np.all(np.diff(ci) > 0))
        ok &= bool(np.array_equal(val, u[ci]))
        dropped = np.setdiff1d(np.arange(d), ci)
        if len(dropped):
            kept_min = np.abs(u[ci]).min()
            drop_max = np.abs(u[dropped]).max()
            ok &= bool(kept_min >= drop_max)
            tie = np.abs(u[ci]) == drop_max
            if tie.any():
                ok &= bool(ci[tie].max() < dropped[np.abs(u[dropped]) == drop_max].min())
    return ok


def minibatch_schedule_holds(seed=7):
    """Pin: minibatches of b rows equal, for each batch in row order, every row
    updated from a frozen copy of the embedding taken at the batch start."""
    n, d, k = 40, 16, 5
    a, zci, zval = _small_graph(seed, n, d, k)
    lr = float(np.float32(0.3))
    ok = True
    for b, r0, r1 in ((1, 0, n), (7, 0, n), (n, 0, n), (5, 3, 31)):
        got_ci, got_val = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, lr, b, r0, r1)
        ci, v = zci.copy(), zval.copy()
        for s in range(r0, r1, b):
            e = min(r1, s + b)
            frozen_ci, frozen_v = ci.copy(), v.copy()
            for i in range(s, e):
                F = oracle.embed_force(a.rp, a.ci, a.val, frozen_ci, frozen_v, d, k, i)
                zi = np.zeros(d)
                zi[frozen_ci[i * k:(i + 1) * k]] = frozen_v[i * k:(i + 1) * k]
                ci[i * k:(i + 1) * k], v[i * k:(i + 1) * k] = oracle.embed_select(zi, F, lr, k)
        ok &= bool(np.array_equal(got_ci, ci) and np.array_equal(got_val, v))
    return ok


def test_force_is_the_loglikelihood_gradient():
    assert force_is_loglik_gradient()


def test_closed_form_orthogonal_rows():
    assert closed_form_holds()


def test_topk_defining_property():
    assert topk_property_holds()


def test_minibatch_schedule():
    assert minibatch_schedule_holds()


def test_lr_zero_and_isolated_rows_keep_their_entries():
    n, d, k = 40, 16, 5
    a, zci, zval = _small_graph(11, n, d, k)
    assert np.all(zval != 0)
    got_ci, got_val = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, 0.0, 8)
    assert np.array_equal(got_ci, zci) and np.array_equal(got_val, zval)
    empty = synth.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    got_ci, got_val = oracle.embed_epoch(empty.rp, empty.ci, empty.val, zci, zval, d, k, 0.5, 8)
    assert np.array_equal(got_ci, zci) and np.array_equal(got_val, zval)


def test_k_equal_d_keeps_every_column():
    n, d = 30, 6
    a, zci, zval = _small_graph(13, n, d, d, ns=2, ef=3)
    got_ci, got_val = oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, d, 0.1, 4)
    assert np.array_equal(got_ci, np.tile(np.arange(d, dtype=np.int32), n))


def test_bad_arguments_are_rejected():
    a, zci, zval = _small_graph(1)
    with pytest.raises(ValueError):
        oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, 16, 17, 0.1, 4)
    with pytest.raises(ValueError):
        oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, 16, 5, 0.1, 0)
