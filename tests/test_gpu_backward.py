"""GPU backward of the plus-times TS-SpGEMM against the oracle.

A^T is integer index work: compared exactly. Gradients are FP32 outputs of FP64
sums over signed data: |gpu - oracle| <= 1e-5 * (sum of |terms|), the
forward-error scale (plain relative error is undefined under cancellation).
The oracle gradient itself is pinned to FP64 central differences (exact for a
bilinear loss) in the CPU suite and again here at n = 2048, d = 32.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import random_csr, rows_of
from tests.gpu_util import compare_f32, note, require_gpu, to_dev

pytestmark = pytest.mark.gpu
RTOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _tss():
    import paper_2408_11988_amd as tss

    return tss


@pytest.mark.parametrize("case", ["random", "rmat14", "rmat18"])
def test_transpose_exact(case):
    rng = np.random.default_rng(31)
    if case == "random":
        a = random_csr(rng, 700, 700, 0.01, empty_rows=0.2, dense_rows=3)
    else:
        a = synth.rmat(int(case[4:]), 16, 5)
    note(f"transpose {case} nnz={a.nnz}")
    AT, perm = _tss().transpose(to_dev(a, with_values=False))
    trp, tci, tperm = oracle.transpose(a.rp, a.ci, a.ncols)
    assert np.array_equal(AT.rowptr.cpu().numpy(), trp)
    assert np.array_equal(AT.colidx.cpu().numpy(), tci)
    assert np.array_equal(perm.cpu().numpy(), tperm)
    if case == "rmat18":
        assert np.diff(trp).max() > 4096  # columns spanning several sort tiles


def _grads_gpu(a, b, g, tuning=None):
    tss = _tss()
    A, B = to_dev(a), to_dev(b)
    C, plan = tss.spgemm(A, B, tuning=tuning, return_plan=True)
    G = C.with_vals(torch.from_numpy(g.astype(np.float32)).cuda())
    ga = tss.grad_a(plan, A, B, G)
    AT, perm = tss.transpose(A)
    gb = tss.grad_b(plan, AT, perm, A, B, G)
    torch.cuda.synchronize()
    return ga.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64), C


def _check(a, b, ga, gb, crp, cci, g):
    ref_a = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, b.val, crp, cci, g)
    ref_b = oracle.grad_b(a.rp, a.ci, a.val, b.rp, b.ci, crp, cci, g)
    sc_a = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, np.abs(b.val), crp, cci, np.abs(g))
    sc_b = oracle.grad_b(a.rp, a.ci, np.abs(a.val), b.rp, b.ci, crp, cci, np.abs(g))
    assert np.all(np.abs(ga - ref_a) <= RTOL * sc_a + 1e-30), np.max(np.abs(ga - ref_a) / np.maximum(sc_a, 1e-30))
    assert np.all(np.abs(gb - ref_b) <= RTOL * sc_b + 1e-30), np.max(np.abs(gb - ref_b) / np.maximum(sc_b, 1e-30))


@pytest.mark.parametrize("d", [7, 32, 100, 256])
def test_gradients_random(d):
    rng = np.random.default_rng(800 + d)
    n = 400
    a = random_csr(rng, n, n, 0.02, kind="normal", empty_rows=0.2, dense_rows=3)
    b = random_csr(rng, n, d, min(0.4, 8.0 / d + 0.02), kind="normal", empty_rows=0.2)
    note(f"gradients random n={n} d={d}")
    crp, cci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    g = rng.standard_normal(len(cci))
    g = g.astype(np.float32).astype(np.float64)
    ga, gb, C = _grads_gpu(a, b, g)
    assert np.array_equal(C.rowptr.cpu().numpy().astype(np.int64), crp)
    _check(a, b, ga, gb, crp, cci, g)
    # every work class and group width gives the same bits
    for tune in (dict(light_max_flops=1, wave_max_flops=4, split_flops=16), dict(group_lanes=4),
                 dict(group_lanes=64), dict(light_max_flops=1 << 30, wave_max_flops=1 << 30, split_flops=1 << 30)):
        ga2, gb2, _ = _grads_gpu(a, b, g, tuning=tune)
        assert np.array_equal(ga, ga2) and np.array_equal(gb, gb2), tune


@pytest.mark.parametrize("d", [5, 64, 256])
def test_backward_one_call(d):
    """tsspgemm_backward (one pass over A's rows writing dL/dA and the sampled
    G, one over A^T for dL/dB) against the separate calls (bit for bit: the
    same sums in the same order) and the oracle. A has dense columns, so
    A^T rows span several dL/dB chunks, and dense rows (workgroup and split
    rows of the forward plan)."""
    rng = np.random.default_rng(900 + d)
    n = 1500
    a0 = random_csr(rng, n, n, 0.004, kind="normal", empty_rows=0.1, dense_rows=2)
    pat = np.zeros((n, n), dtype=bool)
    pat[rows_of(a0.rp), a0.ci] = True
    pat[:, [7, 900]] = True  # two columns of n entries: A^T rows of 3 chunks
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(pat.sum(axis=1))
    ci = np.nonzero(pat)[1].astype(np.int32)
    a = synth.Csr(n, n, rp, ci, rng.standard_normal(len(ci)).astype(np.float32))
    b = random_csr(rng, n, d, min(0.5, 6.0 / d + 0.02), kind="normal", empty_rows=0.1)
    crp, cci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    g = rng.standard_normal(len(cci)).astype(np.float32).astype(np.float64)
    tss = _tss()
    for tune in (None, dict(light_max_flops=1, wave_max_flops=8, split_flops=64)):
        note(f"backward one call n={n} d={d} tuning={tune}")
        A, B = to_dev(a), to_dev(b)
        C, plan = tss.spgemm(A, B, tuning=tune, return_plan=True)
        G = C.with_vals(torch.from_numpy(g.astype(np.float32)).cuda())
        AT, perm = tss.transpose(A)
        ga, gb = tss.backward(plan, AT, perm, A, B, G)
        ga1 = tss.grad_a(plan, A, B, G)
        gb1 = tss.grad_b(plan, AT, perm, A, B, G)
        ga_only, _ = tss.backward(plan, None, None, A, B, G, need_b=False)
        _, gb_only = tss.backward(plan, AT, perm, A, B, G, need_a=False)
        torch.cuda.synchronize()
        assert torch.equal(ga, ga1) and torch.equal(gb, gb1)
        assert torch.equal(ga, ga_only) and torch.equal(gb, gb_only)
        _check(a, b, ga.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64), crp, cci, g)


def test_gradients_match_fp64_finite_differences():
    """Differentiable-layer workload at n = 2048 (R-MAT scale 11), d = 32, B 5%
    N(0,1), W N(0,1): GPU gradients against FP64 central differences of the
    oracle forward on 1024 coordinates of A and of B, and along a random
    direction."""
    a, b = synth.workload_embedding(scale=11, d=32, density=0.05)
    note(f"FD check n=2048 d=32 nnzA={a.nnz} nnzB={b.nnz}")
    crp, cci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    c = synth.Csr(a.nrows, b.ncols, crp.astype(np.int32), cci)
    w = synth.w_on_pattern(c, 5).astype(np.float64)
    ga, gb, _ = _grads_gpu(a, b, w)
    sc_a = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, np.abs(b.val), crp, cci, np.abs(w))
    sc_b = oracle.grad_b(a.rp, a.ci, np.abs(a.val), b.rp, b.ci, crp, cci, np.abs(w))
    av, bv = a.val.astype(np.float64), b.val.astype(np.float64)

    def loss(x, y):
        _, _, val = oracle.spgemm(a.rp, a.ci, x, b.rp, b.ci, y)
        return float(val @ w)

    h = 2.0**-10
    rng = np.random.default_rng(11)
    for p in rng.choice(a.nnz, size=min(1024, a.nnz), replace=False):
        e = np.zeros_like(av)
        e[p] = h
        fd = (loss(av + e, bv) - loss(av - e, bv)) / (2 * h)
        assert abs(ga[p] - fd) <= RTOL * sc_a[p] + 1e-9, (p, ga[p], fd)
    for q in rng.choice(b.nnz, size=min(1024, b.nnz), replace=False):
        e = np.zeros_like(bv)
        e[q] = h
        fd = (loss(av, bv + e) - loss(av, bv - e)) / (2 * h)
        assert abs(gb[q] - fd) <= RTOL * sc_b[q] + 1e-9, (q, gb[q], fd)
    u, v = rng.standard_normal(a.nnz), rng.standard_normal(b.nnz)
    fd = (loss(av + h * u, bv + h * v) - loss(av - h * u, bv - h * v)) / (2 * h)
    assert abs(fd - (ga @ u + gb @ v)) <= RTOL * (np.abs(u) @ sc_a + np.abs(v) @ sc_b)


def test_autograd_function():
    tss = _tss()
    a, b = synth.workload_embedding(scale=10, d=64, density=0.05)
    A, B = to_dev(a), to_dev(b)
    op = tss.TSSpGEMMOp(A, B)
    av = A.vals.clone().requires_grad_(True)
    bv = B.vals.clone().requires_grad_(True)
    c = op(av, bv)
    crp, cci, cval = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    assert np.array_equal(op.c_colidx.cpu().numpy(), cci)
    assert np.all(np.abs(c.detach().cpu().numpy() - cval) <= 1e-5 * oracle.spgemm(
        a.rp, a.ci, np.abs(a.val), b.rp, b.ci, np.abs(b.val))[2])
    w = torch.from_numpy(synth.w_on_pattern(synth.Csr(a.nrows, b.ncols, crp.astype(np.int32), cci), 3)).cuda()
    note("autograd backward")
    loss = (c * w).sum()
    loss.backward()
    G = op.c_pattern().with_vals(w)
    ga = tss.grad_a(op.plan, op.A.with_vals(av.detach()), op.B.with_vals(bv.detach()), G)
    AT, perm = op.transpose()
    gb = tss.grad_b(op.plan, AT, perm, op.A.with_vals(av.detach()), op.B.with_vals(bv.detach()), G)
    assert torch.equal(av.grad, ga) and torch.equal(bv.grad, gb)
    # a second step with new values reuses the plan
    with torch.no_grad():
        av2 = (av * 0.5).detach().requires_grad_(True)
    c2 = op(av2, bv)
    assert torch.allclose(c2, c.detach() * 0.5, rtol=1e-6, atol=0)


def test_embedding_scale20_sampled():
    """Full-size differentiable layer: R-MAT scale 20, d = 256, B 5% N(0,1):
    forward, dL/dA and dL/dB on sampled rows against the oracle."""
    tss = _tss()
    a, b = synth.workload_embedding(scale=20, d=256, density=0.05)
    note(f"embedding R-MAT 20 d=256 nnzA={a.nnz} nnzB={b.nnz}")
    A, B = to_dev(a), to_dev(b)
    op = tss.TSSpGEMMOp(A, B)
    av = A.vals.clone().requires_grad_(True)
    bv = B.vals.clone().requires_grad_(True)
    c = op(av, bv)
    crp = op.c_rowptr.cpu().numpy()
    cci = op.c_colidx.cpu().numpy()
    w = synth.w_on_pattern(synth.Csr(a.nrows, b.ncols, crp, cci), 7)
    (c * torch.from_numpy(w).cuda()).sum().backward()
    torch.cuda.synchronize()
    ga, gb = av.grad.cpu().numpy(), bv.grad.cpu().numpy()
    rng = np.random.default_rng(5)
    flops = oracle.row_flops(a.rp, a.ci, b.rp)
    rows = np.unique(np.concatenate([np.argsort(flops)[-8:], rng.choice(a.nrows, 300, replace=False)])).astype(np.int32)
    deg = np.diff(a.rp)
    krows = np.unique(np.concatenate([np.argsort(deg)[-8:], rng.choice(a.nrows, 300, replace=False)])).astype(np.int32)
    w64 = w.astype(np.float64)
    note("oracle dL/dA rows")
    ref = oracle.grad_a_rows(a.rp, a.ci, b.rp, b.ci, b.val, crp, cci, w64, rows)
    sc = oracle.grad_a_rows(a.rp, a.ci, b.rp, b.ci, np.abs(b.val), crp, cci, np.abs(w64), rows)
    sel = np.concatenate([np.arange(a.rp[i], a.rp[i + 1]) for i in rows])
    assert np.all(np.abs(ga[sel] - ref) <= RTOL * sc + 1e-30)
    note("oracle dL/dB rows")
    ref = oracle.grad_b_rows(a.rp, a.ci, a.val, b.rp, b.ci, crp, cci, w64, krows)
    sc = oracle.grad_b_rows(a.rp, a.ci, np.abs(a.val), b.rp, b.ci, crp, cci, np.abs(w64), krows)
    sel = np.concatenate([np.arange(b.rp[k], b.rp[k + 1]) for k in krows])
    assert np.all(np.abs(gb[sel] - ref) <= RTOL * sc + 1e-30)


def test_gradients_reject_masked_plan():
    """A forward product taken with a complement mask drops entries of pat(C)
    that the gradient formulas read, so the library refuses such a plan."""
    import paper_2408_11988_amd as tss

    rng = np.random.default_rng(77)
    n, d = 64, 16
    a = random_csr(rng, n, n, 0.1)
    b = random_csr(rng, n, d, 0.3)
    m = random_csr(rng, n, d, 0.2)
    A, B, M = to_dev(a), to_dev(b), to_dev(m, with_values=False)
    C, plan = tss.spgemm(A, B, mask=M, return_plan=True)
    G = C.with_vals(torch.ones_like(C.vals))
    with pytest.raises(tss.TSSpGEMMError) as e:
        tss.grad_a(plan, A, B, G)
    assert "mask" in str(e.value)


@pytest.mark.parametrize("d", [64, 256])
def test_numeric_repeats_record_b_row_bounds(d):
    """A plan whose numeric phase repeats records each A entry's B row bounds
    at its second numeric call and reads them from the third on (and in the
    backward). Every call, with new values of A and B on the same patterns,
    matches the oracle; the backward before and after the record is the
    same bit for bit (the same sums in the same order)."""
    rng = np.random.default_rng(1200 + d)
    n = 1500
    a = random_csr(rng, n, n, 0.006, kind="normal", empty_rows=0.1, dense_rows=2)
    b = random_csr(rng, n, d, min(0.5, 6.0 / d + 0.02), kind="normal", empty_rows=0.1)
    tss = _tss()
    A, B = to_dev(a), to_dev(b)
    C, plan = tss.spgemm(A, B, return_plan=True)  # symbolic + numeric call 1
    crp, cci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    g = rng.standard_normal(len(cci)).astype(np.float32)
    G = C.with_vals(torch.from_numpy(g).cuda())
    AT, perm = tss.transpose(A)
    ga0, gb0 = tss.backward(plan, AT, perm, A, B, G)
    torch.cuda.synchronize()
    ga0, gb0 = ga0.clone(), gb0.clone()
    for call in (2, 3, 4):
        av = rng.standard_normal(a.nnz).astype(np.float32)
        bv = rng.standard_normal(b.nnz).astype(np.float32)
        a2, b2 = a.with_values(av), b.with_values(bv)
        A2 = A.with_vals(torch.from_numpy(av).cuda())
        B2 = B.with_vals(torch.from_numpy(bv).cuda())
        ci = torch.empty(max(C.nnz, 1), dtype=torch.int32, device="cuda")
        cv = torch.empty(max(C.nnz, 1), dtype=torch.float32, device="cuda")
        note(f"numeric call {call} d={d}")
        tss.numeric(plan, A2, B2, ci, cv)
        torch.cuda.synchronize()
        compare_f32(a2, b2, tss.DeviceCsr(C.nrows, C.ncols, C.rowptr, ci[:C.nnz], cv[:C.nnz]), signed=True)
    ga1, gb1 = tss.backward(plan, AT, perm, A, B, G)
    torch.cuda.synchronize()
    assert torch.equal(ga0, ga1) and torch.equal(gb0, gb1)


def test_numeric_captured_in_graph_before_the_record():
    """A numeric call captured into a HIP graph as the plan's second call
    allocates nothing and records nothing (its kernels only run at replay):
    the next eager call records the B row bounds, and the graph's replays
    (new values copied into its inputs), the eager calls and the backward all
    match the oracle."""
    rng = np.random.default_rng(1300)
    n, d = 1500, 128
    a = random_csr(rng, n, n, 0.006, kind="normal", empty_rows=0.1, dense_rows=2)
    b = random_csr(rng, n, d, 0.08, kind="normal", empty_rows=0.1)
    tss = _tss()
    A, B = to_dev(a), to_dev(b)
    C, plan = tss.spgemm(A, B, return_plan=True)  # symbolic + numeric call 1
    A2 = A.with_vals(torch.from_numpy(a.val.copy()).cuda())
    B2 = B.with_vals(torch.from_numpy(b.val.copy()).cuda())
    gci = torch.empty(max(C.nnz, 1), dtype=torch.int32, device="cuda")
    gcv = torch.empty(max(C.nnz, 1), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    note("capture numeric call 2")
    with torch.cuda.graph(graph):
        tss.numeric(plan, A2, B2, gci, gcv)
    torch.cuda.synchronize()
    for step in range(4):
        av = rng.standard_normal(a.nnz).astype(np.float32)
        bv = rng.standard_normal(b.nnz).astype(np.float32)
        a2, b2 = a.with_values(av), b.with_values(bv)
        A2.vals.copy_(torch.from_numpy(av))
        B2.vals.copy_(torch.from_numpy(bv))
        note(f"replay {step}")
        graph.replay()
        torch.cuda.synchronize()
        compare_f32(a2, b2, tss.DeviceCsr(C.nrows, C.ncols, C.rowptr, gci[:C.nnz], gcv[:C.nnz]), signed=True)
        # eager calls between the replays: the first records the bounds, the
        # rest read them
        ci = torch.empty_like(gci)
        cv = torch.empty_like(gcv)
        note(f"eager numeric after replay {step}")
        tss.numeric(plan, A2, B2, ci, cv)
        torch.cuda.synchronize()
        compare_f32(a2, b2, tss.DeviceCsr(C.nrows, C.ncols, C.rowptr, ci[:C.nnz], cv[:C.nnz]), signed=True)
