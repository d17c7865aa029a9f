"""GPU parity of the plain TS-SpGEMM (symbolic + numeric) against the oracle.

Structure and integer / Boolean values are compared bit for bit; FP32
plus-times values within relative 1e-5 of the FP64 oracle (tests/gpu_util.py).
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import random_csr
from tests.gpu_util import compare_bool, compare_f32, compare_int, note, require_gpu, same_structure_close_values, to_dev

pytestmark = pytest.mark.gpu

D_VALUES = [1, 5, 31, 32, 33, 64, 100, 128, 255, 256, 512, 1000, 1024]
WIDE_D = [1025, 2048, 5000, 65536]  # past the dense accumulator: the hash accumulator


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    import paper_2408_11988_amd as tss

    note(f"library {tss.version()}")


def _tss():
    import paper_2408_11988_amd as tss

    return tss


ACCS = ["lds", "hash"]
# thresholds that send rows of these small cases to every work class
ALL_CLASSES = dict(light_max_flops=16, wave_max_flops=64, split_flops=256)


@pytest.mark.parametrize("classes", ["default", "all", "all_flat", "all_vec4"])
@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("d", D_VALUES)
def test_plus_times_random(d, acc, classes):
    rng = np.random.default_rng(1000 + d)
    n = 300
    a = random_csr(rng, n, n, 0.03, empty_rows=0.2, dense_rows=2)
    b = random_csr(rng, n, d, min(0.5, 6.0 / d + 0.02), empty_rows=0.1)
    tun = dict(accumulator=acc, **(ALL_CLASSES if classes.startswith("all") else {}))
    if classes == "all_flat":
        tun["products"] = "flat"
    if classes == "all_vec4":
        tun["products"] = "vec4"
    note(f"plus_times random n={n} d={d} nnzA={a.nnz} nnzB={b.nnz} tuning={tun}")
    C, plan = _tss().spgemm(to_dev(a), to_dev(b), tuning=tun, return_plan=True)
    torch.cuda.synchronize()
    frac = compare_f32(a, b, C)
    assert frac > 0.999
    # the dense A rows fill their patterns early: the symbolic pass counts the
    # rest of their products from B's row lengths
    assert plan.stats()["flops"] == int(oracle.row_flops(a.rp, a.ci, b.rp).sum())


@pytest.mark.parametrize("d", WIDE_D)
def test_plus_times_wide(d):
    """d > 1024 (hash accumulator chosen automatically): a few dense A rows
    make rows with hundreds to thousands of outputs (split rows, or the
    long-row kernel; the d-bit bitmap in the symbolic pass), the rest stay in
    the LDS tables."""
    rng = np.random.default_rng(1500 + d)
    n = 400
    a = random_csr(rng, n, n, 0.02, empty_rows=0.2, dense_rows=3)
    b = random_csr(rng, n, d, min(0.3, 12.0 / d), empty_rows=0.1)
    note(f"plus_times wide n={n} d={d} nnzA={a.nnz} nnzB={b.nnz}")
    C, plan = _tss().spgemm(to_dev(a), to_dev(b), return_plan=True)
    torch.cuda.synchronize()
    frac = compare_f32(a, b, C)
    assert frac > 0.999
    assert plan.stats()["flops"] == int(oracle.row_flops(a.rp, a.ci, b.rp).sum())
    cnt = np.diff(C.rowptr.cpu().numpy())
    assert cnt.max() > 512 and 0 < np.median(cnt[cnt > 0]) <= 512  # both numeric kernels ran


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("d", [7, 64, 300])
def test_plus_times_signed(d, acc):
    rng = np.random.default_rng(2000 + d)
    n = 257
    a = random_csr(rng, n, n, 0.05, kind="normal", empty_rows=0.1, dense_rows=1)
    b = random_csr(rng, n, d, 0.2, kind="normal")
    note(f"plus_times signed n={n} d={d} acc={acc}")
    C = _tss().spgemm(to_dev(a), to_dev(b), tuning=dict(accumulator=acc, **ALL_CLASSES))
    torch.cuda.synchronize()
    compare_f32(a, b, C, signed=True)


@pytest.mark.parametrize("d,acc", [(d, acc) for d in (3, 64, 129, 1024, 3000) for acc in ACCS
                                   if d <= 1024 or acc == "hash"])  # the LDS strip needs d <= 1024
def test_int32_exact(d, acc):
    rng = np.random.default_rng(3000 + d)
    n = 200
    a = random_csr(rng, n, n, 0.05, kind="int", dense_rows=1)
    b = random_csr(rng, n, d, min(0.1, 20.0 / d), kind="int")
    note(f"int32 n={n} d={d} acc={acc}")
    for tun in (dict(accumulator=acc), dict(accumulator=acc, **ALL_CLASSES),
                dict(accumulator=acc, products="vec4", **ALL_CLASSES)):
        C = _tss().spgemm(to_dev(a, dtype=torch.int32), to_dev(b, dtype=torch.int32), semiring="plus_times_i32",
                          tuning=tun)
        torch.cuda.synchronize()
        compare_int(a, b, C)


@pytest.mark.parametrize("d", [1, 40, 64, 512, 1024, 2000])
def test_or_and_and_masks(d):
    rng = np.random.default_rng(4000 + d)
    n = 220
    a = random_csr(rng, n, n, 0.04, dense_rows=1)
    b = random_csr(rng, n, d, 0.05)
    m = random_csr(rng, n, d, 0.3)
    tss = _tss()
    note(f"or_and n={n} d={d}")
    A, B = to_dev(a, with_values=False), to_dev(b, with_values=False)
    C = tss.spgemm(A, B, semiring="or_and")
    torch.cuda.synchronize()
    compare_bool(a, b, C)
    note(f"or_and csr mask n={n} d={d}")
    M = to_dev(m, with_values=False)
    C = tss.spgemm(A, B, semiring="or_and", mask=M)
    compare_bool(a, b, C, mask=m)
    note(f"masked_bool csr mask n={n} d={d}")
    C = tss.masked_bool(A, B, M)
    compare_bool(a, b, C, mask=m)
    # the same mask as a bitmap
    wp = tss.bitmap_words(d)
    bits = np.zeros((n, wp), dtype=np.uint32)
    rows = np.repeat(np.arange(n), np.diff(m.rp))
    np.bitwise_or.at(bits, (rows, m.ci // 32), (np.uint32(1) << (m.ci % 32).astype(np.uint32)))
    note(f"masked_bool bitmap mask n={n} d={d}")
    C = tss.masked_bool(A, B, torch.from_numpy(bits.view(np.int32)).cuda())
    compare_bool(a, b, C, mask=m)
    # plus-times with a complement mask drops the masked entries, values unchanged
    a2 = synth.Csr(n, n, a.rp, a.ci, rng.random(a.nnz).astype(np.float32))
    b2 = synth.Csr(n, d, b.rp, b.ci, rng.random(b.nnz).astype(np.float32))
    rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci, m.rp, m.ci)
    frp, fci, fval = oracle.spgemm(a2.rp, a2.ci, a2.val, b2.rp, b2.ci, b2.val)
    full = {(i, j): v for i in range(n) for j, v in zip(fci[frp[i]:frp[i + 1]], fval[frp[i]:frp[i + 1]])}
    for acc in ACCS if d <= 1024 else ["hash"]:
        note(f"plus_times csr mask n={n} d={d} acc={acc}")
        C = tss.spgemm(to_dev(a2), to_dev(b2), mask=M, tuning=dict(accumulator=acc, **ALL_CLASSES))
        g_rp, g_ci, g_val = C.to_host()
        assert np.array_equal(g_rp.astype(np.int64), rp) and np.array_equal(g_ci, ci)
        ref = np.array([full[(i, j)] for i in range(n) for j in g_ci[g_rp[i]:g_rp[i + 1]]])
        assert np.all(np.abs(g_val - ref) <= 1e-5 * np.abs(ref))


def test_modes_and_tuning_do_not_change_results():
    """Wavefront, workgroup and split rows, and every group width, give the
    same structure and values within the tolerance. Each setting sums in
    FP64 in an order of its own, so a value may round to a neighbouring FP32
    in rare cases; nearly all values are bit-identical."""
    rng = np.random.default_rng(5)
    n, d = 600, 128
    a = random_csr(rng, n, n, 0.02, dense_rows=6)
    b = random_csr(rng, n, d, 0.15)
    tss = _tss()
    A, B = to_dev(a), to_dev(b)
    note("tuning reference run")
    ref, plan = tss.spgemm(A, B, return_plan=True)
    compare_f32(a, b, ref)
    ref_h = ref.to_host()
    configs = [dict(group_lanes=g) for g in (4, 8, 16, 32, 64)]
    configs += [dict(group_lanes=g, products=pl) for g in (8, 32, 64) for pl in ("rows", "flat", "vec4")]
    configs += [dict(group_lanes=g, products="vec4") for g in (4, 16)]
    configs += [dict(light_max_flops=200, wave_max_flops=260, split_flops=1000, products="vec4")]
    configs += [dict(light_max_flops=1, wave_max_flops=16, split_flops=64),
                dict(light_max_flops=1, wave_max_flops=1, split_flops=1),
                dict(light_max_flops=200, wave_max_flops=260, split_flops=1000),
                dict(light_max_flops=200, wave_max_flops=260, split_flops=1000, products="flat"),
                dict(light_max_flops=200, wave_max_flops=260, split_flops=1000, products="rows"),
                dict(light_max_flops=1 << 30, wave_max_flops=1 << 30, split_flops=1 << 30),
                dict(wave_max_flops=500, split_flops=100000, sym_split_nnz=3), dict(sym_split_nnz=1)]
    for cfg in configs:
        note(f"tuning {cfg}")
        C, p = tss.spgemm(A, B, tuning=cfg, return_plan=True)
        assert same_structure_close_values(ref, C) > 0.999, cfg
        st = p.stats()
        assert st["flops"] == plan.stats()["flops"]
    # the hash accumulator: same structure, values within the tolerance (its
    # sums may run in another order)
    note("hash accumulator")
    C = tss.spgemm(A, B, tuning=dict(accumulator="hash"))
    got = C.to_host()
    assert np.array_equal(ref_h[0], got[0]) and np.array_equal(ref_h[1], got[1])
    compare_f32(a, b, C)
    # rows here have ~230 +- 70 products, the dense rows ~11500: all four classes occur
    st = tss.spgemm(A, B, tuning=dict(light_max_flops=200, wave_max_flops=260, split_flops=1000),
                    return_plan=True)[1].stats()
    assert st["split_rows"] > 0 and st["block_rows"] > 0 and st["wave_rows"] > 0 and st["light_rows"] > 0


def test_plan_reuse_and_determinism():
    a, b = synth.workload_er_small()
    tss = _tss()
    A, B = to_dev(a), to_dev(b)
    note("ER 4096 x 64 (config 1)")
    C1, plan = tss.spgemm(A, B, return_plan=True)
    torch.cuda.synchronize()
    frac = compare_f32(a, b, C1)
    assert frac > 0.999
    assert plan.stats()["flops"] == int(oracle.row_flops(a.rp, a.ci, b.rp).sum())
    note("plan reuse, new values")
    b2 = b.with_values((b.val * 0.5 + 0.25).astype(np.float32))
    B2 = to_dev(b2)
    C2 = tss.spgemm(A, B2, plan=plan)
    compare_f32(a, b2, C2)
    c_ci = torch.empty_like(C2.colidx)
    c_v = torch.empty_like(C2.vals)
    tss.numeric(plan, A, B2, c_ci, c_v)
    assert torch.equal(c_ci, C2.colidx) and torch.equal(c_v, C2.vals)


@pytest.mark.parametrize("acc", ["auto"] + ACCS)
def test_rmat_scale16_full(acc):
    a, b = synth.workload_rmat_plain(scale=16, d=128)
    tss = _tss()
    note(f"R-MAT 16 d=128 nnzA={a.nnz} nnzB={b.nnz} acc={acc}")
    C, plan = tss.spgemm(to_dev(a), to_dev(b), return_plan=True, tuning=dict(accumulator=acc))
    torch.cuda.synchronize()
    frac = compare_f32(a, b, C, threads=8)
    assert frac > 0.999
    st = plan.stats()
    assert st["nnz"] == C.nnz


@pytest.fixture(scope="module")
def rmat20_d128():
    """The full-size plain workload (R-MAT scale 20, d = 128) and the oracle's
    product over every row, computed once for the module."""
    a, b = synth.workload_rmat_plain(scale=20, d=128)
    note(f"oracle on every row of R-MAT 20 d=128 (nnzA={a.nnz} nnzB={b.nnz})")
    ref = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, threads=16)
    return a, b, ref


@pytest.mark.timeout(300)
@pytest.mark.parametrize("acc", ["auto"] + ACCS)
def test_rmat_scale20_d128_full(acc, rmat20_d128):
    """Full-size plain workload (R-MAT scale 20, d = 128): every row against the
    oracle (structure bit for bit, values within the tolerance), plus the
    per-row invariants. "auto" is the configuration the benchmark times."""
    a, b, ref = rmat20_d128
    tss = _tss()
    note(f"R-MAT 20 d=128 nnzA={a.nnz} nnzB={b.nnz} acc={acc}")
    C, plan = tss.spgemm(to_dev(a), to_dev(b), return_plan=True, tuning=dict(accumulator=acc))
    torch.cuda.synchronize()
    g_rp, g_ci, _ = C.to_host()
    flops = oracle.row_flops(a.rp, a.ci, b.rp)
    assert plan.stats()["flops"] == int(flops.sum())
    cnt = np.diff(g_rp.astype(np.int64))
    assert np.all(cnt <= np.minimum(128, flops)) and np.all((cnt == 0) == (flops == 0))
    note(f"compare every row with the oracle, acc={acc}")
    frac = compare_f32(a, b, C, ref=ref)
    assert frac > 0.999


def test_edge_cases():
    tss = _tss()
    rng = np.random.default_rng(9)
    # no rows
    z = synth.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    zb = synth.Csr(0, 8, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    note("n = 0")
    C = tss.spgemm(to_dev(z), to_dev(zb))
    assert C.nnz == 0 and C.rowptr.cpu().tolist() == [0]
    # empty A, empty B
    n, d = 100, 64
    ea = synth.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    b = random_csr(rng, n, d, 0.1)
    note("empty A")
    C = tss.spgemm(to_dev(ea), to_dev(b))
    assert C.nnz == 0 and int(C.rowptr.cpu()[-1]) == 0
    eb = synth.Csr(n, d, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    a = random_csr(rng, n, n, 0.1)
    note("empty B")
    C = tss.spgemm(to_dev(a), to_dev(eb))
    assert C.nnz == 0
    # identity
    eye = synth.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    note("identity")
    C = tss.spgemm(to_dev(eye), to_dev(b))
    r, c, v = C.to_host()
    assert np.array_equal(r, b.rp) and np.array_equal(c, b.ci) and np.array_equal(v, b.val)


@pytest.mark.parametrize("d,tun", [(2048, None), (64, {"accumulator": "hash"})])
def test_edge_cases_hash(d, tun):
    """The hash accumulator's edge cases: no rows, empty A, empty B, the
    identity, and one row of exactly 512 products (the least split row)
    beside rows of 511 and 513."""
    tss = _tss()
    rng = np.random.default_rng(19)
    z = synth.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    zb = synth.Csr(0, d, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    note(f"hash n = 0, d = {d}")
    C = tss.spgemm(to_dev(z), to_dev(zb), tuning=tun)
    assert C.nnz == 0 and C.rowptr.cpu().tolist() == [0]
    n = 100
    ea = synth.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    b = random_csr(rng, n, d, min(0.1, 8.0 / d))
    note("hash empty A")
    C = tss.spgemm(to_dev(ea), to_dev(b), tuning=tun)
    assert C.nnz == 0 and int(C.rowptr.cpu()[-1]) == 0
    eb = synth.Csr(n, d, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    a = random_csr(rng, n, n, 0.1)
    note("hash empty B")
    C = tss.spgemm(to_dev(a), to_dev(eb), tuning=tun)
    assert C.nnz == 0
    eye = synth.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    note("hash identity")
    C = tss.spgemm(to_dev(eye), to_dev(b), tuning=tun)
    r, c, v = C.to_host()
    assert np.array_equal(r, b.rp) and np.array_equal(c, b.ci) and np.array_equal(v, b.val)
    # B rows of 8 entries each; A rows of 63, 64 and 65 entries: 504, 512, 520
    # products (only the last two are split rows)
    nb = 300
    bci = np.concatenate([np.sort(rng.choice(d, 8, replace=False)) for _ in range(nb)]).astype(np.int32)
    bb = synth.Csr(nb, d, np.arange(0, 8 * nb + 1, 8, dtype=np.int32), bci, rng.random(8 * nb).astype(np.float32))
    rows = [np.sort(rng.choice(nb, m, replace=False)) for m in (63, 64, 65)] + [np.zeros(0, np.int64)] * (nb - 3)
    arp = np.concatenate([[0], np.cumsum([len(x) for x in rows])]).astype(np.int32)
    ab = synth.Csr(nb, nb, arp, np.concatenate(rows).astype(np.int32), rng.random(int(arp[-1])).astype(np.float32))
    note("hash rows at the split threshold")
    C, plan = tss.spgemm(to_dev(ab), to_dev(bb), tuning=tun, return_plan=True)
    torch.cuda.synchronize()
    assert plan.stats()["split_rows"] == 2
    assert compare_f32(ab, bb, C) > 0.999


def test_error_paths_on_device():
    tss = _tss()
    from paper_2408_11988_amd import _lib

    rng = np.random.default_rng(10)
    n = 64
    a = random_csr(rng, n, n, 0.1)
    big = random_csr(rng, n, 2048, 0.01)
    note("d = 2048 with the LDS strip forced")
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.spgemm(to_dev(a), to_dev(big), tuning=dict(accumulator="lds"))
    assert e.value.code == _lib.ERR_UNSUPPORTED
    huge = synth.Csr(n, 70000, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    note("d = 70000: beyond the hash accumulator")
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.spgemm(to_dev(a), to_dev(huge))
    assert e.value.code == _lib.ERR_UNSUPPORTED
    note("gradients of a hash plan")
    C, plan = tss.spgemm(to_dev(a), to_dev(big), return_plan=True)
    with pytest.raises(_lib.TSSpGEMMError) as e:
        tss.grad_a(plan, to_dev(a), to_dev(big), C.with_vals(torch.ones_like(C.vals)))
    assert e.value.code == _lib.ERR_UNSUPPORTED
    b = random_csr(rng, n, 32, 0.3)
    A, B = to_dev(a, with_values=False), to_dev(b, with_values=False)
    full = tss.masked_bool(A, B)
    note("masked_bool capacity too small")
    import ctypes

    rp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.empty(4, dtype=torch.int32, device="cuda")
    nnz = ctypes.c_int64(0)
    da, db = A.desc(), B.desc()
    rc = _lib.load().tsspgemm_masked_bool(ctypes.byref(da), ctypes.byref(db), None, ctypes.c_void_p(rp.data_ptr()),
                                          ctypes.c_void_p(ci.data_ptr()), 4, ctypes.byref(nnz),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.ERR_CAPACITY and nnz.value == full.nnz
    assert torch.equal(rp, full.rowptr)
    # validation mode catches an unsorted row before any other kernel reads it
    bad = synth.Csr(n, n, a.rp.copy(), a.ci.copy(), a.val)
    r0 = int(np.argmax(np.diff(a.rp) >= 2))
    bad.ci[a.rp[r0]], bad.ci[a.rp[r0] + 1] = a.ci[a.rp[r0] + 1], a.ci[a.rp[r0]]
    os.environ["TSSPGEMM_VALIDATE"] = "1"
    try:
        note("validation: unsorted row")
        with pytest.raises(_lib.TSSpGEMMError) as e:
            tss.spgemm(to_dev(bad), to_dev(b))
        assert e.value.code == _lib.ERR_MALFORMED
        oob = synth.Csr(n, 32, b.rp.copy(), b.ci.copy(), b.val)
        oob.ci[-1] = 40  # column outside [0, d)
        note("validation: column out of range")
        with pytest.raises(_lib.TSSpGEMMError) as e:
            tss.spgemm(to_dev(a), to_dev(oob))
        assert e.value.code == _lib.ERR_MALFORMED
        note("validation: good input passes")
        compare_f32(a, b, tss.spgemm(to_dev(a), to_dev(b)))
    finally:
        del os.environ["TSSPGEMM_VALIDATE"]


@pytest.mark.parametrize("d", [2048, 9000])
def test_hash_split_rows(d, monkeypatch):
    """Hash accumulator on a power-law A: hub rows are split into chunks of A
    entries (several chunks each). At d = 2048 they sum in LDS first, at
    d = 9000 the widest go straight to global accumulators. The split-slot
    bound is then forced down (rows past it take the one-wavefront path) and
    to zero; the structure must not change and the values stay within the
    tolerance. Also the integer semiring (exact) and OR-AND with a mask."""
    tss = _tss()
    g = synth.rmat(11, 16, 6100 + d)
    a = g.with_values(synth.values(g, "uniform", 6101, synth.S_AVAL))
    b = synth.b_poisson(a.nrows, d, 40.0, 6102 + d)
    b = b.with_values(synth.values(b, "uniform", 6103, synth.S_BVAL))
    flops = oracle.row_flops(a.rp, a.ci, b.rp)
    assert np.max(np.diff(a.rp)) > 512 and np.sum(flops > 2048) > 8  # split rows of several chunks
    ref = None
    for cap in (None, "3", "0"):
        if cap is None:
            monkeypatch.delenv("TSSPGEMM_HASH_SPLIT_CAP", raising=False)
        else:
            monkeypatch.setenv("TSSPGEMM_HASH_SPLIT_CAP", cap)
        note(f"hash split rows n={a.nrows} nnzA={a.nnz} d={d} split cap={cap}")
        C, plan = tss.spgemm(to_dev(a), to_dev(b), return_plan=True)
        torch.cuda.synchronize()
        split = plan.stats()["split_rows"]
        want = {None: int(np.sum(flops >= 512)), "3": 3, "0": 0}[cap]  # split rows: 512 products or more
        assert split == want, (split, want)
        frac = compare_f32(a, b, C, threads=8)
        assert frac > 0.999
        g_rp, g_ci, _ = C.to_host()
        if ref is None:
            ref = (g_rp, g_ci)
        assert np.array_equal(g_rp, ref[0]) and np.array_equal(g_ci, ref[1])
        if cap is None:
            cnt = np.diff(g_rp.astype(np.int64))
            assert cnt[flops > 2048].max() > (4096 if d > 4096 else 512)
    monkeypatch.delenv("TSSPGEMM_HASH_SPLIT_CAP", raising=False)
    ai = synth.Csr(a.nrows, a.ncols, a.rp, a.ci, (np.arange(a.nnz) % 7 - 3).astype(np.int32))
    bi = synth.Csr(b.nrows, b.ncols, b.rp, b.ci, (np.arange(b.nnz) % 5 - 2).astype(np.int32))
    note(f"hash split rows int32 d={d}")
    C = tss.spgemm(to_dev(ai, dtype=torch.int32), to_dev(bi, dtype=torch.int32), semiring="plus_times_i32")
    torch.cuda.synchronize()
    compare_int(ai, bi, C)
    rng = np.random.default_rng(6104 + d)
    m = random_csr(rng, a.nrows, d, 0.2)
    M = to_dev(m, with_values=False)
    note(f"hash split rows or_and with a csr mask d={d}")
    C = tss.spgemm(to_dev(a, with_values=False), to_dev(b, with_values=False), semiring="or_and", mask=M)
    torch.cuda.synchronize()
    compare_bool(a, b, C, mask=m)
    note(f"hash split rows plus_times with a csr mask d={d}")
    C = tss.spgemm(to_dev(a), to_dev(b), mask=M)
    g_rp, g_ci, g_val = C.to_host()
    rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci, m.rp, m.ci)
    assert np.array_equal(g_rp.astype(np.int64), rp) and np.array_equal(g_ci, ci)
    frp, fci, fval = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, threads=8)
    fkey = np.repeat(np.arange(a.nrows, dtype=np.int64), np.diff(frp)) * d + fci
    gkey = np.repeat(np.arange(a.nrows, dtype=np.int64), np.diff(g_rp.astype(np.int64))) * d + g_ci
    ref = fval[np.searchsorted(fkey, gkey)]
    assert np.all(np.abs(g_val - ref) <= 1e-5 * np.abs(ref))
    note(f"hash split rows plus_times with the same mask as a bitmap d={d}")
    wp = tss.bitmap_words(d)
    bits = np.zeros((a.nrows, wp), dtype=np.uint32)
    mrows = np.repeat(np.arange(a.nrows), np.diff(m.rp))
    np.bitwise_or.at(bits, (mrows, m.ci // 32), (np.uint32(1) << (m.ci % 32).astype(np.uint32)))
    C2 = tss.spgemm(to_dev(a), to_dev(b), mask=torch.from_numpy(bits.view(np.int32)).cuda())
    r_rp, r_ci, r_val = C2.to_host()
    assert np.array_equal(r_rp, g_rp) and np.array_equal(r_ci, g_ci)
    assert np.all(np.abs(r_val - ref) <= 1e-5 * np.abs(ref))


def test_hash_plan_reuse_across_shapes():
    """One plan object through hash-accumulator products of different shapes
    and widths (its split, window and class buffers grow or are reused),
    then back to the first: every result against the oracle, the last one
    bit-identical in structure to the first."""
    tss = _tss()
    plan = None
    first = None
    for scale, d, lam, seed in ((10, 2048, 30.0, 6200), (11, 9000, 40.0, 6201), (9, 1500, 20.0, 6202),
                                (10, 2048, 30.0, 6200)):
        g = synth.rmat(scale, 16, seed)
        a = g.with_values(synth.values(g, "uniform", seed, synth.S_AVAL))
        b = synth.b_poisson(a.nrows, d, lam, seed + 1)
        b = b.with_values(synth.values(b, "uniform", seed + 1, synth.S_BVAL))
        note(f"hash plan reuse: R-MAT {scale} d={d}")
        C, plan = tss.spgemm(to_dev(a), to_dev(b), plan=plan, return_plan=True)
        torch.cuda.synchronize()
        assert plan.stats()["split_rows"] > 0
        assert compare_f32(a, b, C, threads=8) > 0.999
        rp, ci, _ = C.to_host()
        if first is None:
            first = (rp, ci)
        elif (scale, d) == (10, 2048):
            assert np.array_equal(rp, first[0]) and np.array_equal(ci, first[1])


@pytest.mark.parametrize("d", [2048, 65536])
def test_wide_d_rmat18_full(d):
    """The varying-d benchmark workload past d = 1024 (R-MAT scale 18, B with
    Poisson(25.6) entries per row; hash accumulator, split hub rows): every
    row checked for the invariants and against the oracle."""
    a, b = synth.workload_wide_d(d)
    tss = _tss()
    note(f"R-MAT 18 d={d} nnzA={a.nnz} nnzB={b.nnz}")
    C, plan = tss.spgemm(to_dev(a), to_dev(b), return_plan=True)
    torch.cuda.synchronize()
    g_rp, g_ci, _ = C.to_host()
    flops = oracle.row_flops(a.rp, a.ci, b.rp)
    assert plan.stats()["flops"] == int(flops.sum()) and plan.stats()["split_rows"] > 0
    cnt = np.diff(g_rp.astype(np.int64))
    assert np.all(cnt <= np.minimum(d, flops)) and np.all((cnt == 0) == (flops == 0))
    rows = np.repeat(np.arange(a.nrows), cnt)
    key = rows * d + g_ci.astype(np.int64)
    assert np.all(np.diff(key) > 0) and g_ci.min() >= 0 and g_ci.max() < d
    note(f"oracle on every row, d={d}")
    frac = compare_f32(a, b, C, threads=16)
    assert frac > 0.999
