"""Batched TS-SpGEMM: parity of every instance with the oracle, the same
structure and values within the tolerance as the plain call, HIP-graph
replays (bit-identical to the eager run), and the autotuner (whose choices
must not change the structure, nor the values beyond the tolerance)."""
import json

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import random_csr
from tests.gpu_util import compare_f32, note, require_gpu, same_structure_close_values, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _instances(seed=0):
    rng = np.random.default_rng(seed)
    out = []
    shapes = [(300, 64, 0.03, 0.1), (1, 5, 1.0, 0.5), (2000, 128, 0.004, 0.2), (0, 16, 0, 0), (500, 1024, 0.01, 0.01),
              (700, 33, 0.02, 0.3), (400, 1, 0.05, 0.5), (900, 200, 0.006, 0.05)]
    for n, d, pa, pb in shapes:
        if n == 0:
            a = synth.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
            b = synth.Csr(0, d, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
        else:
            a = random_csr(rng, n, n, pa, empty_rows=0.2, dense_rows=1 if n > 10 else 0)
            b = random_csr(rng, n, d, pb, empty_rows=0.1)
        out.append((a, b))
    # an instance whose A is empty
    b = random_csr(rng, 50, 40, 0.2)
    out.append((synth.Csr(50, 50, np.zeros(51, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)), b))
    return out


def _same(c1, c2):
    """The batched and the plain result of one instance: identical structure,
    values within the tolerance of each other (both are FP64 sums rounded
    once; a different order of addition may round to a neighbouring FP32)."""
    same_structure_close_values(c1, c2)


@pytest.mark.parametrize("tuned", [False, True])
def test_batched_matches_plain_and_oracle(tuned):
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd.batched import Batched

    host = _instances()
    pairs = [(to_dev(a), to_dev(b)) for a, b in host]
    tunings = None
    if tuned:  # forces every work class somewhere in the batch
        tunings = [dict(group_lanes=16, light_max_flops=64, wave_max_flops=512, split_flops=2048) for _ in host]
        tunings[0]["products"] = "flat"  # each tuned instance keeps its own layout: one flat, two in
        tunings[2]["products"] = "vec4"  # 4-entry chunks, the rest per B row
        tunings[6]["products"] = "vec4"
    note(f"batched {len(pairs)} instances tuned={tuned}")
    bt = Batched(pairs, tunings)
    bt.run()
    torch.cuda.synchronize()
    outs = bt.outputs()
    assert bt.c_offsets[-1].item() == bt.pool
    for t, ((a, b), (A, B), C) in enumerate(zip(host, pairs, outs)):
        plain = tss.spgemm(A, B, tuning=tunings[t] if tunings else dict(group_lanes=bt_group_lanes(pairs)))
        _same(C, plain)
        if a.nrows:
            compare_f32(a, b, C)
        assert bt.flops()[t] == int(oracle.row_flops(a.rp, a.ci, b.rp).sum()) if a.nrows else bt.flops()[t] == 0


def bt_group_lanes(pairs):
    """Group width the batch picks without tunings: from the mean B row length
    over all instances."""
    nn = sum(B.nrows for _, B in pairs)
    nz = sum(B.nnz for _, B in pairs)
    mean = nz / nn if nn else 0
    gl = 8
    while gl < 64 and gl < mean:
        gl *= 2
    return gl


def test_symbolic_split_size_is_the_batchs():
    """The symbolic split size of a batch is its first tuning's, for every
    instance: the item list is sized with it even when the other tunings
    name a far larger one (rows of hundreds of A entries cut in 40-entry
    chunks)."""
    from paper_2408_11988_amd.batched import Batched

    rng = np.random.default_rng(77)
    host = []
    for n, d in ((600, 64), (800, 128), (500, 32)):
        a = random_csr(rng, n, n, 0.01, empty_rows=0.1, dense_rows=4)
        b = random_csr(rng, n, d, 0.1, empty_rows=0.1)
        host.append((a, b))
    assert max(np.diff(a.rp).max() for a, _ in host) > 200
    pairs = [(to_dev(a), to_dev(b)) for a, b in host]
    tunings = [dict(sym_split_nnz=40)] + [dict(sym_split_nnz=1 << 20) for _ in host[1:]]
    note("batched with a 40-entry symbolic split from the first tuning")
    bt = Batched(pairs, tunings)
    bt.run()
    torch.cuda.synchronize()
    for (a, b), C in zip(host, bt.outputs()):
        compare_f32(a, b, C)


def test_graph_replays():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd.batched import Batched

    host = _instances(1)
    pairs = [(to_dev(a), to_dev(b)) for a, b in host]
    tun = [dict(group_lanes=32) for _ in host]
    bt = Batched(pairs, tun)
    bt.run()
    torch.cuda.synchronize()
    eager = [tuple(x.copy() for x in c.to_host()) for c in bt.outputs()]
    note("capture")
    bt.capture()
    rng = np.random.default_rng(3)
    for rep in range(4):
        # unrelated eager work and a synchronisation between replays
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()
        note(f"replay {rep}")
        bt.replay()
        torch.cuda.synchronize()
        for e, c in zip(eager, bt.outputs()):
            for u, v in zip(e, c.to_host()):
                assert np.array_equal(u, v)
    # new B values (same buffers): a replay recomputes them
    for (_, B), (a, b) in zip(pairs, host):
        if B.nnz:
            B.vals.copy_(torch.from_numpy(rng.random(B.nnz).astype(np.float32)))
    bt.replay()
    torch.cuda.synchronize()
    for t, ((A, B), C) in enumerate(zip(pairs, bt.outputs())):
        _same(C, tss.spgemm(A, B, tuning=tun[t]))


@pytest.mark.timeout(600)
def test_batched_workload_64_instances():
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd.batched import Batched

    params = synth.batched_params()
    host = [synth.batched_instance(p) for p in params]
    note(f"64-instance workload: sum n = {sum(a.nrows for a, _ in host)}, sum nnzA = {sum(a.nnz for a, _ in host)}")
    pairs = [(to_dev(a), to_dev(b)) for a, b in host]
    bt = Batched(pairs)
    bt.run()
    torch.cuda.synchronize()
    outs = bt.outputs()
    # every instance against the oracle, element by element
    equal = total = 0
    for t, ((a, b), C) in enumerate(zip(host, outs)):
        note(f"oracle on instance {t}: n={a.nrows} d={b.ncols} nnzA={a.nnz} nnzB={b.nnz}")
        frac = compare_f32(a, b, C, threads=16)
        equal += frac * C.nnz
        total += C.nnz
    assert equal > 0.999 * total  # values equal to the oracle rounded to FP32
    # and, as an extra check, against the plain call of each instance
    gl = bt_group_lanes(pairs)
    for (A, B), C in zip(pairs, outs):
        _same(C, tss.spgemm(A, B, tuning=dict(group_lanes=gl)))


def test_autotuner_does_not_change_results(tmp_path):
    import paper_2408_11988_amd as tss
    from paper_2408_11988_amd.autotune import Autotuner

    a, b = synth.workload_rmat_plain(scale=14, d=64)
    A, B = to_dev(a), to_dev(b)
    path = tmp_path / "tune.json"
    at = Autotuner(str(path))
    note("autotune R-MAT 14")
    best = at.tune(A, B, reps=2)
    at.save()
    assert json.load(open(path))
    ref = tss.spgemm(A, B)
    got = tss.spgemm(A, B, tuning={k: v for k, v in best.items() if k != "ms"})
    _same(ref, got)
    again = Autotuner(str(path)).tune(A, B, reps=2)  # cached
    assert {k: v for k, v in again.items()} == best


def test_batch_autotuner_settings_keep_results(tmp_path):
    """tune_batch's settings (one for the batch, then per class of instances
    with the same LDS strip size, bitmap widths 1 to 16 words): each
    instance's structure equals the oracle's and its values are within the
    tolerance; a second tuner reads the same settings from the cache."""
    from paper_2408_11988_amd.autotune import Autotuner
    from paper_2408_11988_amd.batched import Batched

    rng = np.random.default_rng(11)
    shapes = [(1500, 32, 0.01, 0.1), (1200, 96, 0.01, 0.2), (800, 400, 0.02, 0.05), (2000, 256, 0.004, 0.3),
              (600, 20, 0.03, 0.2)]
    host = [(random_csr(rng, n, n, pa, empty_rows=0.1, dense_rows=1), random_csr(rng, n, d, pb))
            for n, d, pa, pb in shapes]
    pairs = [(to_dev(a), to_dev(b)) for a, b in host]
    path = tmp_path / "tune.json"
    at = Autotuner(str(path))
    note("tune_batch on 5 instances")
    tun = at.tune_batch(pairs, reps=1)
    at.save()
    assert len(tun) == len(pairs) and json.load(open(path))
    bt = Batched(pairs, tun)
    bt.run()
    torch.cuda.synchronize()
    for (a, b), C in zip(host, bt.outputs()):
        compare_f32(a, b, C)
    assert Autotuner(str(path)).tune_batch(pairs, reps=1) == tun
