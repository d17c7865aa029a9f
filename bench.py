"""Benchmark of the TS-SpGEMM hot path on one MI355X.

One step = one full plain TS-SpGEMM C = A B (symbolic phase: B bitmap, row
binning, bitmap-accumulator pattern, popcount scan, numeric binning, one host
sync for nnz(C); numeric phase: the LDS dense-strip kernel) over the R-MAT
scale-20 (edge factor 16) x (n x 128, Poisson(25.6) entries per row) workload,
all inputs resident in HBM. Prints one JSON line.

The same line carries three further measurements of the path (skipped with
--no-extras): the differentiable layer (numeric forward plus dL/dA and dL/dB on
R-MAT scale 20 x n x 256 Normal values), the batched run of 64 mixed instances
replayed from one HIP graph against the same 64 products as plain calls, and
multi-source BFS (Algorithm 3) from 512 sources on R-MAT scale 22, and the
density of B from which the dense-B SpMM beats TS-SpGEMM (Sec. V-C).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras] [--scale S]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of every HIP source and header of the library: any change to a
    kernel, a launch or a threshold invalidates the stored counter figures."""
    import glob

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2408_11988_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    h.update(open(os.path.join(ROOT, "include", "tsspgemm.h"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per numeric launch from the committed rocprofv3 counter summary,
    or None when the summary is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return float(e["bytes_per_launch"])


def copy_bandwidth_gbs(torch):
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(10):
        b.copy_(a)
    e.record()
    e.synchronize()
    t = s.elapsed_time(e) / 10 / 1e3
    del a, b
    return 2 * 4 * n / t / 1e9


def cpu_baseline(a, b, flops_rows, target_s=12.0):
    """The oracle as it stands, on a random sample of rows of the same workload."""
    import numpy as np

    import oracle

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(1234)
    n = a.nrows
    probe = rng.choice(n, size=min(n, 20000), replace=False).astype(np.int32)
    t0 = time.perf_counter()
    oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, rows=probe, threads=threads)
    t_probe = time.perf_counter() - t0
    f_probe = max(1, int(flops_rows[probe].sum()))
    est_full = t_probe * float(flops_rows.sum()) / f_probe
    frac = min(1.0, target_s / max(est_full, 1e-9))
    if frac >= 1.0:
        rows = None
        sample = "all rows"
        fl = int(flops_rows.sum())
    else:
        k = max(1, int(frac * n))
        rows = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
        sample = f"{k} uniformly sampled rows of {n} ({100.0 * k / n:.1f}%)"
        fl = int(flops_rows[rows].sum())
    t0 = time.perf_counter()
    oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, rows=rows, threads=threads)
    t = time.perf_counter() - t0
    return {"value": round(2.0 * fl / t / 1e9, 4), "unit": "GFLOPS", "cores": threads, "kind": "oracle",
            "sample": f"{sample}; {fl} multiplications in {t:.2f} s (ordered-map Gustavson, FP64)"}


def _roofline(bytes_alg: int, ms: float, kernel: str, traffic_key: str | None = None) -> dict:
    """HBM roofline of one launch (or call) from its algorithmic bytes; `traffic`
    is the measured HBM bytes per launch from the committed counter summary
    (null when it is missing or the kernel sources changed since)."""
    gbs = bytes_alg / (ms / 1e3) / 1e9
    traffic = measured_traffic(traffic_key) if traffic_key else None
    return {"bound": "hbm", "kernel": kernel, "bytes_alg_per_launch": int(bytes_alg), "ms": round(ms, 4),
            "achieved": round(gbs, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
            "traffic": traffic}


def _events(n):
    import torch

    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def bench_fwd_bwd(steps: int, warmup: int) -> dict:
    """Differentiable layer: R-MAT scale 20 x B n x 256 (5%, N(0,1)), loss sum(C o W).
    Forward = numeric phase on the cached plan; backward = dL/dA + dL/dB (A^T cached)."""
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, TSSpGEMMOp

    log("fwd+bwd: generating R-MAT 20 x d=256 (5%)")
    a, b = synth.workload_embedding(scale=20, d=256, density=0.05)
    A, B = DeviceCsr.from_host(a), DeviceCsr.from_host(b)
    op = TSSpGEMMOp(A, B)
    op.transpose()
    flops = op.plan.stats()["flops"]
    av = A.vals.clone().requires_grad_(True)
    bv = B.vals.clone().requires_grad_(True)
    c = op(av, bv)
    w = torch.randn(c.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    for _ in range(warmup):
        av.grad = bv.grad = None
        (op(av, bv) * w).sum().backward()
    torch.cuda.synchronize()
    ef, eb = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        e = _events(3)
        av.grad = bv.grad = None
        e[0].record()
        c = op(av, bv)
        e[1].record()
        (c * w).sum().backward()
        e[2].record()
        ef.append(e)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    ms_f = sum(x[0].elapsed_time(x[1]) for x in ef) / steps
    ms_b = sum(x[1].elapsed_time(x[2]) for x in ef) / steps
    # the library's backward call alone (both gradients, G = W on pat(C))
    from paper_2408_11988_amd import backward

    AT, perm = op.transpose()
    Av, Bv = op.A.with_vals(av.detach()), op.B.with_vals(bv.detach())
    G = op.c_pattern().with_vals(w)
    for _ in range(warmup):
        backward(op.plan, AT, perm, Av, Bv, G)
    torch.cuda.synchronize()
    e = _events(2)
    e[0].record()
    for _ in range(steps):
        backward(op.plan, AT, perm, Av, Bv, G)
    e[1].record()
    torch.cuda.synchronize()
    ms_lib_bwd = e[0].elapsed_time(e[1]) / steps
    n, nnz_a, nnz_b, nnz_c = a.nrows, a.nnz, b.nnz, op.nnz
    rp = 4 * (n + 1)
    fwd_bytes = (rp + 8 * nnz_a) + (rp + 8 * nnz_b) + (rp + 8 * nnz_c)
    # inputs A (pattern, values), B, G on pat(C), A^T (pattern, permutation);
    # outputs dL/dA and dL/dB
    bwd_bytes = (rp + 8 * nnz_a) + (rp + 8 * nnz_b) + (rp + 8 * nnz_c) + (rp + 8 * nnz_a) + 4 * nnz_a + 4 * nnz_b
    return {"workload": "R-MAT scale 20 x B n x 256 Bernoulli(0.05) N(0,1), loss sum(C o W)",
            "flops_fwd": flops, "nnz_c": op.nnz, "ms_fwd": round(ms_f, 4), "ms_bwd": round(ms_b, 4),
            "ms_bwd_library": round(ms_lib_bwd, 4),
            "ms_fwd_bwd": round(ms_step, 4), "gflops_fwd": round(2 * flops / ms_f / 1e6, 2),
            "gflops_bwd": round(2 * 2 * flops / ms_b / 1e6, 2),
            "gflops_fwd_bwd": round(2 * 3 * flops / ms_step / 1e6, 2),
            "roofline_fwd": _roofline(fwd_bytes, ms_f, "numeric phase of the forward (one tsspgemm_numeric call)",
                                      "rmat20_d256_forward"),
            "roofline_bwd": _roofline(bwd_bytes, ms_lib_bwd, "tsspgemm_backward (dL/dA and dL/dB, one call)",
                                      "rmat20_d256_backward"),
            "note": "bwd = dL/dA (SDDMM on pat(A)) + dL/dB (A^T G sampled on pat(B)), each as many products as fwd;"
                    " ms_bwd is the autograd backward with the loss's elementwise product and sum; "
                    "ms_bwd_library is the library call alone"}


def bench_batched(steps: int, warmup: int) -> dict:
    """64 instances (n log-uniform in [2^14, 2^18], d in {32..256}, ER or R-MAT,
    B density log-uniform in [1%, 50%]): one graph replay vs 64 plain calls."""
    import tempfile

    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, spgemm
    from paper_2408_11988_amd.autotune import Autotuner
    from paper_2408_11988_amd.batched import Batched

    log("batched: generating 64 instances")
    host = [synth.batched_instance(p) for p in synth.batched_params()]
    pairs = [(DeviceCsr.from_host(a), DeviceCsr.from_host(b)) for a, b in host]
    t0 = time.perf_counter()
    tuner = Autotuner(os.path.join(tempfile.gettempdir(), "tsspgemm_autotune_bench.json"))
    tunings = tuner.tune_batch(pairs, reps=2)
    tuner.save()
    t_tune = time.perf_counter() - t0
    clean = [{k: v for k, v in t.items() if k != "ms"} for t in tunings]
    bt = Batched(pairs, clean)
    bt.capture()
    for _ in range(warmup):
        bt.replay()
    torch.cuda.synchronize()
    e = _events(2)
    e[0].record()
    for _ in range(steps):
        bt.replay()
    e[1].record()
    torch.cuda.synchronize()
    ms_graph = e[0].elapsed_time(e[1]) / steps
    flops = sum(bt.flops())
    # the same 64 products as plain calls with default tuning, one after the
    # other (each synchronizes for nnz)
    for _ in range(warmup):
        for A, B in pairs:
            spgemm(A, B)
    torch.cuda.synchronize()
    reps = max(1, steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        for A, B in pairs:
            spgemm(A, B)
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / reps
    # the numeric phases alone of the 64 products (plans made beforehand),
    # captured as 64 plain numeric calls in one HIP graph
    from paper_2408_11988_amd import numeric, symbolic
    plans = []
    for A, B in pairs:
        plan, _, nnz = symbolic(A, B)
        plans.append((plan, torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda"),
                      torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda")))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for (A, B), (plan, ci, cv) in zip(pairs, plans):
            numeric(plan, A, B, ci, cv)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for (A, B), (plan, ci, cv) in zip(pairs, plans):
            numeric(plan, A, B, ci, cv)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    e = _events(2)
    e[0].record()
    for _ in range(steps):
        graph.replay()
    e[1].record()
    torch.cuda.synchronize()
    ms_num_graph = e[0].elapsed_time(e[1]) / steps
    del graph, plans
    rp_bytes = sum(3 * 4 * (a.nrows + 1) for a, _ in host)
    batch_bytes = rp_bytes + sum(8 * (a.nnz + b.nnz) for a, b in host) + 8 * bt.pool
    return {"workload": "64 instances: n log-uniform [2^14, 2^18], d in {32,64,128,256}, ER/R-MAT (deg 4-32), "
                        "B density log-uniform [1%, 50%], plus-times FP32",
            "roofline": _roofline(batch_bytes, ms_graph, "one graph replay (symbolic + numeric of all 64 instances)",
                                  "batched_64_replay"),
            "roofline_numeric_calls": _roofline(batch_bytes, ms_num_graph,
                                                "the 64 numeric phases captured as plain calls"),
            "sum_n": sum(a.nrows for a, _ in host), "sum_nnz_a": sum(a.nnz for a, _ in host), "flops": flops,
            "nnz_c": bt.pool, "ms_graph_replay": round(ms_graph, 4), "ms_64_plain_calls": round(ms_seq, 4),
            "gflops_graph": round(2 * flops / ms_graph / 1e6, 2), "gflops_plain_calls": round(2 * flops / ms_seq / 1e6, 2),
            "speedup_vs_plain_calls": round(ms_seq / ms_graph, 3),
            "ms_64_numeric_calls_graph": round(ms_num_graph, 4),
            "note": "graph replay = symbolic + numeric of all 64 in one launch per phase; plain calls = 64 x "
                    "(symbolic with its nnz sync + numeric); numeric_calls_graph = the 64 numeric phases only, "
                    "plans made beforehand, captured as plain calls in one HIP graph",
            "autotune_s": round(t_tune, 2)}


def bench_spmm_crossover(reps: int = 5) -> dict:
    """TS-SpGEMM (symbolic + numeric, and numeric alone with the plan reused)
    against the dense-B SpMM on the same products, for a range of B densities:
    R-MAT scale 18 (edge factor 16) x n x 128, U(0,1) values (Sec. V-C)."""
    import numpy as np
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, numeric, spmm, symbolic

    a = synth.rmat(18, 16, synth.CONFIG_SEED + 6)
    a = a.with_values(synth.values(a, "uniform", synth.CONFIG_SEED + 6, synth.S_AVAL))
    A = DeviceCsr.from_host(a)
    n, d = a.nrows, 128

    def med(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e = _events(2)
            e[0].record()
            fn()
            e[1].record()
            e[1].synchronize()
            ts.append(e[0].elapsed_time(e[1]))
        return float(np.median(ts))

    rows = []
    for rho in (0.05, 0.1, 0.2, 0.35, 0.5, 0.65, 0.8, 1.0):
        b = synth.b_bernoulli(n, d, rho, synth.CONFIG_SEED + 7)
        b = b.with_values(synth.values(b, "uniform", synth.CONFIG_SEED + 7, synth.S_BVAL))
        B = DeviceCsr.from_host(b)
        dense = torch.zeros((n, d), dtype=torch.float32, device="cuda")
        rr = torch.repeat_interleave(torch.arange(n, device="cuda"), torch.diff(B.rowptr).to(torch.int64))
        dense[rr, B.colidx.to(torch.int64)] = B.vals
        plan, _, nnz = symbolic(A, B)
        ci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
        cv = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda")

        def full():
            _, _, nz = symbolic(A, B, plan=plan)
            numeric(plan, A, B, ci, cv)

        ms_full = med(full)
        ms_num = med(lambda: numeric(plan, A, B, ci, cv))
        ms_spmm = med(lambda: spmm(A, dense))
        rows.append({"density": rho, "ms_tsspgemm": round(ms_full, 4), "ms_tsspgemm_numeric": round(ms_num, 4),
                     "ms_spmm": round(ms_spmm, 4), "nnz_c": nnz})
        del B, dense, plan, ci, cv
        torch.cuda.empty_cache()
    def wins_from(key):
        # lowest measured density from which SpMM is at least as fast at it
        # and at every higher density (None: TS-SpGEMM wins at the densest)
        out = None
        for r in reversed(rows):
            if r["ms_spmm"] > r[key]:
                break
            out = r["density"]
        return out

    cross = wins_from("ms_tsspgemm")
    cross_num = wins_from("ms_tsspgemm_numeric")
    return {"workload": "R-MAT scale 18 (edge factor 16) x B n x 128 Bernoulli(density), U(0,1), plus-times FP32",
            "nnz_a": a.nnz, "points": rows,
            "spmm_wins_from_density": cross, "spmm_wins_from_density_vs_numeric_only": cross_num,
            "note": "SpMM reads the dense B (zeros included) and writes dense C; TS-SpGEMM reads and writes CSR"}


def bench_embed(cpu: bool) -> dict:
    """Sparse-embedding update (Sec. IV-B): one epoch over an R-MAT 17 graph
    (edge factor 8) with 5 negative samples per vertex, d = 128 at 80% sparsity
    (k = 26), lr 0.02, in minibatches of 256 rows (eager launches and one HIP
    graph of the whole epoch) and of n/2 rows."""
    import numpy as np
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, embed_epoch

    a, zci, zval, k = synth.workload_embed_step()
    d, lr = 128, float(np.float32(0.02))
    n = a.nrows
    A = DeviceCsr.from_host(a)
    z0c, z0v = torch.from_numpy(zci).cuda(), torch.from_numpy(zval).cuda()
    zc, zv = z0c.clone(), z0v.clone()

    def run(batch):
        embed_epoch(A, zc, zv, d, k, lr, batch)

    def timed(fn, reps=5):
        ts = []
        for _ in range(reps):
            zc.copy_(z0c)
            zv.copy_(z0v)
            e = _events(2)
            e[0].record()
            fn()
            e[1].record()
            e[1].synchronize()
            ts.append(e[0].elapsed_time(e[1]))
        return float(np.median(ts))

    half = (n + 1) // 2
    run(256)
    torch.cuda.synchronize()
    ms_256 = timed(lambda: run(256))
    ms_half = timed(lambda: run(half))
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run(256)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        run(256)
    ms_256_graph = timed(graph.replay)
    deg = np.diff(a.rp).astype(np.int64)
    # algorithmic bytes of one epoch: the workspace copy of Z (read + write),
    # per row its A row (8 B an entry + 8 B of row pointers), z_i and every
    # z_j (8 B an entry), the new row, and the copy of the previous
    # minibatch's rows (read + write)
    alg = 16 * n * k + int((8 + 8 * deg + 8 * k * (1 + deg) + 8 * k + 16 * k).sum())
    out = {"workload": f"R-MAT scale 17 (edge factor 8) + 5 negative samples per vertex, n={n}, nnz(A)={a.nnz}, "
                       f"d={d}, k={k} (80% sparse), lr 0.02",
           "ms_epoch_b256": round(ms_256, 3), "ms_epoch_b256_graph": round(ms_256_graph, 3),
           "ms_epoch_b_half": round(ms_half, 3), "minibatches_b256": (n + 255) // 256,
           "rows_per_s_b256_graph": round(n / ms_256_graph * 1e3, 1),
           "force_terms_per_s_b_half": round(a.nnz / ms_half * 1e3, 1),
           "alg_bytes_epoch": alg, "alg_gbs_b_half": round(alg / ms_half / 1e6, 1),
           "alg_gbs_b256_graph": round(alg / ms_256_graph / 1e6, 1)}
    if cpu:
        import oracle

        t0 = time.perf_counter()
        oracle.embed_epoch(a.rp, a.ci, a.val, zci, zval, d, k, lr, 256)
        t = time.perf_counter() - t0
        out["cpu_oracle_ms_epoch_b256"] = round(t * 1e3, 1)
        out["cpu_oracle_cores"] = 1
    return out


def bench_tiles() -> dict:
    """Column-tiled multiply (Sec. III-B, Algorithm 2 on one GPU) on the plain
    workload, R-MAT 20 x 128: for T column tiles, the numeric phases of the T
    tile products (plans made beforehand) and the merge of their outputs,
    against T = 1 (the plain multiply's numeric phase)."""
    import numpy as np
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, column_slice, merge_rows, numeric, symbolic, tile_edges

    a, b = synth.workload_rmat_plain(scale=20, d=128)
    A, B = DeviceCsr.from_host(a), DeviceCsr.from_host(b)

    def med(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            e = _events(2)
            e[0].record()
            fn()
            e[1].record()
            e[1].synchronize()
            ts.append(e[0].elapsed_time(e[1]))
        return float(np.median(ts))

    rows = []
    for T in (1, 2, 4, 8, 16, 32):
        e = tile_edges(a.nrows, T)
        slices = [column_slice(A, e[t], e[t + 1]) for t in range(T)]
        plans = []
        for S in slices:
            plan, rp, nnz = symbolic(S, B)
            plans.append((S, plan, rp, torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda"),
                          torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda")))

        def numerics():
            for S, plan, rp, ci, cv in plans:
                numeric(plan, S, B, ci, cv)

        ms_num = med(numerics)
        parts = [DeviceCsr(a.nrows, b.ncols, rp, ci[:int(rp[-1])], cv[:int(rp[-1])]) for S, plan, rp, ci, cv in plans]
        ms_merge = med(lambda: merge_rows(parts)) if T > 1 else 0.0
        rows.append({"tiles": T, "tile_columns": e[1] - e[0], "b_rows_bytes_per_tile": int(5 * (b.rp[e[1]] - b.rp[0])),
                     "partial_nnz": int(sum(int(p.nnz) for p in parts)), "ms_numeric_sum": round(ms_num, 4),
                     "ms_merge": round(ms_merge, 4), "ms_numeric_and_merge": round(ms_num + ms_merge, 4)})
        del plans, parts, slices
        torch.cuda.empty_cache()
    return {"workload": "R-MAT scale 20 (edge factor 16) x B n x 128 Poisson(25.6)/row, U(0,1), plus-times FP32",
            "points": rows,
            "note": "T = 1 is the plain multiply; B rows of a tile hold 5 B per entry (narrowed id and value)"}


def bench_wide_d() -> dict:
    """Varying d with the product count fixed (Sec. V's d sweep shape): R-MAT
    scale 18 x B n x d with Poisson(25.6) entries per row, plus-times FP32.
    d <= 1024 uses the LDS strip, larger d the hash accumulator (Sec. III-C).
    Medians of 7 symbolic and 7 numeric calls on one plan."""
    import numpy as np
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, numeric, symbolic

    def med(fn, reps=7):
        fn()
        ts = []
        for _ in range(reps):
            e = _events(2)
            e[0].record()
            fn()
            e[1].record()
            e[1].synchronize()
            ts.append(e[0].elapsed_time(e[1]))
        return float(np.median(ts))

    rows = []
    for d in (128, 512, 1024, 2048, 4096, 16384, 65536):
        a, b = synth.workload_wide_d(d)
        A, B = DeviceCsr.from_host(a), DeviceCsr.from_host(b)
        plan, _, nnz = symbolic(A, B)
        st = plan.stats()
        ci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
        cv = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda")
        ms_sym = med(lambda: symbolic(A, B, plan=plan))
        ms_num = med(lambda: numeric(plan, A, B, ci, cv))
        rows.append({"d": d, "accumulator": "lds" if d <= 1024 else "hash", "nnz_c": int(nnz),
                     "flops": int(st["flops"]), "split_rows": int(st["split_rows"]) if d > 1024 else None,
                     "ms_symbolic": round(ms_sym, 4), "ms_numeric": round(ms_num, 4),
                     "gflops_step": round(2 * st["flops"] / (ms_sym + ms_num) / 1e6, 1)})
        del plan, ci, cv, A, B
        torch.cuda.empty_cache()
    return {"workload": "R-MAT scale 18 (edge factor 16) x B n x d Poisson(25.6)/row, U(0,1), plus-times FP32",
            "points": rows}


def bench_er_small(cpu: bool) -> dict:
    """The small ER case (4096 x 4096, 8 draws per row; B 4096 x 64 at 10%):
    a whole plain step (symbolic with its nnz synchronisation, then numeric)
    and the numeric phase alone, medians of 50. Launch-latency bound."""
    import numpy as np
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, numeric, symbolic

    a, b = synth.workload_er_small()
    A, B = DeviceCsr.from_host(a), DeviceCsr.from_host(b)
    plan, _, nnz = symbolic(A, B)
    ci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    cv = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda")
    flops = int(plan.stats()["flops"])

    def med(fn, reps=50):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    def step():
        symbolic(A, B, plan=plan)
        numeric(plan, A, B, ci, cv)

    ms_step = med(step)
    ms_num = med(lambda: numeric(plan, A, B, ci, cv))
    out = {"workload": "ER 4096 x 4096 (8 draws per row) x B 4096 x 64 Bernoulli(0.10), U(0,1), plus-times FP32",
           "nnz_a": a.nnz, "nnz_b": b.nnz, "nnz_c": nnz, "flops": flops, "ms_step": round(ms_step, 4),
           "ms_numeric": round(ms_num, 4), "gflops_step": round(2 * flops / ms_step / 1e6, 2)}
    if cpu:
        import oracle

        t0 = time.perf_counter()
        oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val, threads=1)
        out["cpu_oracle_ms_1_thread"] = round((time.perf_counter() - t0) * 1e3, 2)
    return out


def bench_bfs(cpu: bool) -> dict:
    """Multi-source BFS, R-MAT scale 22, 512 sources: masked Boolean TS-SpGEMM until
    every frontier is empty, levels n x 512 int32."""
    import numpy as np
    import torch

    import synth
    from paper_2408_11988_amd import DeviceCsr, msbfs

    log("bfs: generating R-MAT 22")
    a, srcs = synth.workload_bfs(scale=22, d=512)
    A = DeviceCsr.from_host(a, with_values=False)
    src = torch.from_numpy(srcs).cuda()
    lev, fn = msbfs(A, src)  # warm-up (allocations)
    del lev
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        lev, fn = msbfs(A, src)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        if len(times) < 3:
            del lev
    ms = sorted(times)[1]
    deg = torch.diff(A.rowptr).to(torch.int64)
    reached = (lev >= 0).sum(dim=1).to(torch.int64)
    products = int((deg * reached).sum())  # AND products over the run = sum_s sum_{v reached} deg(v)
    pairs = int(reached.sum())
    # per masked product: A's pattern, the frontier F as CSR, the visited set
    # as an n x d bitmap, the new frontier N as CSR; then the n x d levels
    n, d = a.nrows, 512
    fr = [d] + list(fn)  # nnz(F) entering each product, then after it
    bfs_bytes = sum((4 * (n + 1) + 4 * a.nnz) + (4 * (n + 1) + 4 * fr[t]) + n * d // 8 + (4 * (n + 1) + 4 * fr[t + 1])
                    for t in range(len(fn))) + 4 * n * d
    out = {"workload": "R-MAT scale 22 (edge factor 16, symmetrised, pattern), 512 sources, Boolean masked",
           "roofline": _roofline(bfs_bytes, ms, "the whole multi-source BFS (every masked product and the levels)",
                                  "msbfs_rmat22_d512"),
           "n": a.nrows, "nnz_a": a.nnz, "iterations": len(fn), "frontier_nnz": fn, "ms_total": round(ms, 3),
           "reached_pairs": pairs, "and_products": products,
           "gflops": round(2 * products / ms / 1e6, 2), "traversed_edges_per_s": round(products / ms * 1e3, 1),
           "levels_bytes": a.nrows * 512 * 4}
    if cpu:
        import oracle

        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        k = 32
        t0 = time.perf_counter()
        oracle.bfs_queue(a.rp, a.ci, srcs[:k], threads=threads)
        t = time.perf_counter() - t0
        edges = int((deg * (lev[:, :k] >= 0).sum(dim=1).to(torch.int64)).sum())
        out["cpu_baseline"] = {"value": round(edges / t, 1), "unit": "traversed edges/s", "cores": threads,
                               "kind": "oracle", "sample": f"queue BFS from {k} of the 512 sources, {t:.2f} s"}
    del lev
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--d", type=int, default=128)
    ap.add_argument("--products", choices=["auto", "rows", "flat", "vec4"], default="auto",
                    help="product layout of the plain workload's numeric phase (default: the library's choice)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the plain workload")
    ap.add_argument("--leg", choices=["er_small", "fwd_bwd", "batched", "spmm", "embed", "tiles", "bfs", "wide_d"],
                    help="run only this extra workload and print its JSON (for profiling one workload)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB a few times (reference for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: TS-SpGEMM here is one rank's local multiply "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        torch.cuda.set_device(0)
        bw = copy_bandwidth_gbs(torch)
        print(json.dumps({"copy_bytes_read_per_launch": 1 << 30, "copy_bytes_written_per_launch": 1 << 30,
                          "launches": 12, "copy_bw_gbs": round(bw, 1)}), flush=True)
        return

    if args.leg:
        torch.cuda.set_device(0)
        legs = {"er_small": lambda: bench_er_small(not args.no_cpu),
                "fwd_bwd": lambda: bench_fwd_bwd(args.steps, args.warmup), "tiles": bench_tiles,
                "batched": lambda: bench_batched(args.steps, args.warmup),
                "spmm": bench_spmm_crossover, "embed": lambda: bench_embed(not args.no_cpu),
                "bfs": lambda: bench_bfs(not args.no_cpu), "wide_d": bench_wide_d}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return

    import synth
    from paper_2408_11988_amd import DeviceCsr, _lib

    lib = _lib.load()
    torch.cuda.set_device(0)
    workload = f"rmat{args.scale}_d{args.d}_plain"
    log(f"generating R-MAT scale {args.scale} x d={args.d}")
    a, b = synth.workload_rmat_plain(scale=args.scale, d=args.d)
    A = DeviceCsr.from_host(a)
    B = DeviceCsr.from_host(b)
    da, db = A.desc(), B.desc()
    n, d = a.nrows, b.ncols
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    c_rowptr = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    plan = ctypes.c_void_p(None)
    nnz = ctypes.c_int64(0)

    from paper_2408_11988_amd.api import tuning_struct

    tune = None if args.products == "auto" else ctypes.byref(tuning_struct({"products": args.products}))

    def symbolic():
        _lib.check(lib.tsspgemm_symbolic(ctypes.byref(da), ctypes.byref(db), _lib.PLUS_TIMES_F32, None, tune,
                                         ctypes.c_void_p(c_rowptr.data_ptr()), ctypes.byref(nnz),
                                         ctypes.byref(plan), sp), "symbolic")
        return int(nnz.value)

    nnz_c = symbolic()
    c_colidx = torch.empty(nnz_c, dtype=torch.int32, device="cuda")
    c_vals = torch.empty(nnz_c, dtype=torch.float32, device="cuda")

    def numeric():
        _lib.check(lib.tsspgemm_numeric(plan, ctypes.byref(da), ctypes.byref(db),
                                        ctypes.c_void_p(c_colidx.data_ptr()), ctypes.c_void_p(c_vals.data_ptr()),
                                        sp), "numeric")

    st = [ctypes.c_int64() for _ in range(6)]
    lib.tsspgemm_plan_stats(plan, *[ctypes.byref(x) for x in st])
    flops, _, light_rows, wave_rows, block_rows, split_rows = [int(x.value) for x in st]
    log(f"nnz(A)={a.nnz} nnz(B)={b.nnz} nnz(C)={nnz_c} flops={flops} rows: light={light_rows} wave={wave_rows} "
        f"block={block_rows} split={split_rows}")

    for _ in range(args.warmup):
        symbolic()
        numeric()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        symbolic()
        ev[k][1].record(stream)
        numeric()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_sym = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
    ms_num = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps
    per_step = sorted(e[0].elapsed_time(e[2]) for e in ev)  # HIP events, one step each
    log(f"step {ms_step:.3f} ms  symbolic {ms_sym:.3f} ms  numeric {ms_num:.3f} ms")

    bytes_alg = (4 * (n + 1) + 8 * a.nnz) + (4 * (n + 1) + 8 * b.nnz) + (4 * (n + 1) + 8 * nnz_c)
    achieved = bytes_alg / (ms_num / 1e3) / 1e9
    traffic = measured_traffic(workload)
    copy_bw = copy_bandwidth_gbs(torch)

    result = {
        "metric": "TS-SpGEMM GFLOPS (2x mults/s) + % HBM roofline; batched & fwd+bwd vs plain",
        "value": round(2.0 * flops / (ms_step / 1e3) / 1e9, 3),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision": "FP32 inputs and outputs; products and sums accumulated in FP64, one rounding to FP32",
        "data": "synthetic (seeded R-MAT and Poisson tall-skinny B; inputs resident in HBM)",
        "config": {"workload": f"R-MAT scale {args.scale} (edge factor 16, symmetrised) x B n x {args.d} "
                               f"Poisson({0.2 * args.d:g}) entries/row, plus-times FP32",
                   "n": n, "d": d, "nnz_a": a.nnz, "nnz_b": b.nnz, "nnz_c": nnz_c, "flops": flops},
        "ms_symbolic": round(ms_sym, 4),
        "ms_numeric": round(ms_num, 4),
        "ms_step_events": {"median": round(per_step[len(per_step) // 2], 4), "min": round(per_step[0], 4),
                           "mean": round(sum(per_step) / len(per_step), 4)},
        "gflops_numeric_only": round(2.0 * flops / (ms_num / 1e3) / 1e9, 3),
        "output_nnz_per_s": round(nnz_c / (ms_step / 1e3), 1),
        "roofline": {"bound": "hbm", "kernel": "numeric phase (k_numeric + k_numeric_light + k_split_finalize)",
                     "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "bytes_alg_per_launch": bytes_alg,
                     "bytes_gather_model": 8 * flops + 8 * a.nnz,
                     "traffic_gbs": round(traffic / (ms_num / 1e3) / 1e9, 1) if traffic else None},
        "copy_bw_gbs": round(copy_bw, 1),
    }
    if not args.no_cpu:
        log("timing the oracle on the host")
        import oracle

        flops_rows = oracle.row_flops(a.rp, a.ci, b.rp)
        result["cpu_baseline"] = cpu_baseline(a, b, flops_rows)
    else:
        result["cpu_baseline"] = None
    lib.tsspgemm_plan_destroy(plan)
    del c_colidx, c_vals, A, B
    if not args.no_extras:
        result["er_small"] = bench_er_small(not args.no_cpu)
        log(f"ER small step {result['er_small']['ms_step']} ms")
        result["fwd_bwd"] = bench_fwd_bwd(max(3, args.steps // 2), args.warmup)
        log(f"fwd+bwd {result['fwd_bwd']['ms_fwd']} + {result['fwd_bwd']['ms_bwd']} ms")
        torch.cuda.empty_cache()
        result["batched"] = bench_batched(max(4, args.steps // 2), args.warmup)
        log(f"batched graph {result['batched']['ms_graph_replay']} ms vs plain calls "
            f"{result['batched']['ms_64_plain_calls']} ms")
        torch.cuda.empty_cache()
        result["spmm_crossover"] = bench_spmm_crossover()
        log(f"spmm crossover at density {result['spmm_crossover']['spmm_wins_from_density']}")
        torch.cuda.empty_cache()
        result["tiles"] = bench_tiles()
        log("tiled multiply: " + ", ".join(f"T={r['tiles']} {r['ms_numeric_and_merge']} ms"
                                           for r in result["tiles"]["points"]))
        torch.cuda.empty_cache()
        result["embed"] = bench_embed(not args.no_cpu)
        log(f"embed epoch {result['embed']['ms_epoch_b256_graph']} ms (256-row minibatches, graph), "
            f"{result['embed']['ms_epoch_b_half']} ms (n/2)")
        torch.cuda.empty_cache()
        result["bfs"] = bench_bfs(not args.no_cpu)
        log(f"bfs {result['bfs']['ms_total']} ms, {result['bfs']['iterations']} iterations")
        torch.cuda.empty_cache()
        result["wide_d"] = bench_wide_d()
        log("varying d: " + ", ".join(f"d={r['d']} {r['gflops_step']} GFLOPS" for r in result["wide_d"]["points"]))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
