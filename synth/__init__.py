"""Seeded synthetic inputs for TS-SpGEMM (C = A.B, A square n x n, B n x d).

This module only *draws* inputs; it contains none of the multiply's
arithmetic. Tests hand the same arrays to the CPU oracle and to the GPU
library. The heavy lifting is in ``gen.cpp`` (OpenMP, counter-based
SplitMix64 streams, so results are independent of the thread count).

Workload recipes (stand-ins for the paper's web graphs and random
tall-and-skinny matrices, Sec. V-A, Table V):

* ``er``      Erdos-Renyi: ``draws`` uniform column draws per row, merged.
* ``rmat``    R-MAT (a,b,c,d) = (0.57,0.19,0.19,0.05), edge factor 16,
              symmetrised, self-loops dropped, duplicates merged, no vertex
              permutation.
* ``b_*``     B patterns: per-entry Bernoulli(p) or Poisson(lam) entries per
              row at uniform distinct columns.
* embedding   signed graph (+1 neighbours, -1 uniform negative samples) and
              an initial embedding with exactly k entries per row.
* values      U(0,1] on the FP32 grid ((m+1) 2^-24) or N(0,1), keyed by the
              entry's (row, col) so they do not depend on the pattern.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

# stream ids (must match gen.cpp)
S_AVAL, S_BVAL, S_W, S_AVALN = 3, 5, 9, 10

# seeds: workload c uses CONFIG_SEED + c; instance t of the batched workload
# uses CONFIG_SEED + 4 + 1000 * (t + 1)
CONFIG_SEED = 0x75510000


def build(force: bool = True) -> str:
    """Compile gen.cpp into libsynth.so (g++ -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, u64, f64, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_draw.restype = u64
        lib.synth_draw.argtypes = [u64, u64, u64]
        lib.synth_unit.restype = f64
        lib.synth_unit.argtypes = [u64, u64, u64]
        lib.synth_er.restype = vp
        lib.synth_er.argtypes = [i64, i32, u64]
        lib.synth_rmat.restype = vp
        lib.synth_rmat.argtypes = [i32, i64, i64, f64, f64, f64, u64]
        lib.synth_b_bernoulli.restype = vp
        lib.synth_b_bernoulli.argtypes = [i64, i32, f64, u64]
        lib.synth_b_poisson.restype = vp
        lib.synth_b_poisson.argtypes = [i64, i32, f64, u64]
        lib.synth_n.restype = i64
        lib.synth_n.argtypes = [vp]
        lib.synth_nnz.restype = i64
        lib.synth_nnz.argtypes = [vp]
        lib.synth_copy.restype = None
        lib.synth_copy.argtypes = [vp, vp, vp]
        lib.synth_free.restype = None
        lib.synth_free.argtypes = [vp]
        lib.synth_values.restype = None
        lib.synth_values.argtypes = [vp, vp, i64, i64, i32, i32, u64, u64, vp]
        lib.synth_sources.restype = i32
        lib.synth_sources.argtypes = [vp, i64, i32, u64, vp]
        lib.synth_negatives.restype = vp
        lib.synth_negatives.argtypes = [vp, vp, i64, i32, u64]
        lib.synth_embed_init.restype = None
        lib.synth_embed_init.argtypes = [i64, i32, i32, u64, vp, vp]
        _lib = lib
    return _lib


@dataclass
class Csr:
    """Host CSR: int32 row pointers and column indices, optional values."""

    nrows: int
    ncols: int
    rp: np.ndarray
    ci: np.ndarray
    val: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def with_values(self, val: np.ndarray) -> "Csr":
        return Csr(self.nrows, self.ncols, self.rp, self.ci, val)


def _take(h, ncols: int) -> Csr:
    lib = _load()
    n = lib.synth_n(h)
    nnz = lib.synth_nnz(h)
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(nnz, dtype=np.int32)
    lib.synth_copy(h, rp.ctypes.data, ci.ctypes.data)
    lib.synth_free(h)
    return Csr(int(n), int(ncols), rp, ci)


def draw_u64(seed: int, stream: int, i: int) -> int:
    return int(_load().synth_draw(seed, stream, i))


def draw_unit(seed: int, stream: int, i: int) -> float:
    return float(_load().synth_unit(seed, stream, i))


def er(n: int, draws: int, seed: int) -> Csr:
    """Erdos-Renyi pattern: `draws` uniform columns per row, duplicates merged."""
    return _take(_load().synth_er(n, draws, seed), n)


def rmat(scale: int, edge_factor: int, seed: int, n: int | None = None, a=0.57, b=0.19, c=0.19,
         nedges: int | None = None) -> Csr:
    """Symmetrised R-MAT pattern (self-loops dropped, duplicates merged)."""
    if n is None:
        n = 1 << scale
    if nedges is None:
        nedges = edge_factor * n
    return _take(_load().synth_rmat(scale, n, nedges, a, b, c, seed), n)


def b_bernoulli(n: int, d: int, p: float, seed: int) -> Csr:
    return _take(_load().synth_b_bernoulli(n, d, p, seed), d)


def b_poisson(n: int, d: int, lam: float, seed: int) -> Csr:
    return _take(_load().synth_b_poisson(n, d, lam, seed), d)


def values(m: Csr, kind: str, seed: int, stream: int, rng: int = 0) -> np.ndarray:
    """FP32 values for the stored entries of `m`.

    kind: 'uniform' (U(0,1] on the FP32 grid), 'normal' (N(0,1)), 'int'
    (integers in [-rng, rng], stored as float32)."""
    k = {"uniform": 0, "normal": 1, "int": 2}[kind]
    out = np.empty(m.nnz, dtype=np.float32)
    _load().synth_values(m.rp.ctypes.data, m.ci.ctypes.data, m.nrows, m.ncols, k, rng, seed, stream, out.ctypes.data)
    return out


def sources(a: Csr, d: int, seed: int) -> np.ndarray:
    """d distinct BFS sources, uniform among non-isolated vertices."""
    out = np.empty(d, dtype=np.int32)
    got = _load().synth_sources(a.rp.ctypes.data, a.nrows, d, seed, out.ctypes.data)
    return out[:got]


def frontier(n: int, srcs: np.ndarray) -> Csr:
    """One-hot n x d frontier: row srcs[j] holds column j (sources distinct)."""
    d = len(srcs)
    cnt = np.zeros(n + 1, dtype=np.int64)
    np.add.at(cnt, srcs.astype(np.int64) + 1, 1)
    rp = np.cumsum(cnt).astype(np.int32)
    order = np.argsort(srcs, kind="stable")
    ci = order.astype(np.int32)  # each row holds one column (distinct sources)
    return Csr(n, d, rp, ci)


def negatives(a: Csr, ns: int, seed: int) -> Csr:
    """`ns` distinct negative samples per vertex: uniform among vertices that
    are neither the vertex nor one of its neighbours in `a`."""
    return _take(_load().synth_negatives(a.rp.ctypes.data, a.ci.ctypes.data, a.nrows, ns, seed), a.nrows)


def signed_graph(a: Csr, neg: Csr) -> Csr:
    """The union of the neighbours (+1) and the negative samples (-1) of
    every vertex, as one CSR with sorted columns (the two patterns are
    disjoint)."""
    n = a.nrows
    rows = np.concatenate([np.repeat(np.arange(n), np.diff(a.rp)), np.repeat(np.arange(n), np.diff(neg.rp))])
    cols = np.concatenate([a.ci, neg.ci]).astype(np.int64)
    vals = np.concatenate([np.ones(a.nnz, np.float32), -np.ones(neg.nnz, np.float32)])
    order = np.lexsort((cols, rows))
    cnt = np.bincount(rows, minlength=n)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(cnt)
    return Csr(n, n, rp.astype(np.int32), cols[order].astype(np.int32), vals[order])


def embed_init(n: int, d: int, k: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Initial sparse n x d embedding with exactly k entries per row, stored
    at row * k (column ids sorted, int32; values float32)."""
    ci = np.empty(n * k, dtype=np.int32)
    val = np.empty(n * k, dtype=np.float32)
    _load().synth_embed_init(n, d, k, seed, ci.ctypes.data, val.ctypes.data)
    return ci, val


def w_on_pattern(c: Csr, seed: int) -> np.ndarray:
    """W[i,j] ~ N(0,1) for a dense n x d matrix W, evaluated on c's pattern only."""
    return values(c, "normal", seed, S_W)


# ---------------------------------------------------------------- workloads

def workload_er_small(seed: int = CONFIG_SEED + 1) -> tuple[Csr, Csr]:
    """ER 4096 x 4096, 8 draws/row, U(0,1); B 4096 x 64 Bernoulli(0.10), U(0,1)."""
    a = er(4096, 8, seed)
    a = a.with_values(values(a, "uniform", seed, S_AVAL))
    b = b_bernoulli(4096, 64, 0.10, seed)
    b = b.with_values(values(b, "uniform", seed, S_BVAL))
    return a, b


def workload_rmat_plain(scale: int = 20, d: int = 128, seed: int = CONFIG_SEED + 2) -> tuple[Csr, Csr]:
    """R-MAT scale `scale`, edge factor 16, U(0,1); B n x d, Poisson(0.2 d) per row, U(0,1)."""
    a = rmat(scale, 16, seed)
    a = a.with_values(values(a, "uniform", seed, S_AVAL))
    b = b_poisson(a.nrows, d, 0.2 * d, seed)
    b = b.with_values(values(b, "uniform", seed, S_BVAL))
    return a, b


def workload_wide_d(d: int, scale: int = 18, lam: float = 25.6, seed: int = CONFIG_SEED + 9) -> tuple[Csr, Csr]:
    """The varying-d sweep: R-MAT scale `scale`, edge factor 16, U(0,1); B n x d
    with Poisson(lam) entries per row (the same product count at every d, so
    only the output width changes), U(0,1)."""
    a = rmat(scale, 16, seed)
    a = a.with_values(values(a, "uniform", seed, S_AVAL))
    b = b_poisson(a.nrows, d, lam, seed)
    b = b.with_values(values(b, "uniform", seed, S_BVAL))
    return a, b


def workload_bfs(scale: int = 22, d: int = 512, seed: int = CONFIG_SEED + 3) -> tuple[Csr, np.ndarray]:
    """R-MAT scale `scale` pattern and d distinct non-isolated sources."""
    a = rmat(scale, 16, seed)
    return a, sources(a, d, seed)


def workload_embedding(scale: int = 20, d: int = 256, density: float = 0.05,
                       seed: int = CONFIG_SEED + 5) -> tuple[Csr, Csr]:
    """R-MAT scale `scale` U(0,1); B n x d Bernoulli(density) N(0,1)."""
    a = rmat(scale, 16, seed)
    a = a.with_values(values(a, "uniform", seed, S_AVAL))
    b = b_bernoulli(a.nrows, d, density, seed)
    b = b.with_values(values(b, "normal", seed, S_BVAL))
    return a, b


def workload_embed_step(scale: int = 17, edge_factor: int = 8, d: int = 128, sparsity: float = 0.8, ns: int = 5,
                        seed: int = CONFIG_SEED + 8):
    """Sparse-embedding epoch: R-MAT graph (a Flickr-sized stand-in at scale 17,
    edge factor 8) with `ns` negative samples per vertex as a signed n x n
    matrix (+1 neighbour, -1 negative sample), and an initial n x d embedding
    with k = d - floor(sparsity * d) entries per row. Returns (A, zci, zval, k)."""
    g = rmat(scale, edge_factor, seed)
    a = signed_graph(g, negatives(g, ns, seed))
    k = d - int(math.floor(sparsity * d + 1e-9))
    zci, zval = embed_init(a.nrows, d, k, seed)
    return a, zci, zval, k


def batched_params(count: int = 64, seed: int = CONFIG_SEED + 4, n_lo: int = 14, n_hi: int = 18):
    """Per-instance parameters of the batched workload.

    n = floor(2^U(n_lo, n_hi)); d uniform in {32,64,128,256}; A is ER or R-MAT
    (50/50) with average degree k uniform in [4, 32]; B density log-uniform in
    [1%, 50%]."""
    out = []
    for t in range(count):
        s = seed + 1000 * (t + 1)
        u = [draw_unit(s, 100, q) for q in range(5)]
        n = int(math.floor(2.0 ** (n_lo + (n_hi - n_lo) * u[0])))
        d = (32, 64, 128, 256)[min(3, int(u[1] * 4))]
        kind = "er" if u[2] < 0.5 else "rmat"
        k = 4 + min(28, int(u[3] * 29))
        dens = math.exp(math.log(0.01) + (math.log(0.5) - math.log(0.01)) * u[4])
        out.append(dict(seed=s, n=n, d=d, kind=kind, k=k, density=dens))
    return out


def batched_instance(p: dict) -> tuple[Csr, Csr]:
    s, n, d, k = p["seed"], p["n"], p["d"], p["k"]
    if p["kind"] == "er":
        a = er(n, k, s)
    else:
        scale = max(1, int(math.ceil(math.log2(n))))
        a = rmat(scale, k, s, n=n, nedges=(n * k) // 2)
    a = a.with_values(values(a, "uniform", s, S_AVAL))
    b = b_bernoulli(n, d, p["density"], s)
    b = b.with_values(values(b, "uniform", s, S_BVAL))
    return a, b
