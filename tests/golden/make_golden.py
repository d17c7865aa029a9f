"""Write the regression fixtures in this folder.

The paper prints no worked example with values (its toy examples are in
figures that carry no numbers in text), so these fixtures are not the paper's:
they freeze small seeded inputs (from the generators) together with the
oracle's outputs, so a later change to either shows up as a diff. Stored
floats are written with float.hex, so they round-trip exactly.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def _ints(a):
    return " ".join(str(int(x)) for x in a)


def _floats(a):
    return " ".join(float(x).hex() for x in a)


def write(name, header, fields):
    with open(os.path.join(HERE, name), "w") as f:
        f.write("# " + header + "\n")
        for k, (kind, v) in fields.items():
            f.write(f"{k} {kind} {len(v)}: " + (_ints(v) if kind == "i" else _floats(v)) + "\n")


def spgemm_case():
    seed = 20240811
    a = synth.er(12, 3, seed)
    a = a.with_values(synth.values(a, "uniform", seed, synth.S_AVAL))
    b = synth.b_bernoulli(12, 5, 0.4, seed)
    b = b.with_values(synth.values(b, "uniform", seed, synth.S_BVAL))
    rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    write("spgemm_er12_d5.txt", "Eq. (1) plus-times on ER(12, 3 draws) x Bernoulli(12 x 5, 0.4), seed 20240811",
          {"a_rp": ("i", a.rp), "a_ci": ("i", a.ci), "a_val": ("f", a.val), "b_rp": ("i", b.rp),
           "b_ci": ("i", b.ci), "b_val": ("f", b.val), "c_rp": ("i", rp), "c_ci": ("i", ci), "c_val": ("f", val)})


def bfs_case():
    a, srcs = synth.workload_bfs(scale=6, d=4, seed=20240812)
    lev, fnnz = oracle.msbfs(a.rp, a.ci, srcs)
    write("msbfs_rmat6_d4.txt", "Algorithm 3 levels on R-MAT scale 6 (edge factor 16), 4 sources, seed 20240812",
          {"a_rp": ("i", a.rp), "a_ci": ("i", a.ci), "sources": ("i", srcs), "levels": ("i", lev.ravel()),
           "frontier_nnz": ("i", fnnz)})


def grad_case():
    a, b = synth.workload_embedding(scale=4, d=8, density=0.3, seed=20240813)
    rp, ci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    c = synth.Csr(a.nrows, b.ncols, rp.astype(np.int32), ci)
    g = synth.w_on_pattern(c, 20240813)
    ga = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, b.val, rp, ci, g)
    gb = oracle.grad_b(a.rp, a.ci, a.val, b.rp, b.ci, rp, ci, g)
    write("grad_rmat4_d8.txt", "dL/dA, dL/dB of L = sum(C o W) on R-MAT scale 4 x Bernoulli(16 x 8, 0.3), seed 20240813",
          {"a_rp": ("i", a.rp), "a_ci": ("i", a.ci), "a_val": ("f", a.val), "b_rp": ("i", b.rp),
           "b_ci": ("i", b.ci), "b_val": ("f", b.val), "g": ("f", g), "grad_a": ("f", ga), "grad_b": ("f", gb)})


if __name__ == "__main__":
    spgemm_case()
    bfs_case()
    grad_case()
