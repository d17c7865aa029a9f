"""The oracle's pins must catch plausible mistakes.

Each case copies oracle.cpp to a temporary directory, plants one mistake by a
textual edit (a dropped term, a wrong index, a missing mask, an off-by-one
level, a dropped factor in a gradient), builds it with g++ and checks that the
pin named for it fails. Everything runs on the CPU.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests._util import dense, pattern, random_csr, rows_of

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.cpp")

MUTANTS = {
    # Eq. (1) with the last A term of every row dropped
    "dropped_term": ("for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {\n      int32_t k = aci[p];\n      double a = aval[p];",
                     "for (int32_t p = arp[i]; p + 1 < arp[i + 1]; ++p) {\n      int32_t k = aci[p];\n      double a = aval[p];"),
    # B row picked by the output row instead of A's column (a transposed operand)
    "wrong_index": ("      int32_t k = aci[p];\n      double a = aval[p];",
                    "      int32_t k = (int32_t)(i % (n > 0 ? n : 1));\n      double a = aval[p];"),
    # complement mask ignored
    "mask_ignored": ("for (int32_t q = mrp[i]; q < mrp[i + 1]; ++q) s.erase(mci[q]);",
                     "for (int32_t q = mrp[i]; q < mrp[i + 1]; ++q) (void)mci[q];"),
    # BFS levels one too high
    "level_off_by_one": ("for (int32_t j : F[i]) levels[i * (int64_t)d + j] = iter;",
                         "for (int32_t j : F[i]) levels[i * (int64_t)d + j] = iter + 1;"),
    # S updated with N before the difference is taken (wrong mask timing)
    "mask_after_update": ("      std::set<int32_t> next;  // F = N \\ S\n",
                          "      for (int32_t j : N[i]) S[i].insert(j);\n      std::set<int32_t> next;\n"),
    # dL/dB without the A factor
    "grad_b_dropped_factor": ("acc[{k, bci[q]}] += aval[p] * it->second;", "acc[{k, bci[q]}] += it->second;"),
    # dL/dA multiplying by G only
    "grad_a_dropped_factor": ("      s += it->second * bval[q];\n      }\n      grad_a[p] = s;",
                              "      s += it->second;\n      }\n      grad_a[p] = s;"),
    # merge: the last part dropped
    "merge_drops_last_part": ("  for (int32_t t = 0; t < count; ++t)\n    for (int64_t i = 0; i < n; ++i)",
                              "  for (int32_t t = 0; t + 1 < count; ++t)\n    for (int64_t i = 0; i < n; ++i)"),
    # column tile: the upper bound included
    "slice_upper_bound_included": ("if (aci[p] >= c0 && aci[p] < c1) {", "if (aci[p] >= c0 && aci[p] <= c1) {"),
    # embedding: attractive weight with the wrong sign
    "embed_attract_sign": ("const double w = a > 0 ? 1.0 - sig : (a < 0 ? -sig : 0.0);",
                           "const double w = a > 0 ? sig - 1.0 : (a < 0 ? -sig : 0.0);"),
    # embedding: sig and 1 - sig swapped
    "embed_sigmoid_swapped": ("const double w = a > 0 ? 1.0 - sig : (a < 0 ? -sig : 0.0);",
                              "const double w = a > 0 ? sig : (a < 0 ? sig - 1.0 : 0.0);"),
    # embedding: top-k by signed value instead of magnitude
    "embed_topk_signed": ("const float ax = std::fabs(u[x]), ay = std::fabs(u[y]);",
                          "const float ax = u[x], ay = u[y];"),
    # embedding: learning rate dropped
    "embed_lr_dropped": ("u[c] = (float)(zi[c] + lr * F[c]);", "u[c] = (float)(zi[c] + F[c]);"),
    # embedding: rows written back at once (later rows of a batch see them)
    "embed_no_minibatch": ("      oracle_embed_select(d, k, zi.data(), F.data(), lr, &new_ci[(i - r0) * k], &new_val[(i - r0) * k]);\n    }",
                           "      oracle_embed_select(d, k, zi.data(), F.data(), lr, &new_ci[(i - r0) * k], &new_val[(i - r0) * k]);\n"
                           "      std::copy(&new_ci[(i - r0) * k], &new_ci[(i - r0) * k] + k, zci + i * k);\n"
                           "      std::copy(&new_val[(i - r0) * k], &new_val[(i - r0) * k] + k, zval + i * k);\n    }"),
}


@pytest.fixture
def mutant(tmp_path, request):
    name = request.param
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new, 1)
    path = tmp_path / "oracle_mutant.cpp"
    path.write_text(src)
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(path), "-o", str(lib), "-lpthread"])
    oracle.use_library(str(lib))
    yield name
    oracle.use_library(None)


def _brute_force_pin_holds(seed=0):
    rng = np.random.default_rng(seed)
    ok = True
    for _ in range(6):
        n, d = 20, 12
        a = random_csr(rng, n, n, 0.25)
        b = random_csr(rng, n, d, 0.4)
        rp, ci, val = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
        out = np.zeros((n, d))
        out[rows_of(rp), ci] = val
        ok &= bool(np.allclose(out, dense(a) @ dense(b), rtol=1e-13, atol=0))
    return ok


def _mask_pin_holds():
    rng = np.random.default_rng(1)
    n, d = 20, 10
    a = random_csr(rng, n, n, 0.3)
    b = random_csr(rng, n, d, 0.3)
    m = random_csr(rng, n, d, 0.5)
    rp, ci = oracle.spgemm_bool(a.rp, a.ci, b.rp, b.ci, m.rp, m.ci)
    got = np.zeros((n, d), bool)
    got[rows_of(rp), ci] = True
    return bool(np.array_equal(got, ((pattern(a) @ pattern(b)) > 0) & ~(pattern(m) > 0)))


def _bfs_pin_holds():
    a, srcs = synth.workload_bfs(scale=7, d=8)
    return bool(np.array_equal(oracle.msbfs(a.rp, a.ci, srcs)[0], oracle.bfs_queue(a.rp, a.ci, srcs)))


def _grad_pin_holds():
    rng = np.random.default_rng(2)
    n, d = 15, 8
    a = random_csr(rng, n, n, 0.3, kind="normal")
    b = random_csr(rng, n, d, 0.4, kind="normal")
    rp, ci, _ = oracle.spgemm(a.rp, a.ci, a.val, b.rp, b.ci, b.val)
    gd = np.zeros((n, d))
    g = rng.standard_normal(len(ci))
    gd[rows_of(rp), ci] = g
    ga = oracle.grad_a(a.rp, a.ci, b.rp, b.ci, b.val, rp, ci, g)
    gb = oracle.grad_b(a.rp, a.ci, a.val, b.rp, b.ci, rp, ci, g)
    return bool(np.allclose(ga, (gd @ dense(b).T)[rows_of(a.rp), a.ci], rtol=1e-12, atol=1e-12) and
                np.allclose(gb, (dense(a).T @ gd)[rows_of(b.rp), b.ci], rtol=1e-12, atol=1e-12))


def _tile_pins_hold():
    from tests import test_oracle_tiles as t

    return t.slice_matches_dense() and t.merge_matches_dense()


def _embed_pins_hold():
    from tests import test_oracle_embed as e

    return e.force_is_loglik_gradient() and e.closed_form_holds() and e.topk_property_holds() and \
        e.minibatch_schedule_holds()


PIN_FOR = {
    "dropped_term": _brute_force_pin_holds,
    "wrong_index": _brute_force_pin_holds,
    "mask_ignored": _mask_pin_holds,
    "level_off_by_one": _bfs_pin_holds,
    "mask_after_update": _bfs_pin_holds,
    "grad_b_dropped_factor": _grad_pin_holds,
    "grad_a_dropped_factor": _grad_pin_holds,
    "merge_drops_last_part": _tile_pins_hold,
    "slice_upper_bound_included": _tile_pins_hold,
    "embed_attract_sign": _embed_pins_hold,
    "embed_sigmoid_swapped": _embed_pins_hold,
    "embed_topk_signed": _embed_pins_hold,
    "embed_lr_dropped": _embed_pins_hold,
    "embed_no_minibatch": _embed_pins_hold,
}


def test_pins_hold_for_the_real_oracle():
    for f in set(PIN_FOR.values()):
        assert f(), f.__name__


@pytest.mark.parametrize("mutant", sorted(MUTANTS), indirect=True)
def test_pin_catches_mutant(mutant):
    assert not PIN_FOR[mutant](), f"pin did not catch planted mistake {mutant}"
