"""Empirical tuning of the accumulator, the work-class thresholds and the
lane-group width.

The paper tunes its tile width and height empirically and ships defaults
(Sec. V-A, V-B), and picks the accumulator by d: a dense accumulator (SPA)
up to d = 1024, a hash above (Sec. III-C). On the GPU the knobs are the
accumulator (the LDS strip or the hash path; only the hash for d > 1024),
the group width that streams a B row and the product-count thresholds that
send a row to a lane group, a wavefront, a workgroup, or split chunks. None
of them changes the structure of C; values are FP64 sums rounded once under
every choice (within the tolerance of each other, nearly always identical).

The search is a coordinate descent: the accumulator first, then (for the LDS
strip) the group width, the product layout (per B row or flat), the
light-row threshold and the wavefront / split thresholds, each candidate
timed on the instance's numeric phase (its symbolic phase rebinds rows for
the candidate). Results are cached per feature key in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .api import DeviceCsr, numeric, symbolic

GROUP_LANES = (8, 16, 32, 64)
LIGHT_MAX = (256, 512, 2048, 8192)
WAVE_SPLIT = ((8192, 65536), (16384, 131072), (65536, 262144), (131072, 524288))
PRODUCTS = ("rows", "flat")
ACCUMULATORS = ("lds", "hash")
DEFAULT = {"accumulator": "auto", "group_lanes": 0, "light_max_flops": 1024, "wave_max_flops": 65536,
           "split_flops": 262144, "products": 0}


def features(A: DeviceCsr, B: DeviceCsr, flops: int) -> str:
    """Tuning key: d class, log2 of mean products per non-empty row, log2 of
    the longest A row, and B's density class."""
    n = max(A.nrows, 1)
    arow = torch.diff(A.rowptr)
    nonempty = max(int((arow > 0).sum()), 1)
    maxrow = int(arow.max()) if A.nrows else 0
    dens = B.nnz / max(1, B.nrows * max(B.ncols, 1))
    return "d{}_f{}_m{}_b{}".format(
        int(math.ceil(math.log2(max(B.ncols, 1)))), int(round(math.log2(max(flops / nonempty, 1)))),
        int(round(math.log2(max(maxrow, 1)))), int(round(math.log2(max(dens * 1000, 1)))) if n else 0)


def _time_numeric(A, B, tuning, reps=3):
    plan, rp, nnz = symbolic(A, B, "plus_times", tuning=tuning)
    ci = torch.empty(max(nnz, 1), dtype=torch.int32, device=A.rowptr.device)
    cv = torch.empty(max(nnz, 1), dtype=torch.float32, device=A.rowptr.device)
    numeric(plan, A, B, ci, cv)  # warm
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        s.record()
        numeric(plan, A, B, ci, cv)
        e.record()
        e.synchronize()
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2], plan


def _strip_class(d: int) -> int:
    """LDS strip size class of the batched numeric phase: the smallest power
    of two >= max(d, 32)."""
    c = 32
    while c < d:
        c <<= 1
    return c


class Autotuner:
    def __init__(self, path: str | None = None):
        self.path = path
        self.cache = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def save(self):
        if self.path:
            os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def tune(self, A: DeviceCsr, B: DeviceCsr, reps: int = 3) -> dict:
        t0, plan = _time_numeric(A, B, DEFAULT, reps)
        key = features(A, B, plan.stats()["flops"])
        if key in self.cache:
            return dict(self.cache[key])
        best, best_t = dict(DEFAULT), t0
        if B.ncols <= 1024:  # both accumulators apply; above, only the hash
            for acc in ACCUMULATORS:
                cand = dict(best, accumulator=acc)
                t, _ = _time_numeric(A, B, cand, reps)
                if t < best_t:
                    best, best_t = cand, t
        if best["accumulator"] == "hash" or B.ncols > 1024:  # the other knobs are the strip's
            best["ms"] = round(best_t, 4)
            self.cache[key] = best
            return dict(best)
        for gl in GROUP_LANES:
            cand = dict(best, group_lanes=gl)
            t, _ = _time_numeric(A, B, cand, reps)
            if t < best_t:
                best, best_t = cand, t
        for pl in PRODUCTS:
            cand = dict(best, products=pl)
            t, _ = _time_numeric(A, B, cand, reps)
            if t < best_t:
                best, best_t = cand, t
        for lm in LIGHT_MAX:
            cand = dict(best, light_max_flops=lm)
            t, _ = _time_numeric(A, B, cand, reps)
            if t < best_t:
                best, best_t = cand, t
        for wm, sp in WAVE_SPLIT:
            cand = dict(best, wave_max_flops=wm, split_flops=sp)
            t, _ = _time_numeric(A, B, cand, reps)
            if t < best_t:
                best, best_t = cand, t
        best["ms"] = round(best_t, 4)
        self.cache[key] = best
        return dict(best)

    def tune_batch(self, pairs, reps: int = 3) -> list:
        """Thresholds, group width and product layout for a batch, timed on
        the whole batched run. First one setting for every instance
        (coordinate descent as in tune(), same candidate lists); then, class
        by class of instances with the same LDS strip size (the batched
        numeric phase runs each such class in launches of its own), the same
        descent for that class's instances alone. Cached under the
        instance keys in order."""
        from .batched import Batched

        if not pairs:
            return []
        # products per instance from the library (its symbolic pass at plan time)
        fls = Batched(pairs).flops()
        keys = [features(A, B, fl) for (A, B), fl in zip(pairs, fls)]
        key = "batch:" + "|".join(keys)  # in instance order: the settings are per instance
        if key in self.cache:
            best = dict(self.cache[key])
        else:
            def run_ms(cfgs):
                bt = Batched(pairs, cfgs)
                bt.run()
                s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                times = []
                for _ in range(reps):
                    s.record()
                    bt.run()
                    e.record()
                    e.synchronize()
                    times.append(s.elapsed_time(e))
                times.sort()
                return times[len(times) // 2]

            def descend(cfgs, idx, t0):
                """Coordinate descent over the settings of instances idx."""
                best_t = t0
                for values in ([{"group_lanes": g} for g in GROUP_LANES],
                               [{"products": p} for p in PRODUCTS],
                               [{"light_max_flops": m} for m in LIGHT_MAX],
                               [{"wave_max_flops": w, "split_flops": sp} for w, sp in WAVE_SPLIT]):
                    for change in values:
                        cand = [dict(c, **change) if i in idx else c for i, c in enumerate(cfgs)]
                        t = run_ms(cand)
                        if t < best_t:
                            cfgs, best_t = cand, t
                return cfgs, best_t

            everyone = set(range(len(pairs)))
            cfgs = [dict(DEFAULT) for _ in pairs]
            cfgs, best_t = descend(cfgs, everyone, run_ms(cfgs))
            for cls in sorted({_strip_class(B.ncols) for _, B in pairs}):
                idx = {i for i, (_, B) in enumerate(pairs) if _strip_class(B.ncols) == cls}
                if len(idx) < len(pairs):
                    cfgs, best_t = descend(cfgs, idx, best_t)
            best = {"per_instance": cfgs, "ms": round(best_t, 4)}
            self.cache[key] = best
        return [{k: v for k, v in c.items() if k != "ms"} for c in best["per_instance"]]

