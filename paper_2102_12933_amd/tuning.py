"""Autotuning of the batched schedule and tile shape.

The kernel variants of a single solver are tuned inside the library
(fdu_autotune).  For a batch, this module times candidate (schedule, edges per
thread, vertex passes, vertex mode) settings with HIP events on the
instances' real data and keeps the fastest; results are cached in a JSON file
keyed by the device name and the batch's size class, so a later run with the
same shape reuses the choice without timing.
"""
from __future__ import annotations

import json
import os

import torch

# (schedule, edges per thread, vertex passes, vertex mode)
CANDIDATES = [(0, 4, 8, 2), (0, 16, 16, 2), (0, 4, 8, 3), (0, 16, 8, 3), (0, 1, 8, 3), (1, 4, 8, 0), (1, 4, 8, 2),
              (1, 16, 16, 1), (1, 4, 8, 3), (1, 16, 8, 3), (2, 4, 8, 0)]
CACHE = os.environ.get("FDU_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fdu_tuning.json"))


def _key(batch) -> str:
    nv = sum(s.nv_real for s in batch.solvers)
    size_class = int(round(float(nv) ** 0.5 / 64.0))          # ~sqrt(V) in units of 64
    name = torch.cuda.get_device_properties(0).name or "gpu"
    return f"{name}|n{len(batch.solvers)}|s{size_class}"


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune_batch(batch, cfl: float, reps: int = 3, use_cache: bool = True, candidates=CANDIDATES):
    """Time every candidate with `reps` eager steps (after one warm step) and set
    the fastest.  The instances' states advance during tuning; callers reset
    them afterwards.  Returns (best, {candidate: ms per step})."""
    key = _key(batch)
    cache = _load() if use_cache else {}
    if key in cache:
        best = tuple(cache[key]["best"])
        batch.set_schedule(*best)
        return best, {}
    times = {}
    for cand in candidates:
        batch.set_schedule(*cand)
        batch.step(cfl)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            batch.step(cfl)
        e1.record()
        e1.synchronize()
        times[cand] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    batch.set_schedule(*best)
    if use_cache:
        cache[key] = {"best": list(best), "ms_per_step": {",".join(map(str, c)): t for c, t in times.items()}}
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return best, times
