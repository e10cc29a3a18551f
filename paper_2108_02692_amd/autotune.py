"""Autotuner for batched launches.

For a workload key (codec mix and size class) it times every candidate
(program level, register slot budget, tile width per work item) on the real
batch, keeps the fastest and records it in a JSON cache so later runs reuse
the choice without timing again.
"""
from __future__ import annotations

import json
import os
import time

from . import LEVEL_CO_FU_SCHED, LEVEL_PLAIN
from .batching import ProgramCache, build_batch

DEFAULT_CANDIDATES = (
    (LEVEL_CO_FU_SCHED, 38, 1024), (LEVEL_CO_FU_SCHED, 38, 4096), (LEVEL_CO_FU_SCHED, 38, 16384),
    (LEVEL_CO_FU_SCHED, 44, 1024), (LEVEL_PLAIN, 38, 1024), (LEVEL_PLAIN, 38, 4096),
)
CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch(batch, stream, steps=3, warmup=1):
    import torch
    for _ in range(warmup):
        batch.launch(stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        batch.launch(stream)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune(key, specs, inputs, outputs, stream, candidates=DEFAULT_CANDIDATES, steps=3, path=CACHE_PATH,
         retune=False, log=None):
    """Returns (best candidate dict, table of all timings).  ``key`` names the
    workload in the cache; a cached choice is returned without timing unless
    ``retune``."""
    table = _load(path)
    if key in table and not retune:
        return table[key], None
    results = []
    for level, slots, tile in candidates:
        t0 = time.time()
        cache = ProgramCache(level=level, slots=slots)
        cache.warm({(s.n, s.p, s.erased) for s in specs})
        batch = build_batch(specs, cache, inputs, outputs, tile_bytes=tile, stream=stream)
        ms = time_batch(batch, stream, steps=steps)
        batch.free()
        r = {"level": level, "slots": slots, "tile_bytes": tile, "ms": ms, "setup_s": time.time() - t0}
        results.append(r)
        if log:
            log(r)
    best = min(results, key=lambda r: r["ms"])
    table[key] = best
    _store(path, table)
    return best, results
