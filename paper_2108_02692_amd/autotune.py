"""Autotuner for batched and single-stripe launches.

For a workload key (codec mix and size class, or one stripe's codec, erasure
set and block size) it times every candidate (program level, register slot
budget, strip scheduler and, for batches, tile width per work item: the
unroll of the batch kernel's persistent loop, the consecutive tiles a wave
runs per item) on the real launch, keeps the fastest and records it in a
JSON cache so later runs reuse the choice without timing again.
"""
from __future__ import annotations

import json
import os
import time

from . import LEVEL_CO_FU_SCHED, LEVEL_PLAIN, SCHED_GREEDY, SCHED_PUSH, ec_compile_slp, ec_decode, ec_encode
from .batching import ProgramCache, build_batch

# (level, slot budget, tile bytes per work item, strip scheduler)
DEFAULT_CANDIDATES = (
    (LEVEL_CO_FU_SCHED, 38, 1024, SCHED_PUSH), (LEVEL_CO_FU_SCHED, 38, 4096, SCHED_PUSH),
    (LEVEL_CO_FU_SCHED, 38, 16384, SCHED_PUSH), (LEVEL_CO_FU_SCHED, 44, 1024, SCHED_PUSH),
    (LEVEL_PLAIN, 38, 1024, SCHED_PUSH), (LEVEL_PLAIN, 38, 4096, SCHED_PUSH),
    (LEVEL_CO_FU_SCHED, 38, 1024, SCHED_GREEDY), (LEVEL_CO_FU_SCHED, 44, 1024, SCHED_GREEDY),
    (LEVEL_PLAIN, 38, 1024, SCHED_GREEDY),
)
# (level, slot budget (0 = the compiler's rule), strip scheduler[, native
# kernel]) for one stripe
STRIPE_CANDIDATES = (
    (LEVEL_CO_FU_SCHED, 0, SCHED_PUSH), (LEVEL_CO_FU_SCHED, 0, SCHED_GREEDY),
    (LEVEL_PLAIN, 0, SCHED_PUSH), (LEVEL_PLAIN, 0, SCHED_GREEDY),
)
# the same with the programs' native kernels beside the interpreter (each
# native candidate costs a run-time compile of about a second)
STRIPE_CANDIDATES_NATIVE = STRIPE_CANDIDATES + (
    (LEVEL_CO_FU_SCHED, 0, SCHED_PUSH, True), (LEVEL_CO_FU_SCHED, 0, SCHED_GREEDY, True),
    (LEVEL_PLAIN, 0, SCHED_PUSH, True), (LEVEL_PLAIN, 36, SCHED_PUSH, True),
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
    for level, slots, tile, sched in candidates:
        t0 = time.time()
        cache = ProgramCache(level=level, slots=slots, scheduler=sched)
        cache.warm({(s.n, s.p, s.erased) for s in specs})
        batch = build_batch(specs, cache, inputs, outputs, tile_bytes=tile, stream=stream)
        ms = time_batch(batch, stream, steps=steps)
        batch.free()
        r = {"level": level, "slots": slots, "tile_bytes": tile, "scheduler": sched, "ms": ms,
             "setup_s": time.time() - t0}
        results.append(r)
        if log:
            log(r)
    best = min(results, key=lambda r: r["ms"])
    table[key] = best
    _store(path, table)
    return best, results


def _time_launches(fn, stream, steps=20, warmup=5):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune_stripe(n, p, gen, erased, inputs, outputs, block_bytes, stream, candidates=STRIPE_CANDIDATES,
                path=CACHE_PATH, retune=False, time_fn=None):
    """One stripe's launch: times each (level, slot budget, scheduler[,
    native]) on the caller's buffers (``inputs`` in the program's in_blocks
    order, which is the same for every candidate) and returns (best dict,
    table of all timings), the choice cached under the codec, erasure set
    and block size.  ``time_fn(launch)`` gives the ms per launch (default:
    5 untimed launches, then the mean of 20)."""
    key = "stripe-RS(%d,%d)-%s-%d" % (n, p, ",".join(map(str, erased)) or "enc", block_bytes)
    table = _load(path)
    if key in table and not retune:
        return table[key], None
    time_fn = time_fn or (lambda f: _time_launches(f, stream))
    results = []
    for cand in candidates:
        level, slots, sched = cand[:3]
        native = bool(cand[3]) if len(cand) > 3 else False
        prog = ec_compile_slp(n, p, gen, list(erased), level=level, slot_budget=slots, scheduler=sched,
                              native=native)
        run = ec_decode if erased else ec_encode
        ms = time_fn(lambda: run(prog, inputs, outputs, block_bytes, stream))
        results.append({"level": level, "slots": prog.info["slots"], "scheduler": sched, "native": native,
                        "ms": ms, "records": prog.info["n_records"], "ops": prog.info["n_ops"]})
    best = min(results, key=lambda r: r["ms"])
    table[key] = best
    _store(path, table)
    return best, results
