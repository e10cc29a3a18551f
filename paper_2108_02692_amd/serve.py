"""Serving: the seeded request workload and the library's serving loop.

Requests arrive on a Poisson clock.  The loop (``ec_server_run``, C++)
admits arrived requests while their working set (input + output bytes) fits
an HBM budget, spreads their work over the free launch slots, packs each
slot's share into one launch on that slot's stream, and keeps doing so while
earlier launches run, so requests admitted while others are on the GPU
overlap with them on the device.  Completion is observed by polling each
slot's event; latency is completion minus arrival on the host clock.
Compiled programs for every erasure pattern of the served codecs are built
up front and stay resident on the device.

Workload (seeded): object sizes log-normal (median 256 KiB, sigma 1.0,
clipped to 4 KiB .. 64 MiB); RS(10,4) and RS(6,3) in a 3:1 ratio; 70%
encodes, 30% decodes with an erasure set drawn uniformly from all non-empty
sets of at most p blocks; an object of b bytes is n blocks of
ceil(b / n) bytes rounded up to 512.
"""
from __future__ import annotations

import gc
import time
from dataclasses import dataclass, field

import numpy as np

from . import LEVEL_CO_FU_SCHED, NATIVE_BLOCKS, NATIVE_PAIRS, NATIVE_WHOLE, ec_batch_build, ec_server_create
from .batching import ProgramCache

MAX_OBJECT = 64 << 20  # largest object served (bytes)
DEFAULT_MAX_BATCH = 2048  # requests per launch at most


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    n: int
    p: int
    erased: tuple
    block_bytes: int
    inputs: list = field(default_factory=list)   # device pointers (program in_blocks order)
    outputs: list = field(default_factory=list)  # device pointers of the outputs, set when reported done
    out_off: int = -1
    done: float = -1.0

    @property
    def n_out(self):
        return len(self.erased) if self.erased else self.p

    @property
    def bytes(self):
        return (self.n + self.n_out) * self.block_bytes


class Server:
    """The library's serving loop (``ec_server_run``) with its program cache
    and output arena: every erasure pattern of the served codecs compiled and
    on the device before the clock starts; admission by HBM budget,
    ``n_slots`` launches in flight, each of at most ``max_batch`` requests.
    With ``native_encodes`` the codecs' encode programs (most requests) also
    get native kernels (whole program, pair parts and block parts), which
    a launch of one request runs; batches and decodes keep the
    interpreter."""

    def __init__(self, budget_bytes=16 << 30, n_slots=4, max_batch=DEFAULT_MAX_BATCH, level=LEVEL_CO_FU_SCHED,
                 slots=38, codecs=((10, 4), (6, 3)), warm=True, generator_fn=None, native_encodes=False):
        import torch
        self.budget = budget_bytes
        self.cache = ProgramCache(level=level, slots=slots, generator_fn=generator_fn,
                                  native_keys=[(n, p, ()) for n, p in codecs] if native_encodes else (),
                                  native=NATIVE_WHOLE | NATIVE_PAIRS | NATIVE_BLOCKS)
        if warm:
            self.cache.warm([(n, p, er) for n, p in codecs for er in self.cache.all_patterns(n, p)])
            # every program resident on the device before the clock starts
            self.cache.upload()
        self.arena = torch.empty(budget_bytes, dtype=torch.uint8, device="cuda")
        self.base = self.arena.data_ptr()
        self.batches = 0
        self._native = ec_server_create(self.arena, budget_bytes, budget_bytes, n_slots, max_batch)

    def serve(self, requests, realtime=True, on_done=None):
        """Run requests (sorted by arrival) to completion; returns the wall
        time of the run (the clock starts inside the library, once programs,
        tables and kernels are ready).  ``on_done(reqs)`` sees each finished
        launch while its outputs are still in the arena; ``realtime=False``
        admits every request at once."""
        reqs = [(r.arrival, self.cache.get(r.n, r.p, r.erased), r.inputs, r.block_bytes) for r in requests]
        cb = None
        if on_done is not None:
            def cb(ids, offs):
                done = [requests[i] for i in ids]
                for r, off in zip(done, offs):
                    r.out_off = off
                    r.outputs = [self.base + off + j * r.block_bytes for j in range(r.n_out)]
                on_done(done)
        done_s, offs, wall, nb = self._native.run(reqs, realtime=realtime, on_done=cb)
        for r, t, off in zip(requests, done_s, offs):
            r.done = t
            r.out_off = off
        self.batches += nb
        return wall


def make_requests(duration_s: float, rate: float, seed: int, pool_ptr: int | None = None, pool_bytes: int = 0,
                  ratio_10_4=0.75, encode_frac=0.7, median=256 << 10, sigma=1.0, lo=4 << 10, hi=MAX_OBJECT):
    """Seeded Poisson arrivals over ``duration_s``.  With ``pool_ptr`` the
    inputs are 4 KiB-aligned slices of that read-only device pool at offsets
    drawn with the arrivals (requests share bytes); without, they are left
    empty for ``place_inputs``."""
    import itertools
    rng = np.random.default_rng(seed)
    t, reqs = 0.0, []
    pats = {}
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        n, p = (10, 4) if rng.random() < ratio_10_4 else (6, 3)
        size = int(np.clip(rng.lognormal(np.log(median), sigma), lo, hi))
        bb = ((size + n - 1) // n + 511) // 512 * 512
        erased = ()
        if rng.random() >= encode_frac:
            if (n, p) not in pats:
                pats[(n, p)] = [c for r in range(1, p + 1) for c in itertools.combinations(range(n + p), r)]
            erased = pats[(n, p)][int(rng.integers(len(pats[(n, p)])))]
        inputs = []
        if pool_ptr is not None:
            offs = rng.integers(0, (pool_bytes - bb) // 4096, n) * 4096
            inputs = [pool_ptr + int(o) for o in offs]
        reqs.append(Request(len(reqs), t, n, p, erased, bb, inputs=inputs))
    return reqs


def _span(block_bytes: int) -> int:
    return -(-block_bytes // 4096) * 4096


def input_span(reqs) -> int:
    """Bytes of the pool ``place_inputs`` needs for ``reqs``."""
    return sum(r.n * _span(r.block_bytes) for r in reqs)


def place_inputs(reqs, pool_ptr: int, pool_bytes: int):
    """Gives every request's input blocks their own 4 KiB-aligned ranges of
    the device pool, in arrival order, as distinct objects would have: no
    two requests share input bytes, so no read is served by the memory-side
    cache from another request's read."""
    cur = 0
    for r in reqs:
        sp = _span(r.block_bytes)
        r.inputs = [pool_ptr + cur + i * sp for i in range(r.n)]
        cur += r.n * sp
    if cur > pool_bytes:
        raise ValueError("pool of %d bytes holds less than the %d bytes of inputs" % (pool_bytes, cur))


def batched_reference(server, requests, chunk=8192, reps=3):
    """The same requests through the batched path, with the server's own
    programs: batches of up to ``chunk`` stripes (outputs in one separate
    device buffer), launched back to back on one stream.  Returns GB/s of
    input of the fastest of ``reps`` passes."""
    import torch
    out = torch.empty(sum(r.n_out * r.block_bytes for r in requests), dtype=torch.uint8, device="cuda")
    base, off, stripes = out.data_ptr(), 0, []
    for r in requests:
        outs = [base + off + j * r.block_bytes for j in range(r.n_out)]
        off += r.n_out * r.block_bytes
        stripes.append((server.cache.get(r.n, r.p, r.erased), r.inputs, outs, r.block_bytes))
    stream = torch.cuda.current_stream()
    batches = [ec_batch_build(stripes[i:i + chunk], stream=stream) for i in range(0, len(stripes), chunk)]
    best = float("inf")
    try:
        for _ in range(reps):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for b in batches:
                b.launch(stream)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
    finally:
        for b in batches:
            b.free()
    return sum(r.n * r.block_bytes for r in requests) / best / 1e9


def _pinned(pin):
    """Context: the calling thread on one of its allowed CPUs (the serving
    loop polls; a move to another core or a neighbour's interruption shows
    as a latency outlier), its affinity restored afterwards."""
    import contextlib
    import os

    @contextlib.contextmanager
    def ctx():
        allowed = os.sched_getaffinity(0) if pin else None
        if allowed and len(allowed) > 1:
            os.sched_setaffinity(0, {sorted(allowed)[len(allowed) // 2]})
        try:
            yield
        finally:
            if allowed and len(allowed) > 1:
                os.sched_setaffinity(0, allowed)
    return ctx()


def run(duration_s=2.0, rate=20000.0, seed=7, budget_bytes=16 << 30, n_slots=4, max_batch=DEFAULT_MAX_BATCH,
        slots=38, drain=True, server=None, warm_up=None, pin=True):
    """The serving benchmark at one arrival rate: throughput, latency
    percentiles and requests per launch; with ``drain``, the same requests
    again all present at once (the capacity behind the latencies), and once
    more through the batched path (``batched_reference``).  A drain takes a
    few ms, all of it within the device's slower start after the near-idle
    real-time run: the first drain follows that run directly
    (``drain_cold_GB_s``); ``warm_up()``, if given, then keeps the device
    busy for a while (the caller's choice of work, finished before it
    returns) and the drain is run again (``drain_GB_s``).  With ``pin`` the
    loop's thread stays on one core while the clock runs (measured at 20k
    req/s: p99 within 0.002 ms from run to run on a box, 0.036-0.057 ms
    over three boxes, against 0.036-0.088 ms unpinned)."""
    import torch
    t_setup = time.perf_counter()
    if server is None:
        server = Server(budget_bytes=budget_bytes, n_slots=n_slots, max_batch=max_batch, slots=slots)
    setup_s = time.perf_counter() - t_setup
    # every request's inputs are bytes of their own (seeded random)
    reqs = make_requests(duration_s, rate, seed)
    pool_bytes = input_span(reqs)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pool = torch.randint(0, 256, (pool_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    place_inputs(reqs, pool.data_ptr(), pool_bytes)
    torch.cuda.synchronize()
    # no collector pauses inside the timed loop (the request objects are
    # all allocated beforehand)
    gc.collect()
    gc.disable()
    b0 = server.batches
    try:
        with _pinned(pin):
            wall = server.serve(reqs)
    finally:
        gc.enable()
    torch.cuda.synchronize()
    lat = np.array([r.done - r.arrival for r in reqs])
    in_bytes = sum(r.n * r.block_bytes for r in reqs)
    batches = server.batches - b0
    # the requests of one launch share its completion stamp (taken once per
    # launch), so grouping by it gives every launch's size
    _, per_launch = np.unique(np.array([r.done for r in reqs]), return_counts=True)
    res = {"loop": "native", "requests": len(reqs), "rate_req_s": rate, "arrival_s": duration_s, "wall_s": wall,
           "GB_s": in_bytes / wall / 1e9, "in_bytes": in_bytes,
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "batches": batches,
           "requests_per_launch": len(reqs) / max(1, batches),
           # over launches: median, 99th percentile and largest launch; over
           # requests: the share served by a launch of its own
           "launch_size_p50": float(np.percentile(per_launch, 50)),
           "launch_size_p99": float(np.percentile(per_launch, 99)), "launch_size_max": int(per_launch.max()),
           "requests_alone": float(np.sum(per_launch == 1) / len(reqs)),
           "budget_bytes": budget_bytes, "inflight_slots": n_slots, "max_batch": max_batch,
           "programs": len(server.cache), "setup_s": setup_s}
    if drain:
        def drain_once():
            for r in reqs:
                r.arrival, r.done = 0.0, -1.0
            gc.collect()
            gc.disable()
            b0 = server.batches
            try:
                with _pinned(pin):
                    d = server.serve(reqs, realtime=False)
            finally:
                gc.enable()
            torch.cuda.synchronize()
            return d, server.batches - b0
        d, launches = drain_once()
        res["drain_cold_GB_s"] = in_bytes / d / 1e9
        if warm_up is not None:
            warm_up()
            d, launches = drain_once()
        res.update({"drain_s": d, "drain_GB_s": in_bytes / d / 1e9, "drain_launches": launches})
        ref = batched_reference(server, reqs)
        res.update({"batched_same_GB_s": ref, "drain_vs_batched_same": in_bytes / d / 1e9 / ref})
    res["input_pool_bytes"] = pool_bytes
    del pool
    torch.cuda.empty_cache()
    return res
