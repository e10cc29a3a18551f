"""Serving loop: continuous batching of encode/decode requests.

Requests arrive on a Poisson clock.  The loop admits arrived requests while
their working set (input + output bytes) fits an HBM budget and a batch slot
is free, packs them into one persistent-kernel launch on that slot's stream,
and keeps doing so while earlier batches run, so requests admitted while
others are on the GPU overlap with them on the device.  Completion is
observed by polling each slot's event; latency is completion minus arrival
on the host clock.  Compiled programs for every erasure pattern of the
served codecs are built up front and stay resident on the device.

Workload (seeded): object sizes log-normal (median 256 KiB, sigma 1.0,
clipped to 4 KiB .. 64 MiB); RS(10,4) and RS(6,3) in a 3:1 ratio; 70%
encodes, 30% decodes with an erasure set drawn uniformly from all non-empty
sets of at most p blocks; an object of b bytes is n blocks of
ceil(b / n) bytes rounded up to 512.
"""
from __future__ import annotations

import bisect
import gc
import time
from dataclasses import dataclass, field

import numpy as np

from . import LEVEL_CO_FU_SCHED, Batch, ec_decode, ec_encode, ec_server_create
from .batching import ProgramCache

MAX_OBJECT = 64 << 20  # largest object served (bytes)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    n: int
    p: int
    erased: tuple
    block_bytes: int
    inputs: list = field(default_factory=list)   # device pointers (program in_blocks order)
    outputs: list = field(default_factory=list)  # device pointers, set on admission
    out_off: int = -1
    done: float = -1.0

    @property
    def n_out(self):
        return len(self.erased) if self.erased else self.p

    @property
    def bytes(self):
        return (self.n + self.n_out) * self.block_bytes


class FirstFit:
    """First-fit allocator over [0, size) with coalescing free ranges."""

    def __init__(self, size: int, align: int = 4096):
        self.align = align
        self.starts = [0]
        self.lens = [size]

    def alloc(self, n: int):
        n = (n + self.align - 1) // self.align * self.align
        for i, ln in enumerate(self.lens):
            if ln >= n:
                off = self.starts[i]
                if ln == n:
                    del self.starts[i], self.lens[i]
                else:
                    self.starts[i] += n
                    self.lens[i] -= n
                return off, n
        return -1, 0

    def free(self, off: int, n: int):
        i = bisect.bisect_left(self.starts, off)
        self.starts.insert(i, off)
        self.lens.insert(i, n)
        if i + 1 < len(self.starts) and self.starts[i] + self.lens[i] == self.starts[i + 1]:
            self.lens[i] += self.lens[i + 1]
            del self.starts[i + 1], self.lens[i + 1]
        if i > 0 and self.starts[i - 1] + self.lens[i - 1] == self.starts[i]:
            self.lens[i - 1] += self.lens[i]
            del self.starts[i], self.lens[i]


class Server:
    """Admission by HBM budget, ``n_slots`` batches in flight, each on its own
    stream with a reusable ``ec_batch``.  ``native=True`` (default) runs the
    loop in the library (``ec_server_run``); ``native=False`` runs the same
    loop in Python (the methods below), kept for comparison."""

    def __init__(self, budget_bytes=16 << 30, n_slots=4, max_batch=512, level=LEVEL_CO_FU_SCHED, slots=38,
                 tile_bytes=0, codecs=((10, 4), (6, 3)), warm=True, direct_single=True, native=True,
                 generator_fn=None):
        import torch
        self.torch = torch
        self.budget = budget_bytes
        self.used = 0
        self.max_batch = max_batch
        self.tile_bytes = tile_bytes
        self.direct_single = direct_single
        self.cache = ProgramCache(level=level, slots=slots, generator_fn=generator_fn)
        if warm:
            self.cache.warm([(n, p, er) for n, p in codecs for er in self.cache.all_patterns(n, p)])
            # every program resident on the device before the clock starts
            self.cache.upload()
        self.arena = torch.empty(budget_bytes, dtype=torch.uint8, device="cuda")
        self.base = self.arena.data_ptr()
        self.batches = 0
        self.native = native
        if native:
            # streams, events, batches and their warm-up live in the library
            self._native = ec_server_create(self.arena, budget_bytes, budget_bytes, n_slots, max_batch)
            return
        self.heap = FirstFit(budget_bytes)
        self.slots = []
        # Work items per request: one per tile of a strip; the largest object
        # (64 MiB) over the fewest data blocks of the served codecs.
        max_items = max_batch * (-(-(MAX_OBJECT // min(n for n, _ in codecs)) // 8 // 1024) + 1)
        for _ in range(n_slots):
            b = Batch.create()
            b.reserve(max_batch, max_items)  # no allocation while serving
            self.slots.append({"stream": torch.cuda.Stream(), "batch": b, "event": torch.cuda.Event(),
                               "reqs": None})
        self._warm(codecs)

    def _warm(self, codecs):
        """One tiny encode per codec on every slot's stream, directly and as
        a batch, before any request: the first launches on a new stream (and
        of each kernel) take milliseconds, which the first requests would
        otherwise wait for.  Blocks of 128 B at the start of the (still
        empty) arena serve as inputs and outputs."""
        for n, p in codecs:
            prog = self.cache.get(n, p, ())
            ins = [self.base + 128 * i for i in range(n)]
            outs = [self.base + 128 * (n + j) for j in range(p)]
            for s in self.slots:
                ec_encode(prog, ins, outs, 128, s["stream"])
                s["batch"].set([(prog, ins, outs, 128)], tile_bytes=self.tile_bytes, stream=s["stream"])
                s["batch"].enqueue(s["stream"])
        self.torch.cuda.synchronize()

    def try_admit(self, req: Request) -> bool:
        out_bytes = req.n_out * req.block_bytes
        if self.used + req.bytes > self.budget:
            return False
        off, got = self.heap.alloc(out_bytes)
        if off < 0:
            return False
        req.out_off = off
        req._alloc = got
        req.outputs = [self.base + off + j * req.block_bytes for j in range(req.n_out)]
        self.used += req.bytes
        return True

    def free_slot(self):
        for s in self.slots:
            if s["reqs"] is None:
                return s
        return None

    def launch(self, slot, reqs):
        if len(reqs) == 1 and self.direct_single:
            # one request: a plain launch, without the batch's tables and
            # work counter (measured: 38 us from call to completion against
            # 58 us through a batch, for 26 KiB blocks)
            r = reqs[0]
            prog = self.cache.get(r.n, r.p, r.erased)
            (ec_decode if r.erased else ec_encode)(prog, r.inputs, r.outputs, r.block_bytes, slot["stream"])
        else:
            stripes = [(self.cache.get(r.n, r.p, r.erased), r.inputs, r.outputs, r.block_bytes) for r in reqs]
            slot["batch"].set(stripes, tile_bytes=self.tile_bytes, stream=slot["stream"])
            slot["batch"].enqueue(slot["stream"])
        slot["event"].record(slot["stream"])
        slot["reqs"] = reqs
        self.batches += 1

    def retire(self, now_fn, on_done=None):
        done = []
        for s in self.slots:
            if s["reqs"] is not None and s["event"].query():
                t = now_fn()
                for r in s["reqs"]:
                    r.done = t
                if on_done is not None:
                    on_done(s["reqs"])
                for r in s["reqs"]:
                    self.heap.free(r.out_off, r._alloc)
                    self.used -= r.bytes
                done.extend(s["reqs"])
                s["reqs"] = None
        return done

    def serve(self, requests, t0=None, realtime=True, on_done=None, idle_sleep_s=0.0):
        """Run requests (sorted by arrival) to completion; returns wall time.
        ``on_done(reqs)`` sees each finished batch while its outputs are still
        in the arena; ``realtime=False`` admits every request at once.
        ``idle_sleep_s`` (Python loop only; the native loop always polls):
        pause when nothing can be done.  The default 0 keeps polling, which
        holds one host core; a sleep of even 20 us costs its own wake-up
        latency twice per request (measured at 20k req/s: p50 0.135 ms with
        it, 0.071 ms polling).  ``t0`` (Python loop only): the clock's zero."""
        if self.native:
            return self._serve_native(requests, realtime, on_done)
        now_fn = (lambda: time.perf_counter() - t0)
        if t0 is None:
            t0 = time.perf_counter()
        i, n, finished = 0, len(requests), 0
        while finished < n:
            finished += len(self.retire(now_fn, on_done))
            slot = self.free_slot()
            if slot is not None and i < n:
                now = now_fn() if realtime else float("inf")
                batch = []
                while i < n and requests[i].arrival <= now and len(batch) < self.max_batch:
                    if not self.try_admit(requests[i]):
                        if not batch and all(s["reqs"] is None for s in self.slots):
                            raise ValueError("request %d needs %d bytes, over the %d-byte budget"
                                             % (requests[i].rid, requests[i].bytes, self.budget))
                        break
                    batch.append(requests[i])
                    i += 1
                if batch:
                    self.launch(slot, batch)
                    continue
            if idle_sleep_s > 0 and (slot is None or i >= n or requests[i].arrival > now_fn()):
                time.sleep(idle_sleep_s)
        return now_fn()


    def _serve_native(self, requests, realtime, on_done):
        """The same loop in the library: the clock starts inside the call,
        after the programs, tables and kernels are ready."""
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


def make_requests(duration_s: float, rate: float, seed: int, pool_ptr: int, pool_bytes: int,
                  ratio_10_4=0.75, encode_frac=0.7, median=256 << 10, sigma=1.0, lo=4 << 10, hi=MAX_OBJECT):
    """Seeded Poisson arrivals over ``duration_s``; inputs point into a
    read-only device pool."""
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
        offs = rng.integers(0, (pool_bytes - bb) // 4096, n) * 4096
        reqs.append(Request(len(reqs), t, n, p, erased, bb, inputs=[pool_ptr + int(o) for o in offs]))
    return reqs


def run(duration_s=2.0, rate=20000.0, seed=7, budget_bytes=16 << 30, n_slots=4, max_batch=512, slots=38,
        idle_sleep_s=0.0, native=True):
    """The serving benchmark: returns throughput and latency percentiles."""
    import torch
    pool_bytes = 1 << 30
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pool = torch.randint(0, 256, (pool_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    t_setup = time.perf_counter()
    server = Server(budget_bytes=budget_bytes, n_slots=n_slots, max_batch=max_batch, slots=slots, native=native)
    setup_s = time.perf_counter() - t_setup
    reqs = make_requests(duration_s, rate, seed, pool.data_ptr(), pool_bytes)
    torch.cuda.synchronize()
    # no collector pauses inside the timed loop (the request objects are
    # all allocated beforehand)
    gc.collect()
    gc.disable()
    try:
        wall = server.serve(reqs, idle_sleep_s=idle_sleep_s)
    finally:
        gc.enable()
    torch.cuda.synchronize()
    lat = np.array([r.done - r.arrival for r in reqs])
    in_bytes = sum(r.n * r.block_bytes for r in reqs)
    batches = server.batches
    # drain: the same requests all present at once, as fast as the loop and
    # the device take them (the capacity behind the latencies above)
    for r in reqs:
        r.arrival, r.done = 0.0, -1.0
    gc.collect()
    gc.disable()
    try:
        drain = server.serve(reqs, realtime=False, idle_sleep_s=idle_sleep_s)
    finally:
        gc.enable()
    torch.cuda.synchronize()
    res = {"loop": "native" if native else "python", "requests": len(reqs), "rate_req_s": rate,
           "arrival_s": duration_s, "wall_s": wall,
           "GB_s": in_bytes / wall / 1e9, "in_bytes": in_bytes,
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "batches": batches,
           "budget_bytes": budget_bytes, "inflight_slots": n_slots, "programs": len(server.cache),
           "setup_s": setup_s, "drain_s": drain, "drain_GB_s": in_bytes / drain / 1e9}
    del server, pool
    return res
