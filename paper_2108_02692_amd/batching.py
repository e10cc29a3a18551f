"""Mixed multi-stripe batches on one persistent launch.

A batch mixes codecs, block sizes and encode/decode work.  Programs are
compiled once per (codec, erasure set, level, slot budget) and kept in a
``ProgramCache`` whose bytecode stays resident on the device; stripes are
described by plain tuples and turned into one ``ec_batch`` (a HIP graph of a
counter reset and the persistent executor).
"""
from __future__ import annotations

import itertools
import os
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import LEVEL_PLAIN, SCHED_PUSH, ec_batch_build, ec_compile_slp, ec_matrix_cauchy, ec_program_upload_many

CODECS_DEFAULT = ((6, 3), (10, 4), (12, 4), (14, 4))


@dataclass(frozen=True)
class StripeSpec:
    """One stripe of a mixed workload: codec, block size, erasure set
    (empty = encode)."""
    n: int
    p: int
    block_bytes: int
    erased: tuple = ()

    @property
    def n_in(self):
        return self.n

    @property
    def n_out(self):
        return len(self.erased) if self.erased else self.p


class ProgramCache:
    """Compiled programs keyed by (n, p, erased, level, slots, scheduler);
    thread-safe.  The generator of each codec is ``generator_fn(n, p)``
    ((n+p) x n rows), by default the library's Cauchy matrix.  The
    (n, p, erased) in ``native_keys`` are compiled with the native kernels
    ``native`` (EC_NATIVE_* bits) as well."""

    def __init__(self, level: int = LEVEL_PLAIN, slots: int = 40, generator_fn=None, scheduler: int = SCHED_PUSH,
                 native_keys=(), native: int = 0):
        self.level = level
        self.slots = slots
        self.scheduler = scheduler
        self.native_keys = {(n, p, tuple(er)) for n, p, er in native_keys}
        self.native = native
        self._gen_fn = generator_fn or ec_matrix_cauchy
        self._progs = {}
        self._gens = {}
        self._lock = threading.Lock()

    def generator(self, n, p):
        with self._lock:
            g = self._gens.get((n, p))
            if g is None:
                g = self._gens[(n, p)] = [[int(x) for x in row] for row in self._gen_fn(n, p)]
            return g

    def get(self, n, p, erased=()):
        key = (n, p, tuple(erased), self.level, self.slots, self.scheduler)
        with self._lock:
            prog = self._progs.get(key)
        if prog is None:
            native = self.native if (n, p, tuple(erased)) in self.native_keys else 0
            prog = ec_compile_slp(n, p, self.generator(n, p), list(erased), level=self.level,
                                  slot_budget=self.slots, scheduler=self.scheduler, native=native)
            with self._lock:
                prog = self._progs.setdefault(key, prog)
        return prog

    def warm(self, keys, threads=None):
        """Compile every (n, p, erased) in ``keys`` on host threads."""
        threads = threads or min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda k: self.get(*k), keys))

    def upload(self):
        """Copy every cached program's records to the current device (one
        device allocation at most for all of them)."""
        with self._lock:
            progs = list(self._progs.values())
        ec_program_upload_many(progs)

    def all_patterns(self, n, p):
        return [()] + [c for r in range(1, p + 1) for c in itertools.combinations(range(n + p), r)]

    def __len__(self):
        return len(self._progs)


def mixed_specs(count: int, seed: int, codecs=CODECS_DEFAULT, lo=4096, hi=4 << 20, quantum=512,
                encode_frac=0.7):
    """The batched workload: codecs uniform over ``codecs``, block sizes
    log-uniform on [lo, hi] in multiples of ``quantum``, a fraction
    ``encode_frac`` of encodes and, for decodes, an erasure set uniform over
    all non-empty sets of at most p blocks."""
    from .workloads import log_uniform_sizes
    rng = np.random.default_rng(seed)
    sizes = log_uniform_sizes(rng, count, lo, hi, quantum)
    pats = {}
    out = []
    for k in range(count):
        n, p = codecs[int(rng.integers(len(codecs)))]
        erased = ()
        if rng.random() >= encode_frac:
            key = (n, p)
            if key not in pats:
                pats[key] = [c for r in range(1, p + 1) for c in itertools.combinations(range(n + p), r)]
            erased = pats[key][int(rng.integers(len(pats[key])))]
        out.append(StripeSpec(n, p, int(sizes[k]), erased))
    return out


def mixed_workload(count: int, seed: int = 4, hi: int = 4 << 20, pool_bytes: int | None = None,
                   slice_seed: int = 5):
    """The batched benchmark's stripes and buffers: ``mixed_specs(count,
    seed, hi=hi)``; the input blocks lie in one pool of seeded random bytes
    on the device.  With ``pool_bytes`` None (the benchmark) every input
    block has its own 4 KiB-aligned range of a pool as large as all of
    them, in stripe order, as distinct objects would: no byte is read twice
    in a launch, so no read can be served by the memory-side cache.  With
    ``pool_bytes`` (tests that want a small host copy) each input block is a
    4 KiB-aligned slice of a pool of that size at an offset drawn from
    ``slice_seed``, and stripes share bytes.  Every output block has its own
    range of one output buffer.  Returns (specs, pool, inputs, outputs,
    out_buf) with inputs[k] / outputs[k] lists of tensor views in program
    argument order."""
    import torch
    specs = mixed_specs(count, seed=seed, hi=hi)
    def span(b):
        return -(-b // 4096) * 4096
    distinct = pool_bytes is None
    if distinct:
        pool_bytes = sum(s.n_in * span(s.block_bytes) for s in specs)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pool = torch.randint(0, 256, (pool_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    rng = np.random.default_rng(slice_seed)
    out_total = sum(s.n_out * s.block_bytes for s in specs)
    out_buf = torch.empty(out_total, dtype=torch.uint8, device="cuda")
    inputs, outputs, off, cursor = [], [], 0, 0
    for s in specs:
        if distinct:
            offs = [cursor + i * span(s.block_bytes) for i in range(s.n_in)]
            cursor += s.n_in * span(s.block_bytes)
        else:
            top = (pool_bytes - s.block_bytes) // 4096
            offs = (rng.integers(0, top, s.n_in) * 4096).tolist()
        inputs.append([pool[o:o + s.block_bytes] for o in offs])
        outputs.append([out_buf[off + j * s.block_bytes: off + (j + 1) * s.block_bytes] for j in range(s.n_out)])
        off += s.n_out * s.block_bytes
    return specs, pool, inputs, outputs, out_buf


def build_batch(specs, cache: ProgramCache, inputs, outputs, tile_bytes=0, stream=None):
    """``inputs[k]`` / ``outputs[k]``: device buffers (or pointers) of stripe
    k, in the order of its program's in_blocks / out_blocks."""
    stripes = []
    for k, s in enumerate(specs):
        prog = cache.get(s.n, s.p, s.erased)
        stripes.append((prog, inputs[k], outputs[k], s.block_bytes))
    return ec_batch_build(stripes, tile_bytes=tile_bytes, stream=stream)
