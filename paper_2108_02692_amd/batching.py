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

from . import LEVEL_PLAIN, ec_batch_build, ec_compile_slp, ec_matrix_cauchy

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
    """Compiled programs keyed by (n, p, erased, level, slots); thread-safe.
    The generator is the Cauchy matrix of each codec."""

    def __init__(self, level: int = LEVEL_PLAIN, slots: int = 40):
        self.level = level
        self.slots = slots
        self._progs = {}
        self._gens = {}
        self._lock = threading.Lock()

    def generator(self, n, p):
        with self._lock:
            g = self._gens.get((n, p))
            if g is None:
                g = self._gens[(n, p)] = ec_matrix_cauchy(n, p)
            return g

    def get(self, n, p, erased=()):
        key = (n, p, tuple(erased), self.level, self.slots)
        with self._lock:
            prog = self._progs.get(key)
        if prog is None:
            prog = ec_compile_slp(n, p, self.generator(n, p), list(erased), level=self.level,
                                  slot_budget=self.slots)
            with self._lock:
                prog = self._progs.setdefault(key, prog)
        return prog

    def warm(self, keys, threads=None):
        """Compile every (n, p, erased) in ``keys`` on host threads."""
        threads = threads or min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda k: self.get(*k), keys))

    def upload(self):
        """Copy every cached program's records to the current device."""
        with self._lock:
            progs = list(self._progs.values())
        for prog in progs:
            prog.upload()

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


def build_batch(specs, cache: ProgramCache, inputs, outputs, tile_bytes=0, stream=None):
    """``inputs[k]`` / ``outputs[k]``: device buffers (or pointers) of stripe
    k, in the order of its program's in_blocks / out_blocks."""
    stripes = []
    for k, s in enumerate(specs):
        prog = cache.get(s.n, s.p, s.erased)
        stripes.append((prog, inputs[k], outputs[k], s.block_bytes))
    return ec_batch_build(stripes, tile_bytes=tile_bytes, stream=stream)
