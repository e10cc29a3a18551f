"""Seeded synthetic inputs (no coding arithmetic here).

The paper's workload is randomly generated data arrays; every block here is
uniform random bytes from a fixed seed.  Host blocks come from numpy's
PCG64 (``default_rng``); large device workloads are filled on the GPU by
torch's seeded generator.  Tests, the smoke check and the benchmark all draw
their inputs from this module, so the oracle and the GPU path see the same
bytes.
"""
from __future__ import annotations

import numpy as np


def host_blocks(k: int, block_bytes: int, seed: int):
    """k independent blocks of uniform random bytes (numpy uint8)."""
    rng = np.random.default_rng(seed)
    return [rng.integers(0, 256, block_bytes, dtype=np.uint8) for _ in range(k)]


def to_device(blocks, device="cuda"):
    import torch
    return [torch.from_numpy(b).to(device) for b in blocks]


def device_blocks(k: int, block_bytes: int, seed: int, device="cuda"):
    """k blocks of uniform random bytes generated on the device (for GB-scale
    inputs); returns a list of uint8 tensors, each a separate allocation."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return [torch.randint(0, 256, (block_bytes,), dtype=torch.uint8, device=device, generator=g) for _ in range(k)]


def empty_blocks(k: int, block_bytes: int, device="cuda", fill: int | None = None):
    import torch
    out = [torch.empty(block_bytes, dtype=torch.uint8, device=device) for _ in range(k)]
    if fill is not None:
        for t in out:
            t.fill_(fill)
    return out


def strip_sample(block, offsets, width: int):
    """Bytes [o, o+width) of each of the 8 strips of a block, for every o in
    ``offsets``, concatenated strip by strip into one mini-block of
    8 * len(offsets) * width bytes (a block whose strip c is the gathered
    slices of the original strip c).  Works on numpy arrays and tensors."""
    L = block.shape[0] // 8
    parts = []
    for c in range(8):
        for o in offsets:
            parts.append(block[c * L + o: c * L + o + width])
    if isinstance(block, np.ndarray):
        return np.concatenate(parts)
    import torch
    return torch.cat(parts)


def log_uniform_sizes(rng, count: int, lo: int, hi: int, quantum: int):
    """Sizes log-uniform on [lo, hi], rounded down to a multiple of quantum."""
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), count))
    return np.maximum(quantum, (x // quantum).astype(np.int64) * quantum)
