"""Host side of the serving workload (no GPU): the seeded request generator.
(The loop's output arena allocator is C++, exercised under the host
sanitizers by tests/sanitize/lib_driver.cpp.)"""
import numpy as np

from paper_2108_02692_amd.serve import make_requests


def test_request_stream_shape():
    reqs = make_requests(0.5, 20000.0, seed=7, pool_ptr=1 << 40, pool_bytes=1 << 30)
    assert 9000 < len(reqs) < 11000                       # Poisson count, mean 10000
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) >= 0) and arr[-1] <= 0.5
    frac104 = np.mean([(r.n, r.p) == (10, 4) for r in reqs])
    assert abs(frac104 - 0.75) < 0.03
    enc = np.mean([not r.erased for r in reqs])
    assert abs(enc - 0.7) < 0.03
    for r in reqs[:500]:
        assert r.block_bytes % 512 == 0 and r.block_bytes * r.n >= 4096
        assert len(r.inputs) == r.n
        assert all((1 << 40) <= x and x + r.block_bytes <= (1 << 40) + (1 << 30) for x in r.inputs)
        assert len(set(r.erased)) == len(r.erased) <= r.p
    obj = np.array([r.block_bytes * r.n for r in reqs])
    assert 200 << 10 < np.median(obj) < 330 << 10             # log-normal median 256 KiB (+ rounding)
    again = make_requests(0.5, 20000.0, seed=7, pool_ptr=1 << 40, pool_bytes=1 << 30)
    assert [(r.arrival, r.block_bytes, r.erased) for r in again] == [(r.arrival, r.block_bytes, r.erased) for r in reqs]


def test_distinct_input_layout():
    """place_inputs: every input block its own 4 KiB-aligned range of the
    pool (no two blocks overlap), inside the pool; a pool too small is an
    error."""
    import pytest
    from paper_2108_02692_amd.serve import input_span, place_inputs
    reqs = make_requests(0.05, 20000.0, seed=3)
    assert reqs and all(r.inputs == [] for r in reqs)
    base, need = 1 << 40, input_span(reqs)
    place_inputs(reqs, base, need)
    spans = sorted((x, x + r.block_bytes) for r in reqs for x in r.inputs)
    assert len(spans) == sum(r.n for r in reqs)
    assert all(a % 4096 == 0 and base <= a and b <= base + need for a, b in spans)
    assert all(b0 <= a1 for (_, b0), (a1, _) in zip(spans, spans[1:]))
    with pytest.raises(ValueError):
        place_inputs(reqs, base, need - 4096)


def test_pinned_restores_affinity():
    """The serving loop's pinning keeps the thread on one allowed CPU while
    it runs and gives the full set back afterwards, also on an error."""
    import os
    import pytest
    from paper_2108_02692_amd.serve import _pinned
    allowed = os.sched_getaffinity(0)
    with _pinned(True):
        inside = os.sched_getaffinity(0)
    assert os.sched_getaffinity(0) == allowed
    assert inside <= allowed and (len(inside) == 1 or len(allowed) == 1)
    with pytest.raises(RuntimeError):
        with _pinned(True):
            raise RuntimeError("stop")
    assert os.sched_getaffinity(0) == allowed
    with _pinned(False):
        assert os.sched_getaffinity(0) == allowed
