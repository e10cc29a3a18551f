"""Host logic of the serving loop (no GPU): the output arena allocator and the
seeded request generator."""
import numpy as np

from paper_2108_02692_amd.serve import FirstFit, make_requests


def test_first_fit_reuses_and_coalesces():
    h = FirstFit(1 << 20, align=4096)
    a = h.alloc(5000)
    b = h.alloc(4096)
    c = h.alloc(100)
    assert a == (0, 8192) and b == (8192, 4096) and c == (12288, 4096)
    h.free(*b)
    assert h.alloc(4096) == (8192, 4096)        # hole reused first
    h.free(8192, 4096)
    h.free(*a)
    h.free(*c)
    assert h.starts == [0] and h.lens == [1 << 20]  # everything coalesced
    assert h.alloc((1 << 20) + 1) == (-1, 0)


def test_first_fit_random_never_overlaps():
    rng = np.random.default_rng(3)
    size = 1 << 24
    h = FirstFit(size, align=512)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            h.free(*live.pop(int(rng.integers(len(live)))))
        else:
            off, got = h.alloc(int(rng.integers(1, 200000)))
            if off >= 0:
                live.append((off, got))
        spans = sorted(live)
        for (o1, n1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + n1 <= o2
        assert all(o + n <= size for o, n in spans)
        assert sum(n for _, n in live) + sum(h.lens) == size


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
