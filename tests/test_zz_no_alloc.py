"""ec_batch_run_noalloc (the batched launch for callers that cannot
allocate) against the existing entry point it varies, ec_batch_build +
ec_batch_launch, and the oracle: two calls in a row, the second on fewer and
smaller stripes, outputs poisoned before each; then its capacity and
upload errors."""
import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import batching as B
from paper_2108_02692_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def case(cache, count, hi, seed):
    """Stripes of a seeded mix, their device inputs and the oracle's outputs."""
    specs = B.mixed_specs(count, seed=seed, lo=4096, hi=hi)
    rng = np.random.default_rng(seed + 1)
    stripes, want = [], []
    for s in specs:
        prog = cache.get(s.n, s.p, s.erased)
        G = oracle.cauchy(s.n, s.p)
        data = [rng.integers(0, 256, s.block_bytes, dtype=np.uint8) for _ in range(s.n)]
        blocks = data + oracle.encode(G, s.n, s.p, data)
        ins = [blocks[i] for i in prog.in_blocks]
        want.append([blocks[e] for e in s.erased] if s.erased else blocks[s.n:])
        stripes.append((prog, W.to_device(ins), s.block_bytes))
    cache.upload()
    return stripes, want


def outputs(stripes, want, fill):
    return [W.empty_blocks(len(w), bb, fill=fill) for (_, _, bb), w in zip(stripes, want)]


def host(outs):
    return [[t.cpu().numpy() for t in o] for o in outs]


def test_noalloc_equals_batch_build_twice():
    cache = B.ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=44, generator_fn=oracle.cauchy)
    stream = torch.cuda.current_stream()
    for count, hi, seed in ((300, 1 << 20, 61), (40, 64 << 10, 62)):
        stripes, want = case(cache, count, hi, seed)
        ref = outputs(stripes, want, 0x5A)
        b = E.ec_batch_build([(p, i, o, bb) for (p, i, bb), o in zip(stripes, ref)], stream=stream)
        b.launch(stream)
        got = outputs(stripes, want, 0xA5)
        E.ec_batch_run_noalloc([(p, i, o, bb) for (p, i, bb), o in zip(stripes, got)], stream=stream)
        torch.cuda.synchronize()
        b.free()
        got_h, ref_h = host(got), host(ref)
        for k, (g, r, w) in enumerate(zip(got_h, ref_h, want)):
            for j in range(len(w)):
                assert np.array_equal(g[j], r[j]), "stripe %d output %d: no-alloc differs from ec_batch_launch" % (k, j)
                assert np.array_equal(g[j], w[j]), "stripe %d output %d: differs from the oracle" % (k, j)


def test_noalloc_errors():
    gen = oracle.cauchy(10, 4).tolist()
    stream = torch.cuda.current_stream()
    fresh = E.ec_compile_slp(10, 4, gen, slot_budget=38)  # never uploaded
    d, o = W.empty_blocks(10, 4096, fill=0), W.empty_blocks(4, 4096)
    with pytest.raises(E.EcError) as e:
        E.ec_batch_run_noalloc([(fresh, d, o, 4096)], stream=stream)
    assert e.value.name == "EC_ERR_ARG"
    fresh.upload()
    E.ec_batch_run_noalloc([(fresh, d, o, 4096)], stream=stream)
    torch.cuda.synchronize()
    # more stripes than the tables hold
    outs = [W.empty_blocks(4, 128) for _ in range(1025)]
    with pytest.raises(E.EcError) as e:
        E.ec_batch_run_noalloc([(fresh, d, x, 128) for x in outs], stream=stream)
    assert e.value.name == "EC_ERR_CAPACITY"
    # more work items than the tables hold: 8 stripes of 32 MiB blocks, 4096
    # tiles each, times 32 row parts
    rows = E.ec_compile_slp(10, 4, gen, slot_budget=38, split=E.SPLIT_ROWS)
    rows.upload()
    S = 32 << 20
    d = W.empty_blocks(10, S, fill=0)
    outs = [W.empty_blocks(4, S) for _ in range(8)]
    with pytest.raises(E.EcError) as e:
        E.ec_batch_run_noalloc([(rows, d, x, S) for x in outs], stream=stream)
    assert e.value.name == "EC_ERR_CAPACITY"
    # the same rules as ec_batch_set: an output aliasing an input
    with pytest.raises(E.EcError) as e:
        E.ec_batch_run_noalloc([(fresh, d[:10], [d[0][:4096]] + o[1:], 4096)], stream=stream)
    assert e.value.name == "EC_ERR_ARG"
    del d, outs
    torch.cuda.empty_cache()
