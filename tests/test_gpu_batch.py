"""Batched path on the GPU: a mix of codecs, block sizes, encodes and decodes
in one persistent launch, compared byte for byte with the oracle; the HIP
graph is replayed several times with eager work in between and every replay
is checked (a graph must give the eager result every time)."""
import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import batching as B
from paper_2108_02692_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make_case(specs, cache, seed):
    """Host inputs and expected outputs per stripe (expected from the oracle)."""
    rng = np.random.default_rng(seed)
    ins, want = [], []
    for s in specs:
        G = np.array(cache.generator(s.n, s.p), dtype=np.uint8)
        data = [rng.integers(0, 256, s.block_bytes, dtype=np.uint8) for _ in range(s.n)]
        par = oracle.encode(G, s.n, s.p, data)
        if not s.erased:
            ins.append(data)
            want.append(par)
        else:
            blocks = data + par
            prog = cache.get(s.n, s.p, s.erased)
            ins.append([blocks[i] for i in prog.in_blocks])
            want.append([blocks[e] for e in s.erased])
    return ins, want


def check(outs, want, what):
    for k, (o, w) in enumerate(zip(outs, want)):
        for j, (a, b) in enumerate(zip(o, w)):
            assert np.array_equal(a.cpu().numpy(), b), "%s: stripe %d output %d" % (what, k, j)


@pytest.mark.parametrize("level,slots,tile", [(E.LEVEL_PLAIN, 38, 0), (E.LEVEL_PLAIN, 48, 4096),
                                              (E.LEVEL_CO_FU_SCHED, 44, 0), (E.LEVEL_CO_FU_SCHED, 24, 2048)])
def test_batch_mixed_matches_oracle_and_graph_replays(level, slots, tile):
    specs = B.mixed_specs(96, seed=5, lo=4096, hi=64 * 1024)
    cache = B.ProgramCache(level=level, slots=slots)
    ins_h, want = make_case(specs, cache, seed=6)
    ins = [W.to_device(x) for x in ins_h]
    outs = [W.empty_blocks(s.n_out, s.block_bytes, fill=0xA5) for s in specs]
    stream = torch.cuda.current_stream()
    batch = B.build_batch(specs, cache, ins, outs, tile_bytes=tile, stream=stream)
    assert batch.n_items > 0
    assert batch.in_bytes == sum(s.n_in * s.block_bytes for s in specs)
    batch.enqueue(stream)
    torch.cuda.synchronize()
    check(outs, want, "eager")
    for rep in range(3):
        for o in outs:
            for t in o:
                t.fill_(0x5A + rep)
        torch.cuda.synchronize()
        batch.launch(stream)
        torch.cuda.synchronize()
        check(outs, want, "graph replay %d" % rep)


def test_batch_rejects_mixed_slot_budgets():
    gen = E.ec_matrix_cauchy(6, 3)
    a = E.ec_compile_slp(6, 3, gen, level=E.LEVEL_PLAIN, slot_budget=40)
    b = E.ec_compile_slp(6, 3, gen, level=E.LEVEL_PLAIN, slot_budget=48)
    d = W.empty_blocks(6, 4096, fill=0)
    o1, o2 = W.empty_blocks(3, 4096), W.empty_blocks(3, 4096)
    with pytest.raises(E.EcError) as e:
        E.ec_batch_build([(a, d, o1, 4096), (b, d, o2, 4096)])
    assert e.value.name == "EC_ERR_UNSUPPORTED"


def test_reusable_batch_reserve_and_refill():
    """create + reserve + set/enqueue twice with different stripes (the
    serving pattern), programs uploaded beforehand; both runs match the
    oracle."""
    cache = B.ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=38)
    stream = torch.cuda.current_stream()
    batch = E.Batch.create()
    batch.reserve(64, 4096)
    for seed in (11, 12):
        specs = B.mixed_specs(40, seed=seed, codecs=((10, 4), (6, 3)), lo=4096, hi=32 * 1024)
        for s in specs:
            cache.get(s.n, s.p, s.erased)
        cache.upload()
        ins_h, want = make_case(specs, cache, seed=seed + 100)
        ins = [W.to_device(x) for x in ins_h]
        outs = [W.empty_blocks(s.n_out, s.block_bytes, fill=0xA5) for s in specs]
        batch.set([(cache.get(s.n, s.p, s.erased), ins[k], outs[k], s.block_bytes) for k, s in enumerate(specs)],
                  stream=stream)
        batch.enqueue(stream)
        torch.cuda.synchronize()
        check(outs, want, "refill seed %d" % seed)
    batch.free()
