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


def oracle_gen(n, p):
    """The oracle's Cauchy generator, as the rows the library takes."""
    return [[int(x) for x in row] for row in oracle.cauchy(n, p)]


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
    cache = B.ProgramCache(level=level, slots=slots, generator_fn=oracle.cauchy)
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
    gen = oracle_gen(6, 3)
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
    cache = B.ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=38, generator_fn=oracle.cauchy)
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


@pytest.mark.parametrize("split", [E.SPLIT_AUTO, E.SPLIT_NEVER, E.SPLIT_ALWAYS, E.SPLIT_ROWS, E.SPLIT_PAIRS,
                                   E.SPLIT_STAGED])
def test_batch_edge_shapes_and_mixed_levels(split):
    """One batch holding the extremes: the widest codec (32 blocks), 1-block
    codecs, blocks of 128 B (one lane of one tile per strip) and ragged
    sizes, encodes and decodes, programs of different levels at one slot
    budget; two inputs shared read-only by several stripes."""
    rng = np.random.default_rng(31)
    cases = [(28, 4, (), 128), (1, 1, (), 128), (1, 1, (0,), 256), (2, 1, (1,), 384), (10, 4, (2, 4, 5, 6), 1152),
             (6, 3, (), 3 * 8192 + 128), (14, 4, (0, 13), 4096 + 128), (10, 4, (), 128), (12, 4, (15,), 8 * 1024 * 9)]
    stripes, want, keep = [], [], []
    for k, (n, p, er, S) in enumerate(cases):
        gen = oracle_gen(n, p)
        G = np.array(gen, dtype=np.uint8)
        level = (E.LEVEL_PLAIN, E.LEVEL_CO, E.LEVEL_CO_FU_SCHED)[k % 3]
        prog = E.ec_compile_slp(n, p, gen, list(er), level=level, slot_budget=44,
                                split=split if k % 2 else E.SPLIT_AUTO)
        data = [rng.integers(0, 256, S, dtype=np.uint8) for _ in range(n)]
        blocks = data + oracle.encode(G, n, p, data)
        if er:
            ins = W.to_device([blocks[i] for i in prog.in_blocks])
            exp = [blocks[e] for e in er]
        else:
            ins = W.to_device(data)
            exp = blocks[n:]
        outs = W.empty_blocks(len(exp), S, fill=0xA5)
        stripes.append((prog, ins, outs, S))
        want.append(exp)
        keep.append(prog)
        if k == 4:  # the same inputs again, as a second stripe with its own outputs
            outs2 = W.empty_blocks(len(exp), S, fill=0xA5)
            stripes.append((prog, ins, outs2, S))
            want.append(exp)
    stream = torch.cuda.current_stream()
    batch = E.ec_batch_build(stripes, stream=stream)
    for rep in range(2):
        for _, _, outs, _ in stripes:
            for t in outs:
                t.fill_(0x11 * (rep + 1))
        torch.cuda.synchronize()
        batch.launch(stream)
        torch.cuda.synchronize()
        check([o for _, _, o, _ in stripes], want, "edge batch replay %d" % rep)
    batch.free()


def test_batch_argument_errors():
    gen = oracle_gen(6, 3)
    prog = E.ec_compile_slp(6, 3, gen, slot_budget=38)
    d = W.empty_blocks(6, 4096, fill=0)
    o = W.empty_blocks(3, 4096)
    with pytest.raises(E.EcError) as e:
        E.ec_batch_build([])
    assert e.value.name == "EC_ERR_ARG"
    with pytest.raises(E.EcError) as e:  # block size not a multiple of 128
        E.ec_batch_build([(prog, d, o, 4096 - 64)])
    assert e.value.name == "EC_ERR_ALIGN"
    with pytest.raises(E.EcError) as e:  # an output aliasing an input
        E.ec_batch_build([(prog, d, [d[0], o[1], o[2]], 4096)])
    assert e.value.name == "EC_ERR_ARG"
    o2 = W.empty_blocks(3, 4096)
    with pytest.raises(E.EcError) as e:  # two stripes writing the same block
        E.ec_batch_build([(prog, d, o, 4096), (prog, d, [o2[0], o[1], o2[2]], 4096)])
    assert e.value.name == "EC_ERR_ARG"
    with pytest.raises(E.EcError) as e:  # a stripe reading what another writes
        E.ec_batch_build([(prog, d, o, 4096), (prog, [o[2]] + d[1:], o2, 4096)])
    assert e.value.name == "EC_ERR_ARG"
    half = torch.empty(2 * 4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(E.EcError) as e:  # outputs overlapping by half a block
        E.ec_batch_build([(prog, d, [half[:4096], o[1], o[2]], 4096),
                          (prog, d, [half[2048:6144], o2[1], o2[2]], 4096)])
    assert e.value.name == "EC_ERR_ARG"
    # shared inputs and back-to-back outputs are fine
    E.ec_batch_build([(prog, d, [half[:4096], o[1], o[2]], 4096),
                      (prog, d, [half[4096:], o2[1], o2[2]], 4096)]).free()
    with pytest.raises(E.EcError) as e:  # work items of 1.5 KiB
        E.ec_batch_build([(prog, d, o, 4096)], tile_bytes=1536)
    assert e.value.name == "EC_ERR_UNSUPPORTED"
