"""GPU parity: the HIP executor (through the C ABI) against the CPU oracle.

Every comparison is byte-exact (the path is integer XOR only).  Inputs come
from the seeded generators in ``paper_2108_02692_amd.workloads``; expected
values come from the oracle only: parity blocks from ``oracle.encode`` and,
for decode, the original blocks themselves (the oracle's encode of the data).
Every program is compiled from the oracle's generator matrix.
"""
import functools
import itertools
import os
import random
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def oracle_gen(n, p):
    """The oracle's Cauchy generator, as the rows the library takes."""
    return [[int(x) for x in row] for row in oracle.cauchy(n, p)]


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    E.lib()


def run_encode(prog, data_np, block_bytes, stream=None):
    d = W.to_device(data_np)
    par = W.empty_blocks(len(prog.out_blocks), block_bytes, fill=0xA5)
    E.ec_encode(prog, d, par, block_bytes, stream)
    torch.cuda.synchronize()
    return [p.cpu().numpy() for p in par]


def run_decode(prog, blocks_np, block_bytes):
    surv = W.to_device([blocks_np[i] for i in prog.in_blocks])
    rec = W.empty_blocks(len(prog.out_blocks), block_bytes, fill=0xA5)
    E.ec_decode(prog, surv, rec, block_bytes)
    torch.cuda.synchronize()
    return [r.cpu().numpy() for r in rec]


def assert_blocks_equal(got, want, what):
    for j, (g, w) in enumerate(zip(got, want)):
        if not np.array_equal(g, w):
            bad = np.nonzero(g != w)[0]
            raise AssertionError("%s: block %d differs at %d bytes, first at %d" % (what, j, bad.size, bad[0]))


@functools.lru_cache(maxsize=None)
def rs10_4_1mib():
    n, p, S = 10, 4, 1 << 20
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=0)
    return gen, data, oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)


def compile_many(n, p, gen, patterns, **kw):
    """Compile one program per pattern on host threads (the C call releases
    the GIL)."""
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda er: E.ec_compile_slp(n, p, gen, er, **kw), patterns))


@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO, E.LEVEL_CO_FU, E.LEVEL_CO_FU_SCHED])
@pytest.mark.parametrize("K", [24, 32, 36, 38, 40, 44, 48, 56, 60])
def test_encode_rs10_4_1mib(level, K):
    """RS(10,4) encode, 10 x 1 MiB blocks of seeded random bytes."""
    n, p, S = 10, 4, 1 << 20
    gen, data, want = rs10_4_1mib()
    prog = E.ec_compile_slp(n, p, gen, level=level, slot_budget=K)
    assert_blocks_equal(run_encode(prog, data, S), want, "encode level %d K %d" % (level, K))


@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO, E.LEVEL_CO_FU, E.LEVEL_CO_FU_SCHED])
@pytest.mark.parametrize("K", [24, 32, 36, 38, 40, 44, 48, 56, 60])
def test_greedy_scheduler_rs10_4(level, K):
    """Programs whose strip order comes from the bottom-up greedy heuristic
    (EC_SCHED_GREEDY): RS(10,4) encode and the decode of {2, 4, 5, 6} on
    1 MiB blocks (pair parts) and on 4 MiB + 128 B blocks (whole program,
    ragged last tile), every level and slot budget."""
    n, p = 10, 4
    gen = oracle_gen(n, p)
    G = np.array(gen, dtype=np.uint8)
    er = [2, 4, 5, 6]
    for S in (1 << 20, (4 << 20) + 128):
        data = W.host_blocks(n, S, seed=K + level)
        blocks = data + oracle.encode(G, n, p, data)
        enc = E.ec_compile_slp(n, p, gen, level=level, slot_budget=K, scheduler=E.SCHED_GREEDY)
        assert_blocks_equal(run_encode(enc, data, S), blocks[n:], "greedy encode level %d K %d S %d" % (level, K, S))
        dec = E.ec_compile_slp(n, p, gen, er, level=level, slot_budget=K, scheduler=E.SCHED_GREEDY)
        assert_blocks_equal(run_decode(dec, blocks, S), [blocks[e] for e in er],
                            "greedy decode level %d K %d S %d" % (level, K, S))


@pytest.mark.parametrize("S", [128, 256, 1152, 8192 + 128, 3 * 8192, 65536 + 640])
def test_encode_ragged_sizes(S):
    """Block sizes that leave a partial tile (1 KiB per strip per wave)."""
    n, p = 10, 4
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=S)
    want = oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
    for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
        prog = E.ec_compile_slp(n, p, gen, level=level)
        assert_blocks_equal(run_encode(prog, data, S), want, "encode S=%d level %d" % (S, level))


CODECS = [(6, 3), (12, 4), (14, 4), (8, 4), (9, 4), (8, 3), (9, 3), (10, 3), (8, 2), (9, 2), (10, 2)]


@pytest.mark.parametrize("n,p", CODECS)
def test_encode_other_codecs(n, p):
    S = 64 * 1024
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=n * 10 + p)
    want = oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
    for K in (0, 24, 48):
        prog = E.ec_compile_slp(n, p, gen, slot_budget=K)
        assert_blocks_equal(run_encode(prog, data, S), want, "RS(%d,%d) K %d" % (n, p, K))


def test_encode_row_passes_and_block_widths():
    """RS(8,8) needs several passes over the inputs (64 rows > slots);
    RS(10,4) with other column-block widths."""
    S = 64 * 1024 + 128
    gen = oracle_gen(8, 8)
    data = W.host_blocks(8, S, seed=88)
    want = oracle.encode(np.array(gen, dtype=np.uint8), 8, 8, data)
    for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
        prog = E.ec_compile_slp(8, 8, gen, level=level, slot_budget=48)
        assert prog.info["passes"] >= 2
        assert_blocks_equal(run_encode(prog, data, S), want, "RS(8,8) level %d" % level)
    gen, data, want = rs10_4_1mib()
    for width in (1, 4, 16, 40):
        prog = E.ec_compile_slp(10, 4, gen, block_strips=width, slot_budget=48)
        assert_blocks_equal(run_encode(prog, data, 1 << 20), want, "width %d" % width)


@pytest.mark.parametrize("dist", [4, 12, 20])
def test_encode_decode_with_prefetch(dist):
    n, p, S = 10, 4, (1 << 20) + 640
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=dist)
    blocks = data + oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
    for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
        prog = E.ec_compile_slp(n, p, gen, level=level, prefetch=dist)
        assert_blocks_equal(run_encode(prog, data, S), blocks[n:], "encode level %d prefetch %d" % (level, dist))
        er = (1, 5, 10, 12)
        prog = E.ec_compile_slp(n, p, gen, er, level=level, prefetch=dist)
        assert_blocks_equal(run_decode(prog, blocks, S), [blocks[e] for e in er], "decode prefetch %d" % dist)


@pytest.mark.parametrize("n,p,er", [(1, 3, ()), (1, 3, (0, 2)), (28, 4, ()), (28, 4, (1, 9, 27, 30)),
                                    (4, 12, ()), (4, 12, (0, 3, 5, 15)), (2, 0, ())])
def test_degenerate_and_wide_codecs(n, p, er):
    """Replication (n = 1), the widest stripe (32 blocks), more rows than
    slots (RS(4,12): several passes over the inputs) and no parity at all."""
    S = 8192 + 128
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=n * 100 + p)
    blocks = data + (oracle.encode(np.array(gen, dtype=np.uint8), n, p, data) if p else [])
    for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
        prog = E.ec_compile_slp(n, p, gen, list(er), level=level)
        if er:
            got = run_decode(prog, blocks, S)
            assert_blocks_equal(got, [blocks[e] for e in er], "RS(%d,%d) decode %s" % (n, p, er))
        else:
            assert_blocks_equal(run_encode(prog, data, S), blocks[n:], "RS(%d,%d) encode" % (n, p))


def all_patterns(n, p):
    return [c for r in range(1, p + 1) for c in itertools.combinations(range(n + p), r)]


def test_decode_rs10_4_every_pattern():
    """All 1470 erasure sets of <= 4 blocks (1001 of exactly 4); 2 KiB blocks.
    Recovered blocks must equal the originals (data from the generator,
    parity from the oracle)."""
    n, p, S = 10, 4, 2048
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=7)
    blocks = data + oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
    dev = W.to_device(blocks)
    pats = all_patterns(n, p)
    assert len(pats) == 1470
    for er, prog in zip(pats, compile_many(n, p, gen, pats)):
        rec = W.empty_blocks(len(er), S, fill=0xA5)
        E.ec_decode(prog, [dev[i] for i in prog.in_blocks], rec, S)
        torch.cuda.synchronize()
        assert_blocks_equal([r.cpu().numpy() for r in rec], [blocks[e] for e in er], "decode %s" % (er,))


@pytest.mark.parametrize("er", [(2, 4, 5, 6), (4, 5, 6, 7), (0, 1, 2, 3), (10, 11, 12, 13), (0, 13), (9,)])
@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED])
def test_decode_rs10_4_1mib(er, level):
    n, p, S = 10, 4, 1 << 20
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=1)
    blocks = data + oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
    prog = E.ec_compile_slp(n, p, gen, er, level=level)
    assert_blocks_equal(run_decode(prog, blocks, S), [blocks[e] for e in er], "decode %s" % (er,))


@pytest.mark.parametrize("n,p", CODECS)
def test_decode_other_codecs_sampled(n, p):
    S = 4096
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=3 * n + p)
    blocks = data + oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
    rng = random.Random(n)
    for er in rng.sample(all_patterns(n, p), 40):
        prog = E.ec_compile_slp(n, p, gen, er)
        assert_blocks_equal(run_decode(prog, blocks, S), [blocks[e] for e in er], "RS(%d,%d) %s" % (n, p, er))


def test_largest_block_sampled():
    """The largest block the executor takes (4 GiB - 128 B: strips of just
    under 512 MiB, strip offsets past 2^31 within a block), RS(4,2) encode
    and a two-block decode, checked on sampled strip offsets against the
    oracle."""
    n, p, S = 4, 2, (1 << 32) - 128
    gen = oracle_gen(n, p)
    G = np.array(gen, dtype=np.uint8)
    data = W.device_blocks(n, S, seed=13)
    par = W.empty_blocks(p, S, fill=0xA5)
    E.ec_encode(E.ec_compile_slp(n, p, gen), data, par, S)
    torch.cuda.synchronize()
    L = S // 8
    offs = [0, 1024, L // 2 + 48, L - 1024, L - 16]
    blocks = data + par
    mini = [W.strip_sample(b, offs, 16).cpu().numpy() for b in blocks]
    assert_blocks_equal(mini[n:], oracle.encode(G, n, p, mini[:n]), "largest block encode")
    er = [0, 3]
    prog = E.ec_compile_slp(n, p, gen, er)
    rec = W.empty_blocks(len(er), S, fill=0xA5)
    E.ec_decode(prog, [blocks[i] for i in prog.in_blocks], rec, S)
    torch.cuda.synchronize()
    got = [W.strip_sample(r, offs, 16).cpu().numpy() for r in rec]
    assert_blocks_equal(got, [mini[e] for e in prog.out_blocks], "largest block decode")
    del data, par, rec, blocks
    torch.cuda.empty_cache()


def test_outputs_fully_written_and_inputs_untouched():
    n, p, S = 10, 4, 4096 + 128
    gen = oracle_gen(n, p)
    data = W.host_blocks(n, S, seed=5)
    d = W.to_device(data)
    prog = E.ec_compile_slp(n, p, gen)
    for fill in (0x00, 0xFF, 0xA5):
        par = W.empty_blocks(p, S, fill=fill)
        E.ec_encode(prog, d, par, S)
        torch.cuda.synchronize()
        want = oracle.encode(np.array(gen, dtype=np.uint8), n, p, data)
        assert_blocks_equal([x.cpu().numpy() for x in par], want, "fill %x" % fill)
    assert_blocks_equal([x.cpu().numpy() for x in d], data, "inputs")


def test_two_streams_concurrently():
    n, p, S = 10, 4, 1 << 18
    gen = oracle_gen(n, p)
    prog_a = E.ec_compile_slp(n, p, gen)
    prog_b = E.ec_compile_slp(n, p, gen, level=E.LEVEL_PLAIN, slot_budget=48)
    da, db = W.host_blocks(n, S, seed=21), W.host_blocks(n, S, seed=22)
    ta, tb = W.to_device(da), W.to_device(db)
    pa, pb = W.empty_blocks(p, S), W.empty_blocks(p, S)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    E.ec_encode(prog_a, ta, pa, S, sa)
    E.ec_encode(prog_b, tb, pb, S, sb)
    torch.cuda.synchronize()
    G = np.array(gen, dtype=np.uint8)
    assert_blocks_equal([x.cpu().numpy() for x in pa], oracle.encode(G, n, p, da), "stream a")
    assert_blocks_equal([x.cpu().numpy() for x in pb], oracle.encode(G, n, p, db), "stream b")


@pytest.mark.parametrize("S", [256 << 10, 4 << 20])
def test_graph_captured_launches_replay(S):
    """ec_encode and ec_decode captured in a HIP graph (after uploading the
    programs) and replayed three times, with new input bytes and poisoned
    outputs written eagerly between the replays: every replay equals the
    oracle on that replay's inputs (256 KiB blocks take row parts, 4 MiB
    block parts)."""
    n, p, er = 10, 4, [2, 4, 5, 11]
    gen = oracle_gen(n, p)
    G = np.array(gen, dtype=np.uint8)
    enc = E.ec_compile_slp(n, p, gen)
    dec = E.ec_compile_slp(n, p, gen, er)
    enc.upload()
    dec.upload()
    d, par = W.empty_blocks(n, S), W.empty_blocks(p, S)
    surv, rec = W.empty_blocks(len(dec.in_blocks), S), W.empty_blocks(len(dec.out_blocks), S)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        E.ec_encode(enc, d, par, S, s)
        E.ec_decode(dec, surv, rec, S, s)
    for rep in range(3):
        data = W.host_blocks(n, S, seed=100 + rep)
        blocks = data + oracle.encode(G, n, p, data)
        for t, x in zip(d, data):
            t.copy_(torch.from_numpy(x))
        for t, b in zip(surv, dec.in_blocks):
            t.copy_(torch.from_numpy(blocks[b]))
        for t in par + rec:
            t.fill_(0x3C + rep)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        assert_blocks_equal([x.cpu().numpy() for x in par], blocks[n:], "graph encode replay %d" % rep)
        assert_blocks_equal([x.cpu().numpy() for x in rec], [blocks[e] for e in dec.out_blocks],
                            "graph decode replay %d" % rep)


def test_launch_argument_errors():
    n, p, S = 10, 4, 4096
    gen = oracle_gen(n, p)
    prog = E.ec_compile_slp(n, p, gen)
    dec = E.ec_compile_slp(n, p, gen, [1])
    d = W.empty_blocks(n, S, fill=0)
    par = W.empty_blocks(p, S)
    big = torch.zeros(S + 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(E.EcError) as e:
        E.ec_encode(prog, d, par, S - 64)
    assert e.value.name == "EC_ERR_ALIGN"
    with pytest.raises(E.EcError) as e:
        E.ec_encode(prog, d[:-1] + [big[8:]], par, S)
    assert e.value.name == "EC_ERR_ALIGN"
    with pytest.raises(E.EcError) as e:
        E.ec_encode(prog, d, par[:-1] + [d[0]], S)
    assert e.value.name == "EC_ERR_ARG"
    with pytest.raises(E.EcError) as e:
        E.ec_decode(prog, d, par, S)
    assert e.value.name == "EC_ERR_ARG"
    with pytest.raises(E.EcError) as e:
        E.ec_encode(dec, d, par, S)
    assert e.value.name == "EC_ERR_ARG"


@pytest.mark.parametrize("n,p,er", [(10, 4, ()), (10, 4, (2, 4, 5, 6)), (6, 3, ()), (14, 4, (0, 13)), (2, 1, ()),
                                    (4, 12, ()), (2, 10, ()), (4, 12, tuple(range(1, 12))), (12, 6, ()),
                                    (8, 8, (0, 3, 9, 10, 11, 12, 13, 15))])
def test_row_split_matches_oracle(n, p, er):
    """Short stripes run one wave per (tile, part): row, pair, block and
    pass parts forced, the split off and left to the library, on ragged and
    small block sizes, equal the oracle."""
    gen = oracle_gen(n, p)
    G = np.array(gen, dtype=np.uint8)
    for S in (4096 + 128, 1 << 20, 3 * (1 << 20) + 384):
        data = W.host_blocks(n, S, seed=S % 1000 + n)
        blocks = data + oracle.encode(G, n, p, data)
        want = [blocks[e] for e in er] if er else blocks[n:]
        for split in (E.SPLIT_ROWS, E.SPLIT_PAIRS, E.SPLIT_ALWAYS, E.SPLIT_PASSES, E.SPLIT_NEVER, E.SPLIT_AUTO):
            prog = E.ec_compile_slp(n, p, gen, list(er), split=split)
            got = run_decode(prog, blocks, S) if er else run_encode(prog, data, S)
            assert_blocks_equal(got, want, "RS(%d,%d) %s S=%d split %d" % (n, p, er, S, split))


def test_random_cases_match_oracle():
    """Seeded random cases over the whole compile space: codec (up to 32
    blocks), erasure set, level, slot budget, split policy and block size
    (any multiple of 128 B up to 384 KiB), each compared with the oracle."""
    rng = random.Random(2024)
    budgets = (0, 24, 32, 36, 38, 40, 44, 48, 56, 60)
    levels = (E.LEVEL_PLAIN, E.LEVEL_CO, E.LEVEL_CO_FU, E.LEVEL_CO_FU_SCHED)
    splits = (E.SPLIT_AUTO, E.SPLIT_NEVER, E.SPLIT_ALWAYS, E.SPLIT_ROWS, E.SPLIT_PAIRS)
    done = 0
    while done < 40:
        n = rng.randint(1, 20)
        p = rng.randint(0, min(8, 32 - n))
        k = rng.randint(0, p)
        er = tuple(sorted(rng.sample(range(n + p), k)))
        S = 128 * rng.randint(1, 3072)
        gen = oracle_gen(n, p)
        try:
            prog = E.ec_compile_slp(n, p, gen, list(er), level=rng.choice(levels),
                                    slot_budget=rng.choice(budgets), split=rng.choice(splits))
        except E.EcError as e:  # a budget too small for the codec
            assert e.name == "EC_ERR_CAPACITY", e
            continue
        if not prog.out_blocks:
            continue
        G = np.array(gen, dtype=np.uint8)
        data = W.host_blocks(n, S, seed=rng.randint(0, 1 << 30))
        blocks = data + oracle.encode(G, n, p, data) if p else data
        what = "RS(%d,%d) %s S=%d %s" % (n, p, er, S, prog.info)
        if er:
            assert_blocks_equal(run_decode(prog, blocks, S), [blocks[e] for e in er], what)
        else:
            assert_blocks_equal(run_encode(prog, data, S), blocks[n:], what)
        done += 1


@pytest.mark.parametrize("S", [128, 8192 + 128, 1 << 20, 32 << 20])
def test_stripe_stream_reference_kernel(S):
    """ec_stripe_stream (the coding launch's data movement without a program,
    a measurement reference): every output strip is the XOR of all input
    strips at the same offset (numpy), on ragged sizes and on 4 MiB strips
    (the segment tile order); ec_device_copy copies exactly."""
    n_in, n_out = 10, 4
    data = W.host_blocks(n_in, S, seed=S % 997)
    want = np.bitwise_xor.reduce(np.stack([b.reshape(8, S // 8) for b in data]).reshape(-1, S // 8), axis=0)
    out = W.empty_blocks(n_out, S, fill=0xA5)
    E.ec_stripe_stream(W.to_device(data), out, S)
    torch.cuda.synchronize()
    for j, o in enumerate(out):
        got = o.cpu().numpy().reshape(8, S // 8)
        for r in range(8):
            assert np.array_equal(got[r], want), "output %d strip %d" % (j, r)
    src = torch.from_numpy(data[0]).cuda()
    dst = torch.full((S + 64,), 0x5A, dtype=torch.uint8, device="cuda")
    E.ec_device_copy(dst, src, S)
    torch.cuda.synchronize()
    assert torch.equal(dst[:S], src) and bool((dst[S:] == 0x5A).all())
