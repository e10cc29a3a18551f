"""The staged launch (EC_SPLIT_STAGED: each tile's input strips copied into
LDS, one workgroup of 4 waves per tile, wave w on stage part w) against the
oracle, byte for byte: codecs from 2 to 29 blocks (up to the 20 input blocks
that fit the LDS), encodes and decodes, both program levels, several slot
budgets and both strip schedulers, on block sizes from one lane of one tile
(128 B) through ragged tails to several MiB.  Outputs are poisoned first;
generators and expected values come from the oracle only."""
import os

import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
SIZES = (128, 8320, 1 << 20, (3 << 20) + 1152)


def oracle_gen(n, p):
    return [[int(x) for x in row] for row in oracle.cauchy(n, p)]


def check_program(prog, n, p, er, sizes, seed):
    G = oracle.cauchy(n, p)
    rng = np.random.default_rng(seed)
    for S in sizes:
        data = [rng.integers(0, 256, S, dtype=np.uint8) for _ in range(n)]
        blocks = data + oracle.encode(G, n, p, data, threads=THREADS)
        ins = W.to_device([blocks[i] for i in prog.in_blocks])
        outs = W.empty_blocks(len(prog.out_blocks), S, fill=0xA5)
        if er:
            E.ec_decode(prog, ins, outs, S)
        else:
            E.ec_encode(prog, ins, outs, S)
        torch.cuda.synchronize()
        for j, b in enumerate(prog.out_blocks):
            got = outs[j].cpu().numpy()
            if not np.array_equal(got, blocks[b]):
                bad = np.nonzero(got != blocks[b])[0]
                raise AssertionError("RS(%d,%d) erased %s, %d B: block %d, %d bytes differ, first at %d"
                                     % (n, p, er, S, b, bad.size, bad[0]))


@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED])
@pytest.mark.parametrize("n,p,er", [(10, 4, ()), (10, 4, (2, 4, 5, 6)), (6, 3, (1, 7)), (14, 4, (0, 13)),
                                    (20, 9, ()), (2, 1, ()), (1, 1, (0,)), (4, 12, ()), (12, 6, ()),
                                    (4, 12, tuple(range(1, 12)))])
def test_staged_matches_oracle(n, p, er, level):
    prog = E.ec_compile_slp(n, p, oracle_gen(n, p), list(er), level=level, split=E.SPLIT_STAGED)
    assert prog.info["n_stage_parts"] == min(4, 8 * len(prog.out_blocks))
    check_program(prog, n, p, er, SIZES if n <= 14 else SIZES[:3], seed=n * 100 + p + level)


@pytest.mark.parametrize("K", [24, 32, 48, 60])
@pytest.mark.parametrize("sched", [E.SCHED_PUSH, E.SCHED_GREEDY])
def test_staged_slot_budgets_and_schedulers(K, sched):
    """Every staged kernel instance the tests reach through RS(10,4), each
    strip scheduler."""
    for er in ((), (0, 5, 11)):
        prog = E.ec_compile_slp(10, 4, oracle_gen(10, 4), list(er), slot_budget=K, scheduler=sched,
                                split=E.SPLIT_STAGED)
        assert prog.info["slots"] == K
        check_program(prog, 10, 4, er, (8320, (1 << 20) + 1152), seed=K + sched)


def test_staged_stream_order_and_reuse():
    """Two staged launches on one stream, the second reading the first's
    outputs (a decode of the parity just encoded): stream order holds."""
    n, p, S = 10, 4, (2 << 20) + 128
    gen = oracle_gen(n, p)
    G = oracle.cauchy(n, p)
    rng = np.random.default_rng(5)
    data = [rng.integers(0, 256, S, dtype=np.uint8) for _ in range(n)]
    blocks = data + oracle.encode(G, n, p, data, threads=THREADS)
    enc = E.ec_compile_slp(n, p, gen, split=E.SPLIT_STAGED)
    er = [0, 3, 7, 9]
    dec = E.ec_compile_slp(n, p, gen, er, split=E.SPLIT_STAGED)
    dev = W.to_device(data)
    par = W.empty_blocks(p, S, fill=0xA5)
    rec = W.empty_blocks(len(er), S, fill=0xA5)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        E.ec_encode(enc, dev, par, S, stream)
        everything = dev + par
        E.ec_decode(dec, [everything[i] for i in dec.in_blocks], rec, S, stream)
    stream.synchronize()
    for j in range(p):
        assert np.array_equal(par[j].cpu().numpy(), blocks[n + j]), "parity %d" % j
    for j, e in enumerate(dec.out_blocks):
        assert np.array_equal(rec[j].cpu().numpy(), blocks[e]), "recovered block %d" % e
