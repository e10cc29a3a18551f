"""Native kernels on the GPU (ec_compile_opts.native): byte for byte
against the oracle on codecs from 2 to 32 blocks, both levels, slot budgets
from 24 to 60, encodes and decodes, block sizes from one lane of one tile
(128 B) through ragged tails to several MiB; the pair-part and block-part
kernels and the default split with native kernels; captured in a HIP graph and replayed
with new inputs; and explicit row splits, which keep the interpreter.
Generators and expected values come from the oracle; outputs are poisoned
first."""
import os

import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_gen(n, p):
    return [[int(x) for x in row] for row in oracle.cauchy(n, p)]


def run_and_check(prog, n, p, er, sizes, seed):
    G = oracle.cauchy(n, p)
    rng = np.random.default_rng(seed)
    for S in sizes:
        data = [rng.integers(0, 256, S, dtype=np.uint8) for _ in range(n)]
        blocks = data + oracle.encode(G, n, p, data, threads=THREADS)
        ins = W.to_device([blocks[i] for i in prog.in_blocks])
        outs = W.empty_blocks(len(prog.out_blocks), S, fill=0xA5)
        (E.ec_decode if er else E.ec_encode)(prog, ins, outs, S)
        torch.cuda.synchronize()
        for j, b in enumerate(prog.out_blocks):
            got = outs[j].cpu().numpy()
            if not np.array_equal(got, blocks[b]):
                bad = np.nonzero(got != blocks[b])[0]
                raise AssertionError("RS(%d,%d) erased %s, %d B: block %d, %d bytes differ, first at %d"
                                     % (n, p, er, S, b, bad.size, bad[0]))


@pytest.mark.parametrize("n,p,er,level,K", [
    (10, 4, (), E.LEVEL_CO_FU_SCHED, 0), (10, 4, (), E.LEVEL_PLAIN, 0), (10, 4, (2, 4, 5, 6), E.LEVEL_CO_FU_SCHED, 0),
    (10, 4, (0, 11, 13), E.LEVEL_PLAIN, 0), (6, 3, (1, 7), E.LEVEL_CO_FU_SCHED, 24), (14, 4, (0, 13), E.LEVEL_PLAIN, 48),
    (12, 6, (), E.LEVEL_CO_FU_SCHED, 48), (2, 1, (), E.LEVEL_PLAIN, 0), (1, 1, (0,), E.LEVEL_PLAIN, 0),
    (28, 4, (), E.LEVEL_PLAIN, 0), (4, 12, tuple(range(1, 12)), E.LEVEL_CO_FU_SCHED, 0),
    (10, 4, (3,), E.LEVEL_CO_FU_SCHED, 60), (8, 8, (), E.LEVEL_CO_FU_SCHED, 32)])
def test_native_matches_oracle(n, p, er, level, K):
    """One wave per tile on every size (no row split), so the native kernel
    runs every launch."""
    prog = E.ec_compile_slp(n, p, oracle_gen(n, p), list(er), level=level, slot_budget=K, native=True,
                            split=E.SPLIT_NEVER)
    assert prog.info["native"] == 1
    sizes = (128, 8320, (1 << 20) + 1152) + (((4 << 20) + 128,) if n <= 14 else ())
    run_and_check(prog, n, p, er, sizes, seed=n * 101 + p + level)


def test_native_beside_split_launches():
    """With the whole-program kernel the default split runs it at every
    size; an explicit split (row or block parts) keeps the interpreter on
    the same program.  All equal the oracle."""
    n, p = 10, 4
    for er in ((), (1, 5, 12)):
        prog = E.ec_compile_slp(n, p, oracle_gen(n, p), list(er), native=True)
        run_and_check(prog, n, p, er, (8192, 1 << 20, 16 << 20), seed=7 + len(er))
        for split in (E.SPLIT_ROWS, E.SPLIT_ALWAYS):
            prog = E.ec_compile_slp(n, p, oracle_gen(n, p), list(er), native=True, split=split)
            run_and_check(prog, n, p, er, (8192, (1 << 20) + 128), seed=11 + split)


@pytest.mark.parametrize("S", [1 << 20, 16 << 20])
def test_native_graph_replay(S):
    """Native launches captured in a HIP graph (after the upload loads the
    kernels) and replayed three times with new inputs and poisoned outputs
    written eagerly between the replays."""
    n, p, er = 10, 4, [2, 4, 5, 11]
    gen = oracle_gen(n, p)
    G = oracle.cauchy(n, p)
    enc = E.ec_compile_slp(n, p, gen, native=True, split=E.SPLIT_NEVER)
    dec = E.ec_compile_slp(n, p, gen, er, native=True, split=E.SPLIT_NEVER)
    E.ec_program_upload_many([enc, dec])
    d, par = W.empty_blocks(n, S), W.empty_blocks(p, S)
    surv, rec = W.empty_blocks(len(dec.in_blocks), S), W.empty_blocks(len(dec.out_blocks), S)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        E.ec_encode(enc, d, par, S, s)
        E.ec_decode(dec, surv, rec, S, s)
    for rep in range(3):
        data = W.host_blocks(n, S, seed=200 + rep)
        blocks = data + oracle.encode(G, n, p, data, threads=THREADS)
        for t, x in zip(d, data):
            t.copy_(torch.from_numpy(x))
        for t, b in zip(surv, dec.in_blocks):
            t.copy_(torch.from_numpy(blocks[b]))
        for t in par + rec:
            t.fill_(0x5A + rep)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        for j in range(p):
            assert np.array_equal(par[j].cpu().numpy(), blocks[n + j]), "replay %d parity %d" % (rep, j)
        for j, e in enumerate(dec.out_blocks):
            assert np.array_equal(rec[j].cpu().numpy(), blocks[e]), "replay %d block %d" % (rep, e)


@pytest.mark.parametrize("n,p,er,level", [(10, 4, (), E.LEVEL_PLAIN), (10, 4, (), E.LEVEL_CO_FU_SCHED),
                                          (10, 4, (0, 3, 11, 12), E.LEVEL_CO_FU_SCHED), (6, 3, (1, 7), E.LEVEL_PLAIN),
                                          (14, 4, (5,), E.LEVEL_PLAIN)])
def test_native_pairs_and_default_split(n, p, er, level):
    """The native kernels under the default split (pair parts on short
    stripes, block parts on longer ones, the whole program beyond), and the
    pair and block kernels forced on every size: byte for byte against the
    oracle, ragged tails included."""
    gen = oracle_gen(n, p)
    every = E.NATIVE_WHOLE | E.NATIVE_PAIRS | E.NATIVE_BLOCKS
    allk = E.ec_compile_slp(n, p, gen, list(er), level=level, native=every)
    want = every if allk.info["n_parts"] else E.NATIVE_WHOLE | E.NATIVE_PAIRS
    assert allk.info["native"] == want
    run_and_check(allk, n, p, er, (128, 8320, 64 << 10, (512 << 10) + 128, 1 << 20, (2 << 20) + 1152, 8 << 20),
                  seed=n + p + level)
    pairs = E.ec_compile_slp(n, p, gen, list(er), level=level, native=E.NATIVE_PAIRS, split=E.SPLIT_PAIRS)
    assert pairs.info["native"] == E.NATIVE_PAIRS
    run_and_check(pairs, n, p, er, (8320, (1 << 20) + 128, 3 << 20), seed=7 * n + p)
    if allk.info["n_parts"]:
        blocks = E.ec_compile_slp(n, p, gen, list(er), level=level, native=E.NATIVE_BLOCKS, split=E.SPLIT_ALWAYS)
        assert blocks.info["native"] == E.NATIVE_BLOCKS
        run_and_check(blocks, n, p, er, (128, 8320, (1 << 20) + 128, 3 << 20), seed=9 * n + p)


def test_native_pairs_graph_replay():
    """The pair kernel captured in a HIP graph after the upload loads it,
    replayed with new inputs."""
    n, p, S = 10, 4, 256 << 10
    gen = oracle_gen(n, p)
    G = oracle.cauchy(n, p)
    enc = E.ec_compile_slp(n, p, gen, native=E.NATIVE_PAIRS)
    enc.upload()
    d, par = W.empty_blocks(n, S), W.empty_blocks(p, S)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        E.ec_encode(enc, d, par, S, s)
    for rep in range(3):
        data = W.host_blocks(n, S, seed=300 + rep)
        want = oracle.encode(G, n, p, data, threads=THREADS)
        for t, x in zip(d, data):
            t.copy_(torch.from_numpy(x))
        for t in par:
            t.fill_(0x66 + rep)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        for j in range(p):
            assert np.array_equal(par[j].cpu().numpy(), want[j]), "replay %d parity %d" % (rep, j)
