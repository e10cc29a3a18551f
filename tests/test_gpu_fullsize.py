"""Every output byte of the benchmarked configurations against the oracle.

* RS(10,4) encode of 10 x 64 MiB blocks (both program levels the benchmark
  times, under both strip schedulers) and the decode of erasure sets at that size: every byte, the oracle
  running on host threads over disjoint strip-offset ranges.  At 64 MiB the
  executor takes tiles from 8 distant segments of the strips (strips 4 MiB
  apart or a multiple of it); a smaller codec at 32 MiB blocks (4 MiB
  strips) covers the same order in a single launch and in a one-stripe
  batch.
* The 8192-stripe batched mix of the benchmark (four codecs, blocks of
  4 KiB - 4 MiB, 70% encodes), under every (level, slot budget, work-item
  width, strip scheduler) the autotuner chooses between: every output byte of every stripe
  through the bitmatrix relation of ``strip_check`` (the oracle's
  bitmatrix), and a
  seeded subset of stripes, with the largest block of each codec and
  operation, byte for byte against the oracle's encode and decode.

Generators and expected values come from the oracle only.  Outputs are
poisoned before every launch.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import strip_check as SC
import paper_2108_02692_amd as E
from paper_2108_02692_amd import autotune
from paper_2108_02692_amd import batching as B
from paper_2108_02692_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def gen_rows(n, p):
    return [[int(x) for x in row] for row in oracle.cauchy(n, p)]


def first_diff(got: np.ndarray, want: np.ndarray, what: str):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError("%s: %d bytes differ, first at %d" % (what, bad.size, bad[0]))


@pytest.fixture(scope="module")
def rs10_4_64mib():
    torch.cuda.set_device(0)
    n, p, S = 10, 4, 64 << 20
    data = W.device_blocks(n, S, seed=11)
    host = [d.cpu().numpy() for d in data]
    G = oracle.cauchy(n, p)
    par = oracle.encode(G, n, p, host, threads=THREADS)
    yield n, p, S, G, data, host, par
    del data
    torch.cuda.empty_cache()


@pytest.mark.parametrize("level,sched", [(E.LEVEL_CO_FU_SCHED, E.SCHED_PUSH), (E.LEVEL_PLAIN, E.SCHED_PUSH),
                                         (E.LEVEL_CO_FU_SCHED, E.SCHED_GREEDY), (E.LEVEL_PLAIN, E.SCHED_GREEDY)])
def test_encode_64mib_every_byte(rs10_4_64mib, level, sched):
    n, p, S, G, data, host, want = rs10_4_64mib
    prog = E.ec_compile_slp(n, p, gen_rows(n, p), level=level, scheduler=sched)
    out = W.empty_blocks(p, S, fill=0xA5)
    E.ec_encode(prog, data, out, S)
    torch.cuda.synchronize()
    for j in range(p):
        first_diff(out[j].cpu().numpy(), want[j], "64 MiB encode level %d parity %d" % (level, j))


@pytest.mark.parametrize("er", [(2, 4, 5, 6), (4, 5, 6, 7), (0, 11, 13), (12,)])
def test_decode_64mib_every_byte(rs10_4_64mib, er):
    """Survivors = the seeded data and the oracle's parity; every byte of
    every erased block against the oracle's decode (which the oracle's
    round-trip pins make equal to the erased block itself)."""
    n, p, S, G, data, host, par = rs10_4_64mib
    blocks = host + par
    dev = list(data) + W.to_device(par)
    prog = E.ec_compile_slp(n, p, gen_rows(n, p), list(er))
    rec = W.empty_blocks(len(er), S, fill=0xA5)
    E.ec_decode(prog, [dev[i] for i in prog.in_blocks], rec, S)
    torch.cuda.synchronize()
    want = oracle.decode(G, n, p, list(er), [None if i in er else blocks[i] for i in range(n + p)],
                         threads=THREADS)
    for j, e in enumerate(prog.out_blocks):
        got = rec[j].cpu().numpy()
        first_diff(got, want[list(er).index(e)], "64 MiB decode %s block %d" % (er, e))
        first_diff(got, blocks[e], "64 MiB decode %s block %d vs original" % (er, e))


@pytest.mark.parametrize("level", [E.LEVEL_CO_FU_SCHED, E.LEVEL_PLAIN])
def test_native_64mib_every_byte(rs10_4_64mib, level):
    """The native kernels of the benchmarked programs on the 64 MiB encode
    and the {2,4,5,6} decode: every byte against the oracle."""
    n, p, S, G, data, host, par = rs10_4_64mib
    gen = gen_rows(n, p)
    enc = E.ec_compile_slp(n, p, gen, level=level, native=True)
    out = W.empty_blocks(p, S, fill=0xA5)
    E.ec_encode(enc, data, out, S)
    torch.cuda.synchronize()
    for j in range(p):
        first_diff(out[j].cpu().numpy(), par[j], "native 64 MiB encode level %d parity %d" % (level, j))
    del out
    er = [2, 4, 5, 6]
    blocks = host + par
    dev = list(data) + W.to_device(par)
    dec = E.ec_compile_slp(n, p, gen, er, level=level, native=True)
    rec = W.empty_blocks(len(er), S, fill=0xA5)
    E.ec_decode(dec, [dev[i] for i in dec.in_blocks], rec, S)
    torch.cuda.synchronize()
    for j, e in enumerate(dec.out_blocks):
        first_diff(rec[j].cpu().numpy(), blocks[e], "native 64 MiB decode %s block %d" % (er, e))


@pytest.mark.parametrize("level", [E.LEVEL_CO_FU_SCHED, E.LEVEL_PLAIN])
def test_staged_64mib_every_byte(rs10_4_64mib, level):
    """The staged launch (tiles copied into LDS, one workgroup per tile) on
    the 64 MiB encode and the {2,4,5,6} decode: every byte against the
    oracle."""
    n, p, S, G, data, host, par = rs10_4_64mib
    gen = gen_rows(n, p)
    enc = E.ec_compile_slp(n, p, gen, level=level, split=E.SPLIT_STAGED)
    out = W.empty_blocks(p, S, fill=0xA5)
    E.ec_encode(enc, data, out, S)
    torch.cuda.synchronize()
    for j in range(p):
        first_diff(out[j].cpu().numpy(), par[j], "staged 64 MiB encode level %d parity %d" % (level, j))
    del out
    er = [2, 4, 5, 6]
    blocks = host + par
    dev = list(data) + W.to_device(par)
    dec = E.ec_compile_slp(n, p, gen, er, level=level, split=E.SPLIT_STAGED)
    rec = W.empty_blocks(len(er), S, fill=0xA5)
    E.ec_decode(dec, [dev[i] for i in dec.in_blocks], rec, S)
    torch.cuda.synchronize()
    for j, e in enumerate(dec.out_blocks):
        first_diff(rec[j].cpu().numpy(), blocks[e], "staged 64 MiB decode %s block %d" % (er, e))


def test_segment_order_single_launch_and_batch():
    """RS(4,2) on 32 MiB blocks (4 MiB strips: the segment tile order),
    encode and a two-block decode, as single launches and as one-stripe
    batches, every byte against the oracle."""
    n, p, S = 4, 2, 32 << 20
    G = oracle.cauchy(n, p)
    gen = gen_rows(n, p)
    data = W.device_blocks(n, S, seed=41)
    host = [d.cpu().numpy() for d in data]
    par = oracle.encode(G, n, p, host, threads=THREADS)
    blocks_h = host + par
    dev = list(data) + W.to_device(par)
    er = [1, 4]
    enc = E.ec_compile_slp(n, p, gen)
    dec = E.ec_compile_slp(n, p, gen, er)
    want_dec = oracle.decode(G, n, p, er, [None if i in er else blocks_h[i] for i in range(n + p)],
                             threads=THREADS)
    stream = torch.cuda.current_stream()
    for mode in ("single", "batch"):
        out = W.empty_blocks(p, S, fill=0xA5)
        rec = W.empty_blocks(len(er), S, fill=0xA5)
        surv = [dev[i] for i in dec.in_blocks]
        if mode == "single":
            E.ec_encode(enc, data, out, S, stream)
            E.ec_decode(dec, surv, rec, S, stream)
        else:
            for prog, ins, outs in ((enc, data, out), (dec, surv, rec)):
                b = E.ec_batch_build([(prog, ins, outs, S)], stream=stream)
                b.launch(stream)
                torch.cuda.synchronize()
                b.free()
        torch.cuda.synchronize()
        for j in range(p):
            first_diff(out[j].cpu().numpy(), par[j], "%s encode parity %d" % (mode, j))
        for j, e in enumerate(dec.out_blocks):
            first_diff(rec[j].cpu().numpy(), want_dec[er.index(e)], "%s decode block %d" % (mode, e))


@pytest.mark.parametrize("n,p,er,K,native", [(12, 6, (), 48, 0), (12, 6, (0, 3, 7, 12, 16, 17), 48, 0),
                                             (4, 12, (), 0, 0), (12, 6, (), 0, 0), (12, 6, (0, 3, 7, 12, 16, 17), 0, 0),
                                             (10, 6, (), 0, 0), (12, 6, (), 0, 1), (10, 6, (1, 4, 9, 11, 13, 15), 0, 1)])
def test_wide_codecs_64mib_every_byte(n, p, er, K, native):
    """Codecs with more rows than 48 slots hold: by default a 56- or
    60-slot program in one pass where the rows fit, else (and with 48 slots
    forced) several passes run as pass parts, the library's default for such
    stripes; the one-pass programs also as native kernels.  64 MiB blocks,
    every byte of every output against the oracle."""
    S = 64 << 20
    G = oracle.cauchy(n, p)
    data = W.device_blocks(n, S, seed=n + 7 * p)
    host = [d.cpu().numpy() for d in data]
    par = oracle.encode(G, n, p, host, threads=THREADS)
    prog = E.ec_compile_slp(n, p, gen_rows(n, p), list(er), slot_budget=K, native=native)
    assert prog.info["native"] == native
    if K == 48 or (n, p) == (4, 12):
        assert prog.info["passes"] > 1 and prog.info["n_pass_parts"] >= prog.info["passes"]
    else:
        assert prog.info["passes"] == 1 and prog.info["slots"] in (56, 60)
    if er:
        blocks = host + par
        dev = list(data) + W.to_device(par)
        out = W.empty_blocks(len(er), S, fill=0xA5)
        E.ec_decode(prog, [dev[i] for i in prog.in_blocks], out, S)
        torch.cuda.synchronize()
        want = [blocks[e] for e in prog.out_blocks]
    else:
        out = W.empty_blocks(p, S, fill=0xA5)
        E.ec_encode(prog, data, out, S)
        torch.cuda.synchronize()
        want = par
    for j, w in enumerate(want):
        first_diff(out[j].cpu().numpy(), w, "RS(%d,%d) %s K %d, output %d" % (n, p, er, K, j))
    del data, out
    torch.cuda.empty_cache()


def _subset(specs, count=24, seed=8):
    """The largest stripe of each (codec, encode/decode), then seeded others."""
    pick = {}
    for k, s in enumerate(specs):
        key = (s.n, s.p, bool(s.erased))
        if key not in pick or s.block_bytes > specs[pick[key]].block_bytes:
            pick[key] = k
    chosen = set(pick.values())
    rng = np.random.default_rng(seed)
    for k in rng.permutation(len(specs)).tolist():
        if len(chosen) >= len(pick) + count:
            break
        chosen.add(k)
    return sorted(chosen)


@pytest.fixture(scope="module")
def mix8192():
    torch.cuda.set_device(0)
    # a 4 GiB pool that stripes share (the benchmark gives each its own
    # bytes; sharing changes no result and keeps the host copy small)
    specs, pool, inputs, outputs, out_buf = B.mixed_workload(8192, pool_bytes=4 << 30)
    pool_h = pool.cpu().numpy()
    base = pool.data_ptr()
    offs = [[t.data_ptr() - base for t in ins] for ins in inputs]
    M = SC.masks(max(s.block_bytes for s in specs) // 64)
    mats = {}

    def matrix(s, in_blocks):
        key = (s.n, s.p, s.erased)
        if key not in mats:
            mats[key] = SC.stripe_matrix(oracle.cauchy(s.n, s.p), s.n, s.p, s.erased, in_blocks)
        return mats[key]

    def fin(k):
        s = specs[k]
        return np.concatenate([SC.strip_fingerprints(pool_h[o:o + s.block_bytes], M) for o in offs[k]])

    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        fins = list(ex.map(fin, range(len(specs))))
    yield specs, inputs, outputs, out_buf, pool_h, offs, M, fins, matrix
    del pool, inputs, outputs, out_buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("level,slots,tile,sched", autotune.DEFAULT_CANDIDATES)
def test_batch_8192_mix_every_byte(mix8192, level, slots, tile, sched):
    specs, inputs, outputs, out_buf, pool_h, offs, M, fins, matrix = mix8192
    cache = B.ProgramCache(level=level, slots=slots, generator_fn=oracle.cauchy, scheduler=sched)
    cache.warm({(s.n, s.p, s.erased) for s in specs})
    stream = torch.cuda.current_stream()
    batch = B.build_batch(specs, cache, inputs, outputs, tile_bytes=tile, stream=stream)
    out_buf.fill_(0xA5)
    torch.cuda.synchronize()
    batch.launch(stream)
    torch.cuda.synchronize()
    out_h = out_buf.cpu().numpy()
    obase = out_buf.data_ptr()

    def out_blocks(k):
        s = specs[k]
        return [out_h[t.data_ptr() - obase: t.data_ptr() - obase + s.block_bytes] for t in outputs[k]]

    def check(k):
        s = specs[k]
        prog = cache.get(s.n, s.p, s.erased)
        fout = np.concatenate([SC.strip_fingerprints(b, M) for b in out_blocks(k)])
        want = SC.expected_from_inputs(matrix(s, prog.in_blocks), fins[k])
        return [k] if np.any(fout != want) else []

    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        bad = sum(ex.map(check, range(len(specs))), [])
    assert not bad, "%d stripes fail the bitmatrix relation, first %d (%s)" % (len(bad), bad[0], specs[bad[0]])
    for k in _subset(specs):
        s = specs[k]
        prog = cache.get(s.n, s.p, s.erased)
        ins = [pool_h[o:o + s.block_bytes] for o in offs[k]]
        G = oracle.cauchy(s.n, s.p)
        if not s.erased:
            want = oracle.encode(G, s.n, s.p, ins, threads=THREADS)
        else:
            blocks = [None] * (s.n + s.p)
            for i, b in zip(prog.in_blocks, ins):
                blocks[i] = b
            want = oracle.decode(G, s.n, s.p, list(s.erased), blocks, threads=THREADS)
        for j, got in enumerate(out_blocks(k)):
            first_diff(got, want[j], "stripe %d %s output %d" % (k, s, j))
    batch.free()
