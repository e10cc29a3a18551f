"""Product compiler (host side of libec) against the oracle, on the CPU.

* bitmatrix / plain program: equal to the oracle's bitmatrix of the same
  generator (the one deliberate cross-check of Sec. 1 (ii) between the two);
* XorRePair, fusion, DFS stages and the greedy schedule: statement-for-
  statement equal to the oracle's implementation of Secs. 4-6 (same
  readings of the tie-breaks);
* the executed program and its device bytecode: the bitmatrix rows under the
  set semantics of Sec. 4.1, checked by the independent bytecode simulator;
* error handling of ec_compile_slp.
"""
import itertools
import random

import numpy as np
import pytest

import oracle
from oracle import slp as S
import paper_2108_02692_amd as E
from bytecode_sim import fields, simulate

BIG = S.Compressed.BIG


def oracle_rows(gen, n, p, erased=()):
    G = np.array(gen, dtype=np.uint8)
    if erased:
        D, _ = oracle.decode_matrix(G, n, p, list(erased))
    else:
        D = G[n:]
    return S.rows_from_bitmatrix(oracle.bitmatrix(D))


def to_oracle_terms(stmts, outs):
    """Product export terms -> oracle key space (temps as is, const c -> BIG+c)."""
    def t(x):
        if x == -1:
            return S.ZERO
        if x <= -2:
            return BIG + (-x - 2)
        return x
    return [(v, [t(o) for o in ops]) for v, ops in stmts], [t(o) for o in outs]


def eval_export(stmts, outs):
    env = {}

    def val(x):
        if x == -1:
            return 0
        if x <= -2:
            return 1 << (-x - 2)
        return env[x]
    for v, ops in stmts:
        acc = 0
        for o in ops:
            acc ^= val(o)
        env[v] = acc
    return [val(o) for o in outs]


CODECS = [(10, 4), (6, 3), (12, 4), (14, 4)]


def test_generator_matches_oracle():
    """Every codec the library's generators accept (n >= 1, p >= 0,
    n + p <= 64)."""
    for n in range(1, 65):
        for p in range(0, 65 - n):
            assert np.array_equal(np.array(E.ec_matrix_cauchy(n, p), dtype=np.uint8), oracle.cauchy(n, p)), (n, p)
            assert np.array_equal(np.array(E.ec_matrix_vandermonde(n, p), dtype=np.uint8),
                                  oracle.vandermonde_rows(n, p)), (n, p)


def sample_patterns(n, p, k, seed):
    rng = random.Random(seed)
    pats = [()]
    allp = [c for r in range(1, p + 1) for c in itertools.combinations(range(n + p), r)]
    pats += rng.sample(allp, k)
    return pats


@pytest.mark.parametrize("n,p", CODECS)
def test_plain_program_is_oracle_bitmatrix(n, p):
    gen = E.ec_matrix_cauchy(n, p)
    for er in sample_patterns(n, p, 6, n):
        prog = E.ec_compile_slp(n, p, gen, er, level=E.LEVEL_PLAIN)
        stmts, outs = prog.export(E.STAGE_PLAIN)
        assert eval_export(stmts, outs) == oracle_rows(gen, n, p, er)
        if er:
            assert prog.in_blocks == oracle.survivors(n, p, er)
            assert prog.out_blocks == list(er)


def test_paper_matrix_plain_counts():
    gen = E.ec_matrix_vandermonde(10, 4)
    enc = E.ec_compile_slp(10, 4, gen, level=E.LEVEL_PLAIN)
    assert enc.info["plain_xor2"] == 755
    dec = E.ec_compile_slp(10, 4, gen, [2, 4, 5, 6], level=E.LEVEL_PLAIN)
    assert dec.info["plain_xor2"] == 1368


def oracle_pipeline(rows, n_const, rebuild=True):
    comp = S.repair(rows, n_const, xor_rebuild=rebuild)
    st, outs = comp.to_program()
    fu = S.fuse(st, outs, comp.is_const)
    dfs = S.dfs_order(fu, outs, comp.is_const)
    return (st, outs), fu, dfs


@pytest.mark.parametrize("n,p,er,rebuild", [
    (10, 4, (), True), (10, 4, (2, 4, 5, 6), True), (10, 4, (0, 13), True), (6, 3, (), True),
    (6, 3, (1, 7, 8), True), (10, 4, (), False)])
def test_stages_equal_oracle(n, p, er, rebuild):
    gen = E.ec_matrix_cauchy(n, p)
    rows = oracle_rows(gen, n, p, er)
    (co_st, co_out), fu, dfs = oracle_pipeline(rows, 8 * n, rebuild)
    prog = E.ec_compile_slp(n, p, gen, er, compress=E.COMPRESS_XORREPAIR if rebuild else E.COMPRESS_REPAIR)
    got_co = to_oracle_terms(*prog.export(E.STAGE_CO))
    assert got_co == (co_st, co_out)
    got_fu, outs = to_oracle_terms(*prog.export(E.STAGE_FU))
    assert got_fu == fu and outs == co_out
    got_dfs, _ = to_oracle_terms(*prog.export(E.STAGE_SCHED))
    assert got_dfs == dfs


def test_paper_matrix_stages_equal_oracle():
    gen = E.ec_matrix_vandermonde(10, 4)
    rows = oracle_rows(gen, 10, 4)
    (co_st, co_out), fu, dfs = oracle_pipeline(rows, 80)
    prog = E.ec_compile_slp(10, 4, gen)
    assert to_oracle_terms(*prog.export(E.STAGE_CO)) == (co_st, co_out)
    assert to_oracle_terms(*prog.export(E.STAGE_SCHED))[0] == dfs


def pebbled(stmts, outs):
    """Library greedy export -> the oracle's pebbled form."""
    t = lambda x: BIG + (-x - 2) if x <= -2 else ("p", x)
    return [(("p", v), [t(o) for o in ops]) for v, ops in stmts], [t(o) for o in outs]


@pytest.mark.parametrize("n,p,er,mat", [
    (10, 4, (), "cauchy"), (10, 4, (2, 4, 5, 6), "cauchy"), (6, 3, (1, 7), "cauchy"), (10, 4, (), "vandermonde"),
    (10, 4, (2, 4, 5, 6), "vandermonde")])
def test_greedy_schedule_equals_oracle(n, p, er, mat):
    gen = (E.ec_matrix_cauchy if mat == "cauchy" else E.ec_matrix_vandermonde)(n, p)
    rows = oracle_rows(gen, n, p, er)
    (_, outs), fu, _ = oracle_pipeline(rows, 8 * n)
    prog = E.ec_compile_slp(n, p, gen, er)
    isc = lambda t: isinstance(t, int) and t >= BIG
    want = S.evaluate(fu, outs, 0, isc)
    for cap in (4, 8, 32, 128, 1000):
        peb, ret, npeb = S.greedy_schedule(fu, outs, isc, cap)
        got, got_ret = pebbled(*prog.export_greedy(cap))
        assert got == peb and got_ret == ret
        assert S.evaluate(got, got_ret, 0, isc) == want


def test_greedy_export_errors():
    gen = E.ec_matrix_cauchy(6, 3)
    with pytest.raises(E.EcError, match="EC_ERR_ARG"):
        E.ec_compile_slp(6, 3, gen).export_greedy(0)
    for level in (E.LEVEL_PLAIN, E.LEVEL_CO):
        with pytest.raises(E.EcError, match="EC_ERR_ARG"):
            E.ec_compile_slp(6, 3, gen, level=level).export_greedy(8)
    assert E.ec_compile_slp(6, 3, gen, level=E.LEVEL_CO_FU).export_greedy(8)[0]


@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO, E.LEVEL_CO_FU, E.LEVEL_CO_FU_SCHED])
@pytest.mark.parametrize("K", [24, 32, 36, 38, 40, 44, 48, 56, 60])
def test_bytecode_simulates_to_bitmatrix(level, K):
    n, p = 10, 4
    gen = E.ec_matrix_cauchy(n, p)
    for er in sample_patterns(n, p, 2, K + level):
        prog = E.ec_compile_slp(n, p, gen, er, level=level, slot_budget=K)
        rows = oracle_rows(gen, n, p, er)
        stmts, outs = prog.export(E.STAGE_EXEC)
        assert eval_export(stmts, outs) == rows
        got = simulate(prog.bytecode(), K, n, len(prog.out_blocks))
        assert [got[o] for o in range(len(rows))] == rows
        assert prog.info["n_stores"] == len(rows)
        assert prog.info["slots"] == K
        assert prog.info["n_loads"] == 80 * prog.info["passes"]


def load_order(words):
    """Input strips in the order the records load them (LOAD and INPUT_LD
    records; strip 8 * block + j)."""
    out, pc = [], 0
    while pc < len(words):
        f = fields(words[pc], words[pc + 1])
        if f["kind"] == 6:  # HALT
            break
        if f["kind"] in (2, 5):
            out.append(8 * f["blk"] + f["j"])
        pc += f["bytes"] // 4
    return out


def greedy_first_reads(stmts, outs, capacity, width):
    """The order in which the oracle's bottom-up greedy heuristic (Sec. 6.6)
    first reads the input strips of a program, for an LRU cache of
    `capacity` entries; with width > 0, stable by column block."""
    st, ou = to_oracle_terms(stmts, outs)
    isc = lambda t: isinstance(t, int) and t >= BIG
    peb, _, _ = S.greedy_schedule(st, ou, isc, capacity)
    seen = []
    for _, args in peb:
        for a in args:
            if isc(a) and a - BIG not in seen:
                seen.append(a - BIG)
    return sorted(seen, key=lambda c: c // width) if width else seen


@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO, E.LEVEL_CO_FU, E.LEVEL_CO_FU_SCHED])
@pytest.mark.parametrize("K", [24, 32, 36, 38, 40, 44, 48, 56, 60])
def test_greedy_scheduler_programs(level, K):
    """EC_SCHED_GREEDY at every level and slot budget: the records compute
    the bitmatrix rows (independent simulator), and a single-pass program
    loads the strips in the order the oracle's greedy heuristic first reads
    them in the program's statements, with the slot budget as the cache."""
    n, p = 10, 4
    gen = E.ec_matrix_cauchy(n, p)
    for er in sample_patterns(n, p, 2, 3 * K + level):
        prog = E.ec_compile_slp(n, p, gen, er, level=level, slot_budget=K, scheduler=E.SCHED_GREEDY)
        assert prog.info["scheduler"] == E.SCHED_GREEDY
        rows = oracle_rows(gen, n, p, er)
        stmts, outs = prog.export(E.STAGE_EXEC)
        assert eval_export(stmts, outs) == rows
        got = simulate(prog.bytecode(), K, n, len(prog.out_blocks))
        assert [got[o] for o in range(len(rows))] == rows
        for k in range(prog.info["n_parts"] + prog.info["n_row_parts"] + prog.info["n_pair_parts"]):
            part = simulate(prog.part_bytecode(k), K, n, len(prog.out_blocks))
            assert all(part[o] == rows[o] for o in part)
        if prog.info["passes"] == 1:
            want = greedy_first_reads(stmts, outs, K, 8 if level >= E.LEVEL_CO else 0)
            assert load_order(prog.bytecode()) == want


def test_schedulers_differ_and_default_is_push():
    gen = E.ec_matrix_cauchy(10, 4)
    push = E.ec_compile_slp(10, 4, gen, level=E.LEVEL_CO_FU)
    greedy = E.ec_compile_slp(10, 4, gen, level=E.LEVEL_CO_FU, scheduler=E.SCHED_GREEDY)
    assert push.info["scheduler"] == E.SCHED_PUSH
    assert load_order(push.bytecode()) != load_order(greedy.bytecode())
    with pytest.raises(E.EcError, match="EC_ERR_UNSUPPORTED"):
        E.ec_compile_slp(10, 4, gen, scheduler=2)


@pytest.mark.parametrize("n,p", [(6, 3), (12, 4), (14, 4)])
def test_bytecode_other_codecs(n, p):
    gen = E.ec_matrix_cauchy(n, p)
    for er in sample_patterns(n, p, 3, 7 * n):
        for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
            prog = E.ec_compile_slp(n, p, gen, er, level=level)
            rows = oracle_rows(gen, n, p, er)
            got = simulate(prog.bytecode(), prog.info["slots"], n, len(prog.out_blocks))
            assert [got[o] for o in range(len(rows))] == rows


def test_wide_codec_needs_row_passes():
    # 8 parity blocks = 64 rows: more than the slots, so the inputs stream
    # through once per group of output blocks
    n, p = 8, 8
    gen = E.ec_matrix_cauchy(n, p)
    for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
        prog = E.ec_compile_slp(n, p, gen, level=level, slot_budget=48)
        assert prog.info["passes"] >= 2
        rows = oracle_rows(gen, n, p)
        got = simulate(prog.bytecode(), 48, n, p, tiles=3)
        assert [got[o] for o in range(64)] == rows


@pytest.mark.parametrize("width", [1, 4, 8, 16, 40])
def test_block_width_option_keeps_semantics(width):
    gen = E.ec_matrix_cauchy(10, 4)
    rows = oracle_rows(gen, 10, 4)
    prog = E.ec_compile_slp(10, 4, gen, block_strips=width, slot_budget=48)
    got = simulate(prog.bytecode(), 48, 10, 4)
    assert [got[o] for o in range(32)] == rows


@pytest.mark.parametrize("dist", [1, 4, 12, 64])
def test_prefetch_distance_keeps_semantics(dist):
    gen = E.ec_matrix_cauchy(10, 4)
    for er, level in (((), E.LEVEL_PLAIN), ((), E.LEVEL_CO_FU_SCHED), ((1, 7, 12), E.LEVEL_CO_FU_SCHED)):
        rows = oracle_rows(gen, 10, 4, er)
        prog = E.ec_compile_slp(10, 4, gen, er, level=level, prefetch=dist)
        got = simulate(prog.bytecode(), prog.info["slots"], 10, len(prog.out_blocks))
        assert [got[o] for o in range(len(rows))] == rows


def test_compressed_beats_plain_in_xors():
    gen = E.ec_matrix_cauchy(10, 4)
    plain = E.ec_compile_slp(10, 4, gen, level=E.LEVEL_PLAIN)
    co = E.ec_compile_slp(10, 4, gen)
    assert co.info["n_xor2"] < plain.info["n_xor2"] == 1256
    # the executor's unit of work: one slot XOR (plain: every 1 bit, plus
    # clearing the 32 row slots after their store and the ring slots at the
    # end of the tile)
    assert 1288 + 32 <= plain.info["n_ops"] <= 1288 + 32 + plain.info["ring"]
    assert co.info["n_ops"] < 0.75 * plain.info["n_ops"]


def test_compile_errors():
    gen = E.ec_matrix_cauchy(10, 4)
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, gen, [0, 1, 2, 3, 4])
    assert e.value.name == "EC_ERR_TOO_MANY_ERASURES"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, gen, [0, 0])
    assert e.value.name == "EC_ERR_ARG"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, gen, [14])
    assert e.value.name == "EC_ERR_ARG"
    bad = [list(r) for r in gen]
    bad[10] = list(bad[11])
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, bad, [0, 1, 2, 3])
    assert e.value.name == "EC_ERR_SINGULAR"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, gen, slot_budget=20)
    assert e.value.name == "EC_ERR_UNSUPPORTED"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, gen, block_strips=81)
    assert e.value.name == "EC_ERR_ARG"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, gen, split=E.SPLIT_STAGED + 1)
    assert e.value.name == "EC_ERR_UNSUPPORTED"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(30, 4, E.ec_matrix_cauchy(30, 4))
    assert e.value.name == "EC_ERR_ARG"


@pytest.mark.parametrize("n,p,er", [(10, 4, ()), (10, 4, (2, 4, 5, 6)), (6, 3, (1, 7)), (14, 4, (0, 13)),
                                    (28, 4, ()), (4, 12, ()), (10, 2, (8, 9)), (2, 10, ()), (3, 13, ()),
                                    (4, 12, tuple(range(1, 12))), (20, 9, ())])
@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED])
def test_row_split_parts_cover_the_rows(n, p, er, level):
    """Every row-split part, run by the independent simulator, stores only its
    own output rows; each set of parts (blocks, single rows, pairs of rows,
    passes) stores every output strip with the bitmatrix row's value, exactly
    once."""
    gen = E.ec_matrix_cauchy(n, p)
    rows = oracle_rows(gen, n, p, er)
    prog = E.ec_compile_slp(n, p, gen, er, level=level)
    n_out = len(prog.out_blocks)
    nb, nr, npair = prog.info["n_parts"], prog.info["n_row_parts"], prog.info["n_pair_parts"]
    npass = prog.info["n_pass_parts"]
    assert nb == (min(n_out, 8) if n_out > 1 else 0) or nb == 0
    assert nr == min(8 * n_out, 32) or nr == 0
    assert npair == min(4 * n_out, 16) or npair == 0
    assert (npass >= prog.info["passes"]) if prog.info["passes"] > 1 else npass == 0

    def sizes(unit, groups):  # rows per part of a set of runs of `unit` rows
        units = 8 * n_out // unit
        return {unit * (units // groups), unit * -(-units // groups)} - {0}
    n4 = nb + nr + npair
    for lo, hi, kind in ((0, nb, "block"), (nb, nb + nr, "row"), (nb + nr, n4, "pair"), (n4, n4 + npass, "pass")):
        got = {}
        for q in range(lo, hi):
            part = simulate(prog.part_bytecode(q), prog.info["slots"], len(prog.in_blocks), n_out)
            assert part and not set(part) & set(got)
            if kind in ("block", "pass"):
                assert all(8 * (o // 8) + j in part for o in part for j in range(8))
            else:  # a run of rows right after the previous part's, of even size
                assert sorted(part) == list(range(len(got), len(got) + len(part)))
                assert len(part) in sizes(1 if kind == "row" else 2, hi - lo), (kind, len(part))
            got.update(part)
        if hi > lo:
            assert [got[o] for o in range(len(rows))] == rows
    info = E.ec_compile_slp(n, p, gen, er, level=level, split=E.SPLIT_NEVER).info
    assert info["n_parts"] == 0 and info["n_row_parts"] == 0 and info["n_pair_parts"] == 0
    assert info["n_pass_parts"] == 0
    with pytest.raises(E.EcError):
        prog.part_bytecode(n4 + npass)
    with pytest.raises(E.EcError):
        prog.part_bytecode(-1)


@pytest.mark.parametrize("n,p,er", [(10, 4, ()), (10, 4, (2, 4, 5, 6)), (6, 3, (1, 7)), (14, 4, (0, 13)),
                                    (4, 12, ()), (20, 9, ()), (2, 1, ()), (1, 1, ()), (12, 6, ()),
                                    (4, 12, tuple(range(1, 12)))])
@pytest.mark.parametrize("level", [E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED])
def test_stage_parts_cover_the_rows(n, p, er, level):
    """A staged program carries min(4, rows) stage parts and no other parts;
    run by the independent simulator, the parts store consecutive runs of
    rows that differ in size by at most one, together every output strip
    with the bitmatrix row's value, exactly once, and make no prefetch
    records (their loads read LDS)."""
    gen = E.ec_matrix_cauchy(n, p)
    rows = oracle_rows(gen, n, p, er)
    prog = E.ec_compile_slp(n, p, gen, er, level=level, split=E.SPLIT_STAGED)
    info = prog.info
    n_rows = len(rows)
    assert info["n_stage_parts"] == min(4, n_rows)
    assert info["n_parts"] == info["n_row_parts"] == info["n_pair_parts"] == info["n_pass_parts"] == 0
    got = {}
    for q in range(info["n_stage_parts"]):
        words = prog.part_bytecode(q)
        part = simulate(words, info["slots"], len(prog.in_blocks), len(prog.out_blocks))
        assert sorted(part) == list(range(len(got), len(got) + len(part)))
        assert len(part) in (n_rows // info["n_stage_parts"], -(-n_rows // info["n_stage_parts"]))
        got.update(part)
        pc = 0
        while True:
            f = fields(words[pc], words[pc + 1])
            assert f["kind"] != 7, "prefetch record in a stage part"
            if f["kind"] == 6:
                break
            pc += f["bytes"] // 4
    assert [got[o] for o in range(n_rows)] == rows
    with pytest.raises(E.EcError):
        prog.part_bytecode(info["n_stage_parts"])
    # the whole program is still there (a batch runs it whole)
    assert simulate(prog.bytecode(), info["slots"], len(prog.in_blocks), len(prog.out_blocks)) == \
        {o: rows[o] for o in range(n_rows)}


def test_staged_limits():
    """Staging holds 8 KiB of LDS per input block: at most 20 input blocks."""
    E.ec_compile_slp(20, 4, E.ec_matrix_cauchy(20, 4), split=E.SPLIT_STAGED, level=E.LEVEL_PLAIN)
    for n, p in ((21, 2), (28, 4)):
        with pytest.raises(E.EcError) as e:
            E.ec_compile_slp(n, p, E.ec_matrix_cauchy(n, p), split=E.SPLIT_STAGED)
        assert e.value.name == "EC_ERR_UNSUPPORTED"
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(10, 4, E.ec_matrix_cauchy(10, 4), split=E.SPLIT_STAGED + 1)
    assert e.value.name == "EC_ERR_UNSUPPORTED"
