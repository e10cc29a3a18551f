"""Pins for the oracle's SLP passes against the paper's worked examples
(Secs. 2, 4, 5, 6), brute force on tiny instances, and the printed operation
counts of the RS(10,4) programs (Sec. 7.5)."""
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle import slp as S

BIG = S.Compressed.BIG
a, b, c, d, e, f, g = range(7)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """A fixture of values printed in the paper (each file cites its source)."""
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        return json.load(fh)


def letters_to_bits(ops, names):
    return sum(1 << names.index(x) for x in ops)


def bits(*cs):
    return sum(1 << x for x in cs)


def temps_named(comp):
    """Render temporaries with constants as letters, temps as t1, t2..."""
    def nm(t):
        return "abcdefg"[t - BIG] if t >= BIG else "t%d" % (t + 1)
    return [(nm(x), nm(y)) for x, y in comp.temps]


# P0 of Sec. 4.2: v1=a^b, v2=a^b^c, v3=a^b^c^d, v4=b^c^d
G_P0 = golden("p0_repair")
P0 = [letters_to_bits(G_P0["program"][v], G_P0["constants"]) for v in ("v1", "v2", "v3", "v4")]


def test_repair_on_P0_matches_worked_example():
    comp = S.repair(P0, 4, xor_rebuild=False)
    assert temps_named(comp) == [tuple(t) for t in G_P0["repair_temps"]]
    assert eval_comp(comp) == P0


def eval_comp(comp):
    stmts, outs = comp.to_program()
    env = {}
    def val(t):
        if t == S.ZERO:
            return 0
        return (1 << (t - BIG)) if t >= BIG else env[t]
    for v, ops in stmts:
        env[v] = val(ops[0]) ^ val(ops[1])
    return [val(t) for t in outs]


def test_xorrepair_on_P0_uses_cancellation():
    comp = S.repair(P0, 4, xor_rebuild=True)
    assert temps_named(comp) == [tuple(t) for t in G_P0["xorrepair_temps"]]
    assert eval_comp(comp) == P0


def shortest_xor_count(targets, n_const, max_k, disjoint_only=False):
    """Brute force: least number of binary XORs producing every target value
    (constants are free).  With ``disjoint_only`` XORs may only join disjoint
    sets, i.e. no cancellation."""
    consts = [1 << i for i in range(n_const)]
    need = set(targets) - set(consts)

    def search(have, k):
        if need <= have:
            return True
        if k == 0:
            return False
        terms = sorted(have | set(consts))
        for x, y in itertools.combinations(terms, 2):
            if disjoint_only and (x & y):
                continue
            z = x ^ y
            if z == 0 or z in have or z in consts:
                continue
            if search(have | {z}, k - 1):
                return True
        return False

    for k in range(max_k + 1):
        if search(frozenset(), k):
            return k
    return None


def test_P0_optimality_bruteforce():
    # Sec. 4.2: no equivalent program below 4 XORs, and none below 5 without
    # cancellation
    assert shortest_xor_count(P0, 4, 4) == G_P0["shortest_xors"]
    assert shortest_xor_count(P0, 4, 5, disjoint_only=True) == G_P0["shortest_xors_without_cancellation"]


@pytest.mark.parametrize("seed", range(12))
def test_xorrepair_bounded_by_bruteforce_on_tiny_instances(seed):
    """Random targets over 4 constants: XorRePair's program computes every
    target, and its XOR count lies between the shortest program found by
    exhaustive search (Sec. 4: the shortest-SLP problem it approximates) and
    the plain count; RePair, which cannot cancel, is never shorter than the
    shortest program without cancellation."""
    rng = random.Random(seed)
    targets = []
    while len(targets) < rng.randint(2, 4):
        t = rng.randint(1, 15)
        if bin(t).count("1") >= 2 and t not in targets:
            targets.append(t)
    plain = sum(bin(t).count("1") - 1 for t in targets)
    comp = S.repair(targets, 4, xor_rebuild=True)
    assert eval_comp(comp) == targets
    n_x = len(comp.temps)
    best = shortest_xor_count(targets, 4, plain)
    assert best is not None and best <= n_x <= plain, (targets, best, n_x, plain)
    rp = S.repair(targets, 4, xor_rebuild=False)
    assert eval_comp(rp) == targets
    best_disjoint = shortest_xor_count(targets, 4, plain, disjoint_only=True)
    assert best_disjoint <= len(rp.temps) <= plain, (targets, best_disjoint, len(rp.temps))


def test_intro_example_compress_and_fuse():
    gx = golden("intro_example")
    rows = [letters_to_bits(gx["program"][v], gx["constants"]) for v in ("nu1", "nu2", "nu3")]
    assert sum(r.bit_count() - 1 for r in rows) == gx["plain_xors"]
    comp = S.repair(rows, 7, xor_rebuild=True)
    assert comp.xor_count() == gx["compressed_xors"]
    assert eval_comp(comp) == rows
    stmts, outs = comp.to_program()
    fused = S.fuse(stmts, outs, comp.is_const)
    assert len(fused) == gx["fused_statements"]
    assert S.count_mem(fused) == gx["fused_memory_accesses"] and S.count_xor(fused) == gx["compressed_xors"]


def named_program(prog, base=100):
    """[(name, [ops])] with constants as letters -> integer program (constants
    a.. -> 0.., variables -> base..)."""
    ids = {}
    out = []
    for v, ops in prog:
        conv = [("abcdefg".index(o) if o in "abcdefg" else ids[o]) for o in ops]
        ids.setdefault(v, base + len(ids))
        out.append((ids[v], conv))
    return out, ids


def test_fusion_worked_example():
    gx = golden("fusion_examples")["chain"]
    prog, ids = named_program(gx["program"])
    isc = lambda t: t < 100
    fused = S.fuse(prog, [ids[o] for o in gx["outputs"]], isc)
    want, _ = named_program(gx["fused"])
    assert [(v, ops) for v, ops in fused] == [(ids[gx["fused"][0][0]], want[0][1])]


def test_memory_access_counts_A_B_C():
    gx = golden("fusion_examples")
    # A: the binary version of B's two outputs (a^b^c^d^e then ^f / ^g)
    A_bin = []
    for name, last in ((200, f), (300, g)):
        prev = a
        for k, x in enumerate([b, c, d, e, last]):
            v = name + k
            A_bin.append((v, [prev, x]))
            prev = v
    assert S.count_mem(A_bin) == gx["A_binary_memory_accesses"]
    assert S.count_mem(named_program(gx["B"]["program"])[0]) == gx["B"]["memory_accesses"]
    assert S.count_mem(named_program(gx["C"]["program"])[0]) == gx["C"]["memory_accesses"]


def test_fusion_strictly_lowers_memory_access_random():
    rng = random.Random(5)
    for _ in range(200):
        nc = 6
        stmts = []
        for v in range(100, 100 + rng.randint(2, 9)):
            pool = list(range(nc)) + [s[0] for s in stmts]
            stmts.append((v, rng.sample(pool, 2)))
        outs = [stmts[-1][0]] + ([stmts[0][0]] if rng.random() < 0.5 else [])
        isc = lambda t: t < 100
        fused = S.fuse(stmts, outs, isc)
        before = S.evaluate(stmts, outs, nc, isc)
        after = S.evaluate(fused, outs, nc, isc)
        assert before == after
        if fused != stmts:
            assert S.count_mem(fused) < S.count_mem(stmts)


# ---- Sec. 6: P_eg, P_reg, Q, Q_DFS, Q_greedy on the abstract LRU cache
G_LRU = golden("lru_pebbling")
LRU_PROGS = {k: [(v, list(ops)) for v, ops in prog] for k, prog in G_LRU["programs"].items()}


@pytest.mark.parametrize("name", sorted(G_LRU["programs"]))
def test_lru_metrics_match_printed(name):
    prog = LRU_PROGS[name]
    assert S.ccap(prog) == G_LRU["ccap"][name]
    assert S.iocost(prog, 8) == G_LRU["iocost_8"][name]
    assert S.nvar(prog) == G_LRU["nvar"][name]


def test_P_eg_iocost_at_capacity_10():
    assert S.iocost(LRU_PROGS["P_eg"], 10) == G_LRU["iocost_10_P_eg"]


def test_dfs_reproduces_Q_DFS():
    # G_eg with the figure's goals; children and roots visited by variable
    isc = lambda t: t >= 1000
    prog, goals, _ = g_eg()
    names = {v: i + 1 for i, (v, _) in enumerate(G_LRU["programs"]["P_eg"])}
    order = S.dfs_order(prog, goals, isc)
    inv = {i: v for v, i in names.items()}
    assert [inv[v] for v, _ in order] == G_LRU["dfs"]["order"]
    peb, ret, npeb = S.assign_pebbles(order, goals, isc)
    assert npeb == G_LRU["dfs"]["pebbles"]
    # the pebbles the DFS schedule assigns are the printed Q_DFS's variables
    assert ["p%d" % (pebble[1] + 1) for pebble, _ in peb] == [v for v, _ in G_LRU["programs"]["Q_DFS"]]


def g_eg():
    """G_eg in integer terms: constants A..G = 1000.., variables v1..v5 = 1..5."""
    cmap = {x: 1000 + i for i, x in enumerate("ABCDEFG")}
    names = {}
    prog = []
    for v, ops in G_LRU["programs"]["P_eg"]:
        names[v] = len(names) + 1
        prog.append((names[v], [cmap[o] if o in cmap else names[o] for o in ops]))
    goals = [names[v] for v in G_LRU["dfs"]["goals"]]
    return prog, goals, {c: x for x, c in cmap.items()}


def test_greedy_reproduces_Q_greedy():
    # Sec. 6.6 worked example: capacity 8, the figure's goals
    prog, goals, cname = g_eg()
    peb, ret, npeb = S.greedy_schedule(prog, goals, lambda t: t >= 1000, 8)
    show = lambda a: cname[a] if isinstance(a, int) else "p%d" % (a[1] + 1)
    got = [[show(p), [show(a) for a in args]] for p, args in peb]
    assert got == G_LRU["programs"]["Q_greedy"]
    assert npeb == G_LRU["nvar"]["Q_greedy"]
    assert S.ccap(peb) == G_LRU["ccap"]["Q_greedy"]
    assert S.iocost(peb, 8) == G_LRU["iocost_8"]["Q_greedy"]
    # the goals v2, v3, v5 end on the pebbles the printed program leaves them on
    assert [show(r) for r in ret] == ["p3", "p2", "p1"]


def random_program(rng, n_const, n_stmt):
    stmts = []
    for v in range(n_stmt):
        pool = list(range(1000, 1000 + n_const)) + list(range(v))
        stmts.append((v, rng.sample(pool, rng.randint(2, min(5, len(pool))))))
    used = {o for _, ops in stmts for o in ops}
    goals = [v for v, _ in stmts if v not in used or rng.random() < 0.2]
    return stmts, goals


@pytest.mark.parametrize("seed", range(12))
def test_greedy_keeps_meaning_and_pebbles(seed):
    rng = random.Random(seed)
    stmts, goals = random_program(rng, 12, 30)
    isc = lambda t: isinstance(t, int) and t >= 1000
    want = S.evaluate(stmts, goals, 0, isc)
    for cap in (4, 8, 64):
        peb, ret, npeb = S.greedy_schedule(stmts, goals, isc, cap)
        assert len(peb) == len(stmts)
        assert S.evaluate(peb, ret, 0, isc) == want
        assert S.nvar(peb) == npeb <= len(stmts)
        # distinct goals end on distinct pebbles
        assert len({r for r in ret if not isc(r)}) == len(set(goals))
    # with room for everything every constant is loaded once and nothing is evicted
    peb, _, _ = S.greedy_schedule(stmts, goals, isc, 10 ** 6)
    loads, ev, re = S.lru_run(peb, 10 ** 6)
    assert ev == 0 and re == 0 and loads == len({o for _, ops in stmts for o in ops if isc(o)})


# ---- Sec. 7.5: printed counts of the paper's RS(10,4) programs
@pytest.fixture(scope="module")
def paper_enc_rows():
    G = oracle.vandermonde_rows(10, 4)
    return S.rows_from_bitmatrix(oracle.bitmatrix(G[10:]))


@pytest.fixture(scope="module")
def paper_dec_rows():
    G = oracle.vandermonde_rows(10, 4)
    D, _ = oracle.decode_matrix(G, 10, 4, [2, 4, 5, 6])
    return S.rows_from_bitmatrix(oracle.bitmatrix(D))


G_RS = golden("rs10_4_paper_counts")


def test_paper_plain_counts_exact(paper_enc_rows, paper_dec_rows):
    ones = sum(r.bit_count() for r in paper_enc_rows)
    assert ones == G_RS["encode"]["ones"] and ones - 32 == G_RS["encode"]["plain_xors"]
    assert sum(r.bit_count() for r in paper_dec_rows) - 32 == G_RS["decode_2_4_5_6"]["plain_xors"]


def within(x, ref, tol):
    return abs(x - ref) <= tol * ref


@pytest.mark.slow
def test_paper_compress_fuse_counts_approx(paper_enc_rows, paper_dec_rows):
    tol = G_RS["tolerance"]
    for rows, ref in ((paper_enc_rows, G_RS["encode"]), (paper_dec_rows, G_RS["decode_2_4_5_6"])):
        comp = S.repair(rows, 80, xor_rebuild=True)
        assert eval_comp(comp) == rows
        # the printed compressed/fused columns depend on tie-breaks the paper
        # does not state: pinned within the fixture's tolerances
        assert within(comp.xor_count(), ref["compressed_xors"], tol["compressed_xors"]), comp.xor_count()
        stmts, outs = comp.to_program()
        fused = S.fuse(stmts, outs, comp.is_const)
        assert within(len(fused), ref["fused_statements"], tol["fused_statements"]), len(fused)
        assert within(S.count_mem(fused), ref["fused_memory_accesses"], tol["fused_memory_accesses"])
        assert S.count_xor(fused) == comp.xor_count()


G_SCHED = golden("rs10_4_schedule_measures")


@pytest.mark.slow
def test_paper_schedule_measures_approx(paper_enc_rows, paper_dec_rows):
    tol = G_SCHED["tolerance"]
    about = G_SCHED["about_every_block_size"]
    for rows, ref, name in ((paper_enc_rows, G_SCHED["dfs"]["encode"], "enc"),
                            (paper_dec_rows, G_SCHED["dfs"]["decode_2_4_5_6"], "dec")):
        comp = S.repair(rows, 80, xor_rebuild=True)
        stmts, outs = comp.to_program()
        fused = S.fuse(stmts, outs, comp.is_const)
        order = S.dfs_order(fused, outs, comp.is_const)
        peb, _, npeb = S.assign_pebbles(order, outs, comp.is_const)
        assert within(npeb, ref["nvar"], tol["dfs_nvar"]), (name, npeb)
        assert within(S.ccap(peb), ref["ccap"], tol["dfs_ccap"]), (name, S.ccap(peb))
        if name != "enc":
            continue
        assert within(npeb, about["nvar"], tol["about_nvar"]) and within(S.ccap(peb), about["ccap"], tol["about_ccap"])
        for b in about["block_bytes"]:
            cap = about["l1_bytes"] // b
            g, ret, gn = S.greedy_schedule(fused, outs, comp.is_const, cap)
            isc = lambda t: isinstance(t, int) and comp.is_const(t)
            assert S.evaluate(g, ret, 80, isc) == S.evaluate(fused, outs, 80, comp.is_const)
            assert within(gn, about["nvar"], tol["about_nvar"]), (b, gn)
            assert within(S.ccap(g), about["ccap"], tol["about_ccap"]), (b, S.ccap(g))


@pytest.mark.parametrize("seed", range(6))
def test_ccap_bisection_equals_the_least_capacity(seed):
    # CCap searched by bisection (LRU inclusion) equals the first capacity
    # found by trying every capacity upward
    rng = random.Random(100 + seed)
    stmts, _ = random_program(rng, 16, 40)
    c = max(len(ops) + 1 for _, ops in stmts)
    while S.lru_run(stmts, c)[2]:
        c += 1
    assert S.ccap(stmts) == c
    assert S.lru_run(stmts, c - 1)[2] > 0 or c == max(len(ops) + 1 for _, ops in stmts)
