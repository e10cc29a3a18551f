"""Pins for the oracle's SLP passes against the paper's worked examples
(Secs. 2, 4, 5, 6), brute force on tiny instances, and the printed operation
counts of the RS(10,4) programs (Sec. 7.5)."""
import itertools
import random

import numpy as np
import pytest

import oracle
from oracle import slp as S

BIG = S.Compressed.BIG
a, b, c, d, e, f, g = range(7)


def bits(*cs):
    return sum(1 << x for x in cs)


def temps_named(comp):
    """Render temporaries with constants as letters, temps as t1, t2..."""
    def nm(t):
        return "abcdefg"[t - BIG] if t >= BIG else "t%d" % (t + 1)
    return [(nm(x), nm(y)) for x, y in comp.temps]


# P0 of Sec. 4.2: v1=a^b, v2=a^b^c, v3=a^b^c^d, v4=b^c^d
P0 = [bits(a, b), bits(a, b, c), bits(a, b, c, d), bits(b, c, d)]


def test_repair_on_P0_matches_worked_example():
    comp = S.repair(P0, 4, xor_rebuild=False)
    assert temps_named(comp) == [("a", "b"), ("t1", "c"), ("t2", "d"), ("b", "c"), ("t4", "d")]
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
    assert temps_named(comp) == [("a", "b"), ("t1", "c"), ("t2", "d"), ("t3", "a")]
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
    assert shortest_xor_count(P0, 4, 4) == 4
    assert shortest_xor_count(P0, 4, 5, disjoint_only=True) == 5


def test_intro_example_compress_and_fuse():
    # Sec. 2: nu1 = a^b, nu2 = c^d^e^f, nu3 = c^d^e^g (7 XORs) -> 5 -> 4 stmts
    rows = [bits(a, b), bits(c, d, e, f), bits(c, d, e, g)]
    comp = S.repair(rows, 7, xor_rebuild=True)
    assert comp.xor_count() == 5
    assert eval_comp(comp) == rows
    stmts, outs = comp.to_program()
    fused = S.fuse(stmts, outs, comp.is_const)
    assert len(fused) == 4 and S.count_mem(fused) == 13 and S.count_xor(fused) == 5


def test_fusion_worked_example():
    # Sec. 5.2: v1=a^b; v2=v1^c; v3=v2^d; return v3  ->  v3 = xor(a,b,c,d)
    isc = lambda t: t < 100
    prog = [(101, [a, b]), (102, [101, c]), (103, [102, d])]
    fused = S.fuse(prog, [103], isc)
    assert fused == [(103, [a, b, c, d])]


def test_memory_access_counts_A_B_C():
    # Sec. 5.2 A/B/C: #M = 30 (binary A), 12 (compressed B), 14 (fused C)
    A_bin = []
    for name, last in ((200, f), (300, g)):
        prev = a
        for k, x in enumerate([b, c, d, e, last]):
            v = name + k
            A_bin.append((v, [prev, x]))
            prev = v
    assert S.count_mem(A_bin) == 30
    B = [(1, [a, b, c, d, e]), (2, [1, f]), (3, [1, g])]
    assert S.count_mem(B) == 12
    C = [(2, [a, b, c, d, e, f]), (3, [a, b, c, d, e, g])]
    assert S.count_mem(C) == 14


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
A_, B_, C_, D_, E_, F_, G_ = "ABCDEFG"
P_eg = [("v1", [A_, B_]), ("v2", [C_, D_]), ("v3", ["v1", E_, F_]), ("v4", ["v3", G_, A_]),
        ("v5", ["v1", "v3", "v4"])]
P_reg = P_eg[:4] + [("v1", ["v1", "v3", "v4"])]
Q = [("p1", [B_, A_]), ("p2", [E_, F_, "p1"]), ("p3", [A_, G_, "p2"]), ("p1", ["p1", "p2", "p3"]),
     ("p3", [C_, D_])]
Q_DFS = [("p1", [C_, D_]), ("p2", [A_, B_]), ("p3", ["p2", E_, F_]), ("p4", ["p3", A_, G_]),
         ("p4", ["p2", "p3", "p4"])]
Q_greedy = [("p1", [A_, B_]), ("p2", ["p1", E_, F_]), ("p3", ["p2", A_, G_]), ("p1", ["p1", "p2", "p3"]),
            ("p3", [C_, D_])]


@pytest.mark.parametrize("prog,cc,io8,nv", [
    (P_eg, 10, 13, 5), (P_reg, 10, 12, 4), (Q, 5, 9, 3), (Q_DFS, 7, 10, 4), (Q_greedy, 7, 9, 3)])
def test_lru_metrics_match_printed(prog, cc, io8, nv):
    assert S.ccap(prog) == cc
    assert S.iocost(prog, 8) == io8
    assert S.nvar(prog) == nv


def test_P_eg_iocost_at_capacity_10():
    assert S.iocost(P_eg, 10) == 9


def test_dfs_reproduces_Q_DFS():
    # G_eg with goals {v2, v3, v5} (the figure's double circles)
    cmap = {x: i for i, x in enumerate("ABCDEFG")}
    isc = lambda t: t >= 1000
    prog = [(1, [1000 + cmap["A"], 1000 + cmap["B"]]), (2, [1000 + cmap["C"], 1000 + cmap["D"]]),
            (3, [1, 1000 + cmap["E"], 1000 + cmap["F"]]), (4, [3, 1000 + cmap["G"], 1000 + cmap["A"]]),
            (5, [1, 3, 4])]
    order = S.dfs_order(prog, [2, 3, 5], isc)
    assert [v for v, _ in order] == [2, 1, 3, 4, 5]
    peb, ret, npeb = S.assign_pebbles(order, [2, 3, 5], isc)
    assert npeb == 4
    assert [p for p, _ in peb] == [("p", 0), ("p", 1), ("p", 2), ("p", 3), ("p", 3)]
    assert ret == [("p", 0), ("p", 2), ("p", 3)]


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


def test_paper_plain_counts_exact(paper_enc_rows, paper_dec_rows):
    ones = sum(r.bit_count() for r in paper_enc_rows)
    assert ones == 787 and ones - 32 == 755
    assert sum(r.bit_count() for r in paper_dec_rows) - 32 == 1368


def within(x, ref, tol=0.04):
    return abs(x - ref) <= tol * ref


@pytest.mark.slow
def test_paper_compress_fuse_counts_approx(paper_enc_rows, paper_dec_rows):
    for rows, co, fu_stmt, fu_mem in ((paper_enc_rows, 385, 146, 677), (paper_dec_rows, 511, 206, 923)):
        comp = S.repair(rows, 80, xor_rebuild=True)
        assert eval_comp(comp) == rows
        # the printed compressed/fused columns depend on tie-breaks the paper
        # does not state: XOR count and #M within 3%, statements within 5%
        assert within(comp.xor_count(), co, 0.03), comp.xor_count()
        stmts, outs = comp.to_program()
        fused = S.fuse(stmts, outs, comp.is_const)
        assert within(len(fused), fu_stmt, 0.05), len(fused)
        assert within(S.count_mem(fused), fu_mem, 0.03), S.count_mem(fused)
        assert S.count_xor(fused) == comp.xor_count()
