"""The paper's average reduction ratios over the 1002 RS(10,4) programs
(Sec. 7.3), recomputed with the library's implementation of the paper's
whole-matrix passes (checked statement by statement against the oracle in
test_compiler.py) and pinned to the printed averages."""
import itertools
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rs10_4_average_ratios.json")


def programs():
    """(rows matrix k x 10) of the encoding program and of every decoding
    program that loses at least one data block."""
    n, p = 10, 4
    G = oracle.vandermonde_rows(n, p)
    out = [G[n:]]
    for er in itertools.combinations(range(n + p), p):
        lost = [e for e in er if e < n]
        if not lost:
            continue
        D, surv = oracle.decode_matrix(G, n, p, list(er))
        rows = [D[k] for k, e in enumerate(er) if e < n]
        out.append(np.array(rows, dtype=np.uint8))
    return out


def stage_counts(rows, compress):
    """#xor of the plain and compressed programs and #M of the fused ones."""
    n, k = 10, len(rows)
    gen = np.vstack([np.eye(n, dtype=np.uint8), rows]).tolist()
    prog = E.ec_compile_slp(n, k, gen, level=E.LEVEL_CO_FU, compress=compress)
    xp = prog.info["plain_xor2"]
    co, _ = prog.export(E.STAGE_CO)
    xco = sum(len(ops) - 1 for _, ops in co)
    fu, _ = prog.export(E.STAGE_FU)
    mfu = sum(len(ops) + 1 for _, ops in fu)
    plain, _ = prog.export(E.STAGE_PLAIN)
    mfu_plain = sum(len(ops) + 1 for _, ops in plain)  # fusing binary P gives one statement per row
    return xp, xco, mfu, mfu_plain


@pytest.mark.slow
def test_average_reduction_ratios_match_printed():
    ref = json.load(open(GOLDEN))
    progs = programs()
    assert len(progs) == 1 + 1001 - 1
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        xr = list(ex.map(lambda r: stage_counts(r, E.COMPRESS_XORREPAIR), progs))
        rp = list(ex.map(lambda r: stage_counts(r, E.COMPRESS_REPAIR), progs))
    tol = ref["tolerance_points"]
    xor_xr = np.mean([c / p for p, c, _, _ in xr])
    xor_rp = np.mean([c / p for p, c, _, _ in rp])
    assert abs(xor_xr - ref["xor_ratio"]["xorrepair"]) <= tol, xor_xr
    assert abs(xor_rp - ref["xor_ratio"]["repair"]) <= tol, xor_rp
    co_p = np.mean([c / p for p, c, _, _ in xr])              # binary: #M = 3 #xor on both sides
    fu_p = np.mean([mp / (3 * p) for p, _, _, mp in xr])
    fuco_co = np.mean([m / (3 * c) for _, c, m, _ in xr])
    fuco_p = np.mean([m / (3 * p) for p, _, m, _ in xr])
    got = {"co_over_p": co_p, "fu_over_p": fu_p, "fuco_over_co": fuco_co, "fuco_over_p": fuco_p}
    for k, v in got.items():
        assert abs(v - ref["mem_ratio"][k]) <= tol, (k, v, ref["mem_ratio"][k])


# ---- Sec. 7.5 figure: measures of the optimised programs for RS(d,p)
FIG = json.load(open(os.path.join(os.path.dirname(GOLDEN), "rs_codecs_paper_figure.json")))


def _within(x, ref, band):
    return ref * (1 + band[0]) <= x <= ref * (1 + band[1])


@pytest.mark.slow
@pytest.mark.parametrize("codec", sorted(FIG["codecs"]))
def test_codec_figure_measures(codec):
    """The oracle's pipeline (XorRePair, fusion, DFS and its pebbles, the LRU
    CCap) on the paper's matrix for each codec of the figure, pinned to the
    printed values within the fixture's bands; the library's whole-matrix
    stages for the same programs equal the oracle's statement for
    statement."""
    from oracle import slp as S
    d, p = map(int, codec.split(","))
    ref = dict(zip(FIG["columns"], FIG["codecs"][codec]))
    tol = FIG["tolerance"]
    G = oracle.vandermonde_rows(d, p)
    er = [2, 4, 5, 6][:p]
    D, _ = oracle.decode_matrix(G, d, p, er)
    gen = G.tolist()
    big = S.Compressed.BIG
    term = lambda x: S.ZERO if x == -1 else (big + (-x - 2) if x <= -2 else x)
    for tag, mat, erased in (("enc", G[d:], ()), ("dec", D, er)):
        rows = S.rows_from_bitmatrix(oracle.bitmatrix(mat))
        comp = S.repair(rows, 8 * d, xor_rebuild=True)
        st, outs = comp.to_program()
        fu = S.fuse(st, outs, comp.is_const)
        order = S.dfs_order(fu, outs, comp.is_const)
        peb, _, npeb = S.assign_pebbles(order, outs, comp.is_const)
        got = {"stmt": len(fu), "mem": S.count_mem(fu), "nvar": npeb, "ccap": S.ccap(peb)}
        for k, v in got.items():
            assert _within(v, ref["%s_%s" % (k, tag)], tol[k]), (codec, tag, k, v, ref["%s_%s" % (k, tag)])
        prog = E.ec_compile_slp(d, p, gen, list(erased))
        pfu, pouts = prog.export(E.STAGE_FU)
        assert [(v, [term(o) for o in ops]) for v, ops in pfu] == fu and [term(o) for o in pouts] == outs
        psched, _ = prog.export(E.STAGE_SCHED)
        assert [(v, [term(o) for o in ops]) for v, ops in psched] == order


# ---- Sec. 7.3: average NVar and CCap ratios
def _nvar_ccap(rows):
    """NVar and CCap of P, Co(P), Fu(P), Fu(Co(P)) and Dfs(Fu(Co(P))) for one
    program: the stages are the library's (equal to the oracle's, see
    test_compiler.py), the measures the oracle's LRU model."""
    from oracle import slp as S
    big = S.Compressed.BIG
    term = lambda x: S.ZERO if x == -1 else (big + (-x - 2) if x <= -2 else x)
    conv = lambda st: [(v, [term(o) for o in ops]) for v, ops in st]
    isc = lambda t: isinstance(t, int) and t >= big
    n, k = 10, len(rows)
    gen = np.vstack([np.eye(n, dtype=np.uint8), rows]).tolist()
    prog = E.ec_compile_slp(n, k, gen)
    plain = conv(prog.export(E.STAGE_PLAIN)[0])
    chain = []  # P: each row accumulated in its own variable by binary XORs
    for v, ops in plain:
        chain.append((v, ops[:2]))
        chain += [(v, [v, o]) for o in ops[2:]]
    co = conv(prog.export(E.STAGE_CO)[0])
    fu, fouts = prog.export(E.STAGE_FU)
    fu = conv(fu)
    fouts = [term(o) for o in fouts]
    peb, _, npeb = S.assign_pebbles(conv(prog.export(E.STAGE_SCHED)[0]), fouts, isc)
    nv_p, nv_co = S.nvar(chain), S.nvar(co)
    cc_p, cc_co = S.ccap(chain), S.ccap(co)
    return (nv_co / nv_p, S.nvar(plain) / nv_p, S.nvar(fu) / nv_co, npeb / nv_co,
            cc_co / cc_p, S.ccap(plain) / cc_p, S.ccap(fu) / cc_co, S.ccap(peb) / cc_co)


@pytest.mark.slow
def test_average_nvar_ccap_ratios_match_printed():
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    ref = json.load(open(GOLDEN))
    progs = programs()
    workers = max(1, min(8, os.cpu_count() or 1))
    with ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("fork")) as ex:
        res = np.array(list(ex.map(_nvar_ccap, progs, chunksize=8)))
    avg = res.mean(axis=0)
    keys = ("co_over_p", "fu_over_p", "fuco_over_co", "dfs_over_co")
    tol = ref["tolerance_rel_nvar_ccap"]
    for i, k in enumerate(keys):
        for table, got in (("nvar_ratio", avg[i]), ("ccap_ratio", avg[4 + i])):
            want = ref[table][k]
            assert abs(got - want) <= tol * want, (table, k, got, want)
