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
