"""The whole-output fingerprint check (tests/strip_check.py) on the CPU: it
accepts the oracle's own outputs and rejects planted mistakes in them (one
flipped bit, one skipped tile, two swapped outputs, a wrong survivor)."""
import numpy as np
import pytest

import oracle
import strip_check as SC
from paper_2108_02692_amd import workloads as W


def _case(n, p, S, seed, er=()):
    G = oracle.cauchy(n, p)
    data = W.host_blocks(n, S, seed=seed)
    blocks = data + oracle.encode(G, n, p, data)
    if not er:
        return G, list(range(n)), data, blocks[n:]
    R = oracle.survivors(n, p, er)
    return G, R, [blocks[i] for i in R], oracle.decode(G, n, p, list(er), blocks)


@pytest.mark.parametrize("n,p,er", [(10, 4, ()), (10, 4, (2, 4, 5, 6)), (6, 3, (0, 7)), (14, 4, (13,))])
def test_accepts_oracle_outputs(n, p, er):
    S = 8 * 1024 + 512
    M = SC.masks(S // 64)
    G, R, ins, outs = _case(n, p, S, n + p, er)
    mat = SC.stripe_matrix(G, n, p, er, R)
    assert SC.check_stripe(mat, ins, outs, M) == []


def test_rejects_planted_mistakes():
    n, p, S = 10, 4, 16 * 1024
    M = SC.masks(S // 64)
    G, R, ins, outs = _case(n, p, S, 3)
    mat = SC.stripe_matrix(G, n, p, (), R)
    bad = [o.copy() for o in outs]
    bad[2][5 * (S // 8) + 777] ^= 0x10                       # one bit of strip (2, 5)
    assert SC.check_stripe(mat, ins, bad, M) == [(2, 5)]
    bad = [o.copy() for o in outs]
    bad[1][3 * (S // 8) + 1024: 3 * (S // 8) + 2048] = 0xA5  # a tile of strip (1, 3) never written
    assert SC.check_stripe(mat, ins, bad, M) == [(1, 3)]
    assert len(SC.check_stripe(mat, ins, [outs[1], outs[0]] + outs[2:], M)) == 16
    G, R, ins, outs = _case(n, p, S, 4, (2, 4, 5, 6))
    with pytest.raises(AssertionError):                      # survivors in another order
        SC.stripe_matrix(G, n, p, (2, 4, 5, 6), R[::-1])
