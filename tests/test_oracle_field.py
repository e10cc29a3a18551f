"""Pins for the oracle's field, generator, bitmatrix and RS coder.

Each check compares the oracle with something other than itself: brute-force
field axioms, an independent carry-less multiply, the MDS property, the
bitmatrix identity of Sec. 1 (ii), closed-form layout cases, and the decode
round trip over every erasure set."""
import itertools

import numpy as np
import pytest

import oracle


def clmul_mod(a, b, poly=0x11D):
    """Textbook shift-and-add multiply in GF(2)[x] / (x^8+x^4+x^3+x^2+1)."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a & 0x100:
            a ^= poly
    return r


@pytest.fixture(scope="module")
def T():
    return oracle.gf_mul_table().astype(np.int64)


def test_alpha_is_primitive():
    seen = {oracle.gf_exp(i) for i in range(255)}
    assert seen == set(range(1, 256))
    assert oracle.gf_exp(0) == 1 and oracle.gf_exp(1) == 2 and oracle.gf_exp(8) == 0x1D


def test_mul_matches_shift_and_add(T):
    ref = np.array([[clmul_mod(a, b) for b in range(256)] for a in range(256)])
    assert np.array_equal(T, ref)


def test_field_axioms_bruteforce(T):
    a = np.arange(256)
    assert np.array_equal(T, T.T)  # commutative
    assert np.all(T[1] == a) and np.all(T[0] == 0)
    # associativity and distributivity over all 256^3 triples
    for x in range(256):
        lhs = T[T[x][:, None], a[None, :]]  # (x*y)*z
        rhs = T[x][T]  # x*(y*z)
        assert np.array_equal(lhs, rhs)
        dl = T[x][a[:, None] ^ a[None, :]]  # x*(y+z)
        dr = T[x][:, None] ^ T[x][None, :]
        assert np.array_equal(dl, dr)


def test_inverse():
    for a in range(1, 256):
        assert oracle.gf_mul(a, oracle.gf_inv(a)) == 1


def gf_matmul(T, A, B):
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    out = np.zeros((A.shape[0], B.shape[1]), dtype=np.int64)
    for k in range(A.shape[1]):
        out ^= T[A[:, k][:, None], B[k, :][None, :]]
    return out


@pytest.mark.parametrize("n,p", [(10, 4), (6, 3), (12, 4), (14, 4)])
def test_cauchy_entries_and_mds(T, n, p):
    G = oracle.cauchy(n, p)
    assert np.array_equal(G[:n], np.eye(n, dtype=np.uint8))
    for i in range(p):
        for j in range(n):
            assert oracle.gf_mul(int(G[n + i, j]), i ^ (p + j)) == 1
    # every n x n submatrix of [I; P] is invertible, and the inverse is one
    for rows in itertools.combinations(range(n + p), n):
        M = G[list(rows)]
        Mi = oracle.invert(M)
        assert Mi is not None, rows
        assert np.array_equal(gf_matmul(T, M, Mi), np.eye(n, dtype=np.int64))


def test_invert_detects_singular():
    M = np.array([[1, 2], [2, 4]], dtype=np.uint8)  # row 2 = 2 * row 1
    assert oracle.invert(M) is None


def test_bitmatrix_identity_all_pairs(T):
    # property (ii) of Sec. 1: x*y = B^-1(x~ . B(y)) for all 256 x 256 pairs
    for e in range(256):
        B = oracle.bitmatrix(np.array([[e]], dtype=np.uint8)).astype(np.int64)
        ys = np.arange(256)
        ybits = (ys[None, :] >> np.arange(8)[:, None]) & 1  # 8 x 256
        prod = (B @ ybits) & 1
        val = (prod << np.arange(8)[:, None]).sum(axis=0)
        assert np.array_equal(val, T[e, ys]), e


def rand_blocks(rng, k, S):
    return [rng.integers(0, 256, S, dtype=np.uint8) for _ in range(k)]


def test_all_ones_row_is_bytewise_xor():
    rng = np.random.default_rng(1)
    d = rand_blocks(rng, 7, 256)
    (out,) = oracle.apply(np.ones((1, 7), dtype=np.uint8), d)
    ref = np.bitwise_xor.reduce(np.stack(d), axis=0)
    assert np.array_equal(out, ref)


def test_identity_matrix_copies():
    rng = np.random.default_rng(2)
    d = rand_blocks(rng, 5, 128)
    out = oracle.apply(np.eye(5, dtype=np.uint8), d)
    for a, b in zip(out, d):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,p", [(10, 4), (6, 3)])
def test_single_strip_closed_form(n, p):
    """Block i with strip c all 0xFF, everything else 0: every symbol of block
    i is x^c, so parity strip (j, r) is 0xFF iff bit r of P[j][i]*x^c is set."""
    G = oracle.cauchy(n, p)
    S = 64
    L = S // 8
    for i in (0, n - 1):
        for c in (0, 3, 7):
            d = [np.zeros(S, dtype=np.uint8) for _ in range(n)]
            d[i][c * L:(c + 1) * L] = 0xFF
            par = oracle.encode(G, n, p, d)
            for j in range(p):
                y = oracle.gf_mul(int(G[n + j, i]), 1 << c)
                for r in range(8):
                    want = 0xFF if (y >> r) & 1 else 0
                    assert np.all(par[j][r * L:(r + 1) * L] == want)


def test_encode_is_linear():
    G = oracle.cauchy(10, 4)
    rng = np.random.default_rng(3)
    a = rand_blocks(rng, 10, 512)
    b = rand_blocks(rng, 10, 512)
    pa = oracle.encode(G, 10, 4, a)
    pb = oracle.encode(G, 10, 4, b)
    pab = oracle.encode(G, 10, 4, [x ^ y for x, y in zip(a, b)])
    for u, v, w in zip(pa, pb, pab):
        assert np.array_equal(u ^ v, w)


def all_erasure_sets(n, p):
    for k in range(1, p + 1):
        yield from itertools.combinations(range(n + p), k)


@pytest.mark.parametrize("n,p", [(10, 4), (6, 3), (12, 4)])
def test_decode_round_trip_every_pattern(n, p):
    G = oracle.cauchy(n, p)
    rng = np.random.default_rng(n * 100 + p)
    S = 64
    data = rand_blocks(rng, n, S)
    blocks = data + oracle.encode(G, n, p, data)
    count = 0
    for er in all_erasure_sets(n, p):
        view = [None if i in er else b for i, b in enumerate(blocks)]
        rec = oracle.decode(G, n, p, list(er), view)
        for e, r in zip(er, rec):
            assert np.array_equal(r, blocks[e]), (er, e)
        count += 1
    from math import comb
    assert count == sum(comb(n + p, k) for k in range(1, p + 1))


def test_decode_errors():
    G = oracle.cauchy(10, 4)
    with pytest.raises(ValueError):
        oracle.decode_matrix(G, 10, 4, [0, 1, 2, 3, 4])
    with pytest.raises(ValueError):
        oracle.decode_matrix(G, 10, 4, [14])
    bad = G.copy()
    bad[10] = bad[11]  # two equal parity rows: survivors {..,10,11} singular
    with pytest.raises(ZeroDivisionError):
        oracle.decode_matrix(bad, 10, 4, list(range(8)[:4]))


def test_survivors_prefer_lowest_index():
    assert oracle.survivors(10, 4, [3, 12]) == [0, 1, 2, 4, 5, 6, 7, 8, 9, 10]
