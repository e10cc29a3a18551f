"""Whole-output check of coded stripes at any size, from the oracle's bitmatrix.

Sec. 1 of the paper: multiplying by a GF(2^8) matrix equals multiplying the
bit vectors of the symbols by its bitmatrix.  With the strip layout (strip c
of a block holds bit c of every symbol, the same bit position b in each byte),
this says that every output strip (j, r) is the bytewise XOR of the input
strips (i, c) whose bitmatrix entry B[8j+r][8i+c] is 1, at every byte
offset.  That relation is GF(2)-linear, so it survives any linear
fingerprint applied to all strips alike: here F(s) = XOR over 64-bit words w
of (M[w] AND s[w]) for random masks M.  Checking F(out(j, r)) against the XOR
of F over the row's input strips covers every byte of every output at the
cost of one pass over the data.  A wrong word with d differing bits escapes
one mask with probability 2^-d; two independent masks are used.

The bitmatrix and the coding matrices come from the oracle (whose bitmatrix is
pinned against the field multiplication on all 256 x 256 pairs); nothing here
comes from the library under test.
"""
from __future__ import annotations

import numpy as np

import oracle

N_MASKS = 2


def masks(max_words: int, seed: int = 99) -> np.ndarray:
    """(N_MASKS, max_words) random 64-bit masks."""
    return np.random.default_rng(seed).integers(0, 1 << 64, (N_MASKS, max_words), dtype=np.uint64)


def strip_fingerprints(block: np.ndarray, M: np.ndarray) -> np.ndarray:
    """(8, N_MASKS) uint64 fingerprints of the 8 strips of one block (uint8
    array of S bytes, S a multiple of 64 so that a strip is whole words)."""
    S = block.size
    assert S % 64 == 0, S
    words = block.view(np.uint64).reshape(8, S // 64)
    nw = words.shape[1]
    out = np.empty((8, M.shape[0]), dtype=np.uint64)
    for m in range(M.shape[0]):
        out[:, m] = np.bitwise_xor.reduce(words & M[m, :nw], axis=1)
    return out


def expected_from_inputs(mat: np.ndarray, fin: np.ndarray) -> np.ndarray:
    """Fingerprints the outputs of ``mat`` (rows x cols over GF(2^8)) must
    have, given the (8 cols, N_MASKS) fingerprints of the input strips: each
    output strip's is the XOR of its bitmatrix row's input strips'."""
    B = oracle.bitmatrix(mat).astype(np.int64)             # (8 rows, 8 cols)
    bits = np.unpackbits(fin.view(np.uint8), axis=1)        # (8 cols, 64 N_MASKS)
    want_bits = (B @ bits.astype(np.int64)) & 1             # parity of the selected rows
    return np.packbits(want_bits.astype(np.uint8), axis=1).view(np.uint64)


def stripe_matrix(gen: np.ndarray, n: int, p: int, erased, in_blocks) -> np.ndarray:
    """The matrix from the stripe's inputs (block indices ``in_blocks``, in
    argument order) to its outputs: the parity rows for an encode, the
    oracle's decode rows for an erasure set (whose survivors must be the
    same blocks in the same order)."""
    gen = np.asarray(gen, dtype=np.uint8)
    if not erased:
        assert list(in_blocks) == list(range(n))
        return gen[n:]
    D, R = oracle.decode_matrix(gen, n, p, list(erased))
    assert list(R) == list(in_blocks), (R, in_blocks)
    return D


def check_stripe(mat: np.ndarray, ins, outs, M: np.ndarray) -> list:
    """Output indices (j, r) whose strip fingerprint disagrees."""
    fin = np.concatenate([strip_fingerprints(b, M) for b in ins])
    fout = np.concatenate([strip_fingerprints(b, M) for b in outs])
    want = expected_from_inputs(mat, fin)
    bad = np.nonzero(np.any(fout != want, axis=1))[0]
    return [(int(r) // 8, int(r) % 8) for r in bad]
