"""CPU oracle for the XOR-SLP erasure-coding path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it, and it imports nothing from the product.

Two parts:

* ``rs_oracle.c`` (wrapped here through ctypes): the plain definition of RS
  coding over GF(2^8)/0x11D with log/antilog tables, Cauchy and
  Vandermonde-row generators, Gauss-Jordan inversion and the bitmatrix map.
* ``oracle.slp``: the paper's program transformations (pairing compression,
  XOR fusion, DFS scheduling, the abstract LRU cache) written from Secs. 4-6,
  in pure Python on small programs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile rs_oracle.c into _liboracle.so with gcc (plain -O2)."""
    stale = (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            ip = ctypes.POINTER(ctypes.c_int)
            pp = ctypes.POINTER(ctypes.c_void_p)
            L.oracle_gf_mul.restype = ctypes.c_uint8
            L.oracle_gf_mul.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
            L.oracle_gf_inv.restype = ctypes.c_uint8
            L.oracle_gf_inv.argtypes = [ctypes.c_uint8]
            L.oracle_gf_exp.argtypes = [ctypes.c_int]
            L.oracle_gf_log.argtypes = [ctypes.c_int]
            L.oracle_cauchy.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
            L.oracle_vandermonde_rows.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
            L.oracle_invert.argtypes = [ctypes.c_int, u8p, u8p]
            L.oracle_bitmatrix.restype = None
            L.oracle_bitmatrix.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
            L.oracle_apply.argtypes = [ctypes.c_int, ctypes.c_int, u8p, pp, pp, ctypes.c_size_t]
            L.oracle_apply_range.argtypes = [ctypes.c_int, ctypes.c_int, u8p, pp, pp, ctypes.c_size_t,
                                             ctypes.c_size_t, ctypes.c_size_t]
            L.oracle_encode.argtypes = [ctypes.c_int, ctypes.c_int, u8p, pp, pp, ctypes.c_size_t]
            L.oracle_decode_matrix.argtypes = [ctypes.c_int, ctypes.c_int, u8p, ip, ctypes.c_int, u8p, ip]
            L.oracle_decode.argtypes = [ctypes.c_int, ctypes.c_int, u8p, ip, ctypes.c_int, pp, pp, ctypes.c_size_t]
            _lib = L
    return _lib


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _ptrs(blocks):
    arr = (ctypes.c_void_p * max(1, len(blocks)))()
    for i, b in enumerate(blocks):
        if b is None:
            arr[i] = None
        else:
            assert b.dtype == np.uint8 and b.flags.c_contiguous
            arr[i] = b.ctypes.data
    return arr


# ---------------------------------------------------------------- field
def gf_mul(a: int, b: int) -> int:
    return int(lib().oracle_gf_mul(a, b))


def gf_inv(a: int) -> int:
    return int(lib().oracle_gf_inv(a))


def gf_exp(i: int) -> int:
    return int(lib().oracle_gf_exp(i))


def gf_log(a: int) -> int:
    return int(lib().oracle_gf_log(a))


def gf_mul_table() -> np.ndarray:
    """256 x 256 product table built from the oracle's multiply."""
    t = np.zeros((256, 256), dtype=np.uint8)
    L = lib()
    for a in range(256):
        for b in range(256):
            t[a, b] = L.oracle_gf_mul(a, b)
    return t


# ---------------------------------------------------------------- matrices
def cauchy(n: int, p: int) -> np.ndarray:
    g = np.zeros((n + p, n), dtype=np.uint8)
    if lib().oracle_cauchy(n, p, _u8(g)) != 0:
        raise ValueError("bad codec")
    return g


def vandermonde_rows(n: int, p: int) -> np.ndarray:
    g = np.zeros((n + p, n), dtype=np.uint8)
    if lib().oracle_vandermonde_rows(n, p, _u8(g)) != 0:
        raise ValueError("bad codec")
    return g


def invert(m: np.ndarray):
    m = np.ascontiguousarray(m, dtype=np.uint8)
    n = m.shape[0]
    out = np.zeros_like(m)
    rc = lib().oracle_invert(n, _u8(m), _u8(out))
    return None if rc != 0 else out


def bitmatrix(mat: np.ndarray) -> np.ndarray:
    mat = np.ascontiguousarray(mat, dtype=np.uint8)
    r, c = mat.shape
    bits = np.zeros((8 * r, 8 * c), dtype=np.uint8)
    lib().oracle_bitmatrix(r, c, _u8(mat), _u8(bits))
    return bits


def survivors(n: int, p: int, erased) -> list:
    gone = set(int(e) for e in erased)
    return [b for b in range(n + p) if b not in gone][:n]


def decode_matrix(gen: np.ndarray, n: int, p: int, erased):
    """Rows G[e,:] . M^-1 for each erased e (in the given order) and the
    survivor indices; raises on singular / too many erasures."""
    gen = np.ascontiguousarray(gen, dtype=np.uint8)
    er = (ctypes.c_int * max(1, len(erased)))(*[int(e) for e in erased])
    out = np.zeros((max(1, len(erased)), n), dtype=np.uint8)
    rows = (ctypes.c_int * n)()
    rc = lib().oracle_decode_matrix(n, p, _u8(gen), er, len(erased), _u8(out), rows)
    if rc == -1:
        raise ZeroDivisionError("singular survivor matrix")
    if rc != 0:
        raise ValueError("bad erasure set (rc=%d)" % rc)
    return out[: len(erased)], list(rows)


# ---------------------------------------------------------------- coding
def _run_ranges(rows, cols, mat, ins, outs, S, threads):
    """oracle_apply_range over [0, S/8) cut into ``threads`` contiguous,
    disjoint offset ranges, each on its own host thread (the C call releases
    the interpreter lock; every range writes only its own bytes)."""
    L = S // 8
    mat = np.ascontiguousarray(mat, dtype=np.uint8)
    pin, pout = _ptrs(ins), _ptrs(outs)
    T = max(1, min(int(threads), L))
    cuts = [L * t // T for t in range(T + 1)]

    def one(t):
        return lib().oracle_apply_range(rows, cols, _u8(mat), pin, pout, S, cuts[t], cuts[t + 1])

    if T == 1:
        rcs = [one(0)]
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=T) as ex:
            rcs = list(ex.map(one, range(T)))
    bad = [rc for rc in rcs if rc != 0]
    if bad:
        raise ValueError("oracle_apply_range rc=%d" % bad[0])


def apply(mat: np.ndarray, blocks, threads: int = 1) -> list:
    mat = np.ascontiguousarray(mat, dtype=np.uint8)
    rows, cols = mat.shape
    assert len(blocks) == cols
    S = blocks[0].size
    outs = [np.zeros(S, dtype=np.uint8) for _ in range(rows)]
    _run_ranges(rows, cols, mat, blocks, outs, S, threads)
    return outs


def encode(gen: np.ndarray, n: int, p: int, data, threads: int = 1) -> list:
    """Parity blocks for the n data blocks (each a uint8 array of S bytes);
    ``threads`` > 1 splits the strip offsets over that many host threads."""
    gen = np.ascontiguousarray(gen, dtype=np.uint8)
    assert len(data) == n
    S = data[0].size
    par = [np.zeros(S, dtype=np.uint8) for _ in range(p)]
    if threads > 1:
        if p:
            _run_ranges(p, n, gen[n:], data, par, S, threads)
        return par
    rc = lib().oracle_encode(n, p, _u8(gen), _ptrs(data), _ptrs(par), S)
    if rc != 0:
        raise ValueError("oracle_encode rc=%d" % rc)
    return par


def decode(gen: np.ndarray, n: int, p: int, erased, blocks, threads: int = 1) -> list:
    """Reconstruct every erased block.  ``blocks`` has n+p entries; erased
    entries are ignored (may be None).  ``threads`` as in ``encode``."""
    gen = np.ascontiguousarray(gen, dtype=np.uint8)
    S = next(b.size for i, b in enumerate(blocks) if i not in set(erased) and b is not None)
    if threads > 1:
        D, R = decode_matrix(gen, n, p, erased)
        outs = [np.zeros(S, dtype=np.uint8) for _ in erased]
        if len(erased):
            _run_ranges(len(erased), n, D, [blocks[r] for r in R], outs, S, threads)
        return outs
    er = (ctypes.c_int * max(1, len(erased)))(*[int(e) for e in erased])
    outs = [np.zeros(S, dtype=np.uint8) for _ in erased]
    rc = lib().oracle_decode(n, p, _u8(gen), er, len(erased), _ptrs(blocks), _ptrs(outs), S)
    if rc != 0:
        raise ValueError("oracle_decode rc=%d" % rc)
    return outs
