"""Native kernels on the host: the generated straight-line code is the
program's records, instruction for instruction.

The generated asm is parsed and run symbolically (each register holds the
set of input strips XORed into it, as a Python int), independently of the
library: every output strip must be stored once with the value of its
bitmatrix row (from the oracle), every slot must end at zero (the next tile
starts from zero), and the memory operations must come in the records'
order with the records' waits (which the record simulator checks).  The
kernels are compiled with hiprtc here (no GPU needed)."""
import re

import pytest

import paper_2108_02692_amd as E
from bytecode_sim import KINDS, fields
from test_compiler import oracle_rows

ASM = re.compile(r'^\s*"(.*)\\n\\t"$')


def asm_bodies(src):
    """The instructions of each per-tile asm statement (one per part)."""
    lines = src.splitlines()
    out = []
    for i, ln in enumerate(lines):
        if ln.strip() != "asm volatile(":
            continue
        body = []
        for ln2 in lines[i + 1:]:
            m = ASM.match(ln2)
            if not m:
                break
            body.append(m.group(1))
        out.append(body)
    return out


def asm_body(src):
    bodies = asm_bodies(src)
    assert len(bodies) == 1
    return bodies[0]


def run_symbolic(body, n_in, tiles=2):
    """{(block, strip): value} stored per tile (the same every tile), the
    registers after the last tile, and the memory events in order."""
    reg = {}
    first = None
    events = []
    for t in range(tiles):
        stores = {}
        for ins in body:
            op, _, rest = ins.partition(" ")
            args = [a.strip() for a in rest.split(",")]
            if op == "v_mov_b32":
                reg[int(args[0][1:])] = reg.get(int(args[1][1:]), 0)
            elif op == "v_xor_b32":
                d, a, b = (int(x[1:]) for x in args)
                assert d == a
                reg[d] = reg.get(a, 0) ^ reg.get(b, 0)
            elif op == "global_load_dwordx4":
                lo, hi = map(int, re.match(r"v\[(\d+):(\d+)\]", args[0]).groups())
                j = int(re.match(r"%\[o(\d)\]", args[1]).group(1))
                b, pol = re.match(r"%\[b(\d+)\] (\w+)", args[2]).groups()
                assert pol == "nt" and int(b) < n_in and hi == lo + 3
                for r in range(lo, hi + 1):
                    reg[r] = 1 << (8 * int(b) + j)
                if t == 0:
                    events.append(("load", int(b), j))
            elif op == "global_store_dwordx4":
                j = int(re.match(r"%\[o(\d)\]", args[0]).group(1))
                assert args[1] == "v[0:3]"
                b, pol = re.match(r"%\[b(\d+)\] (\w+)", args[2]).groups()
                assert pol == "nt" and int(b) >= n_in
                assert reg.get(0, 0) == reg.get(1, 0) == reg.get(2, 0) == reg.get(3, 0)
                key = (int(b) - n_in, j)
                assert key not in stores, "strip stored twice"
                stores[key] = reg.get(0, 0)
                if t == 0:
                    events.append(("store", int(b), j))
            elif op == "s_waitcnt":
                if t == 0:
                    events.append(("wait", int(re.match(r"vmcnt\((\d+)\)", args[0]).group(1))))
            elif op == "s_nop":
                pass
            else:
                raise AssertionError("unexpected instruction " + ins)
        if first is None:
            first = stores
        assert stores == first, "tile %d differs" % t
    return first, reg, events


def record_events(words):
    out, pc = [], 0
    while True:
        f = fields(words[pc], words[pc + 1])
        kind = KINDS[f["kind"]]
        if kind == "HALT":
            return out
        if kind in ("INPUT", "INPUT_LD"):
            out.append(("wait", f["wait8"] // 8))
        if kind in ("INPUT_LD", "LOAD"):
            out.append(("load", f["blk"], f["j"]))
        if kind == "STORE":
            out.append(("store", f["blk"], f["j"]))
        pc += f["bytes"] // 4


CASES = [(10, 4, (), E.LEVEL_CO_FU_SCHED, 0), (10, 4, (), E.LEVEL_PLAIN, 0), (10, 4, (2, 4, 5, 6), E.LEVEL_CO_FU_SCHED, 0),
         (6, 3, (1, 7), E.LEVEL_CO_FU_SCHED, 24), (14, 4, (0, 13), E.LEVEL_PLAIN, 48), (2, 1, (), E.LEVEL_PLAIN, 0),
         (12, 6, (), E.LEVEL_CO_FU_SCHED, 48), (28, 4, (), E.LEVEL_PLAIN, 0), (10, 4, (3,), E.LEVEL_CO_FU_SCHED, 60)]


@pytest.mark.parametrize("n,p,er,level,K", CASES)
def test_native_code_is_the_program(n, p, er, level, K):
    gen = E.ec_matrix_cauchy(n, p)
    prog = E.ec_compile_slp(n, p, gen, er, level=level, slot_budget=K, native=True)
    info = prog.info
    assert info["native"] == 1
    n_in, n_out = len(prog.in_blocks), len(prog.out_blocks)
    body = asm_body(prog.native_source())
    stores, reg, events = run_symbolic(body, n_in)
    rows = oracle_rows(gen, n, p, er)
    assert sorted(stores) == [(r // 8, r % 8) for r in range(len(rows))]
    for r, want in enumerate(rows):
        assert stores[(r // 8, r % 8)] == want, "row %d" % r
    assert all(reg.get(v, 0) == 0 for v in range(4, 4 + 4 * info["slots"])), "a slot is left non-zero"
    assert events == record_events(prog.bytecode())
    if info["passes"] > 1:  # a second pass reads the inputs again
        assert sum(e[0] == "load" for e in events) > n_in * 8


@pytest.mark.parametrize("n,p,er,level", [(10, 4, (), E.LEVEL_PLAIN), (10, 4, (2, 4, 5, 6), E.LEVEL_CO_FU_SCHED),
                                          (6, 3, (1, 7), E.LEVEL_PLAIN)])
def test_native_pair_kernel_is_the_pair_parts(n, p, er, level):
    """The pair-part kernel: one asm statement per pair part, each the
    part's records; run symbolically they store every output strip once,
    in consecutive pairs of rows, with the bitmatrix row's value."""
    gen = E.ec_matrix_cauchy(n, p)
    prog = E.ec_compile_slp(n, p, gen, er, level=level, native=E.NATIVE_WHOLE | E.NATIVE_PAIRS)
    info = prog.info
    assert info["native"] == E.NATIVE_WHOLE | E.NATIVE_PAIRS
    n_in = len(prog.in_blocks)
    bodies = asm_bodies(prog.native_source(E.NATIVE_PAIRS))
    assert len(bodies) == info["n_pair_parts"] > 1
    rows = oracle_rows(gen, n, p, er)
    got = {}
    first_pair = info["n_parts"] + info["n_row_parts"]
    for q, body in enumerate(bodies):
        stores, reg, events = run_symbolic(body, n_in)
        keys = sorted(8 * b + j for b, j in stores)
        assert keys == list(range(len(got), len(got) + len(keys))) and len(keys) % 2 == 0
        assert not set(keys) & set(got)
        got.update({8 * b + j: v for (b, j), v in stores.items()})
        assert all(reg.get(v, 0) == 0 for v in range(4, 4 + 4 * info["slots"]))
        assert events == record_events(prog.part_bytecode(first_pair + q))
    assert [got[r] for r in range(len(rows))] == rows
    # a program without pair parts gets no pair kernel
    one = E.ec_compile_slp(n, p, gen, er, level=level, native=E.NATIVE_PAIRS, split=E.SPLIT_NEVER)
    assert one.info["native"] == 0


@pytest.mark.parametrize("n,p,er,level", [(10, 4, (), E.LEVEL_PLAIN), (10, 4, (), E.LEVEL_CO_FU_SCHED),
                                          (10, 4, (0, 3, 11, 12), E.LEVEL_CO_FU_SCHED), (6, 3, (1, 7), E.LEVEL_PLAIN),
                                          (12, 6, (), E.LEVEL_CO_FU_SCHED)])
def test_native_block_kernel_is_the_block_parts(n, p, er, level):
    """The block-part kernel: one asm statement per output block, each that
    block part's records; run symbolically each stores exactly its block's
    8 rows, once, with the bitmatrix rows' values."""
    gen = E.ec_matrix_cauchy(n, p)
    prog = E.ec_compile_slp(n, p, gen, er, level=level, native=E.NATIVE_BLOCKS)
    info = prog.info
    assert info["native"] == E.NATIVE_BLOCKS
    n_in, n_out = len(prog.in_blocks), len(prog.out_blocks)
    bodies = asm_bodies(prog.native_source(E.NATIVE_BLOCKS))
    assert len(bodies) == info["n_parts"] > 1
    rows = oracle_rows(gen, n, p, er)
    got = {}
    for q, body in enumerate(bodies):
        stores, reg, events = run_symbolic(body, n_in)
        assert stores and not set(stores) & set(got)
        got.update(stores)
        assert all(reg.get(v, 0) == 0 for v in range(4, 4 + 4 * info["slots"]))
        assert events == record_events(prog.part_bytecode(q))
    assert sorted(got) == [(r // 8, r % 8) for r in range(8 * n_out)]
    assert [got[(r // 8, r % 8)] for r in range(len(rows))] == rows
    # one lost block: no block parts, so no block kernel
    one = E.ec_compile_slp(n, p, gen, [1], level=level, native=E.NATIVE_BLOCKS)
    assert one.info["n_parts"] == 0 and one.info["native"] == 0


def test_native_options_and_errors():
    gen = E.ec_matrix_cauchy(10, 4)
    plain = E.ec_compile_slp(10, 4, gen)
    assert plain.info["native"] == 0
    with pytest.raises(E.EcError) as e:
        plain.native_source()
    assert e.value.name == "EC_ERR_ARG"
    for kw in ({"native": 8}, {"native": 1, "split": E.SPLIT_STAGED}):
        with pytest.raises(E.EcError) as e:
            E.ec_compile_slp(10, 4, gen, **kw)
        assert e.value.name == "EC_ERR_UNSUPPORTED"
    # the same program compiled twice gives the same kernel
    a = E.ec_compile_slp(10, 4, gen, [1, 2], native=True).native_source()
    b = E.ec_compile_slp(10, 4, gen, [1, 2], native=True).native_source()
    assert a == b and "ec_native_kernel" in a
    with pytest.raises(E.EcError) as e:  # compiled without the pair kernel
        E.ec_compile_slp(10, 4, gen, [1, 2], native=True).native_source(E.NATIVE_PAIRS)
    assert e.value.name == "EC_ERR_ARG"


def test_program_cache_native_keys():
    """A cache compiles exactly its native keys with native kernels (the
    serving loop's encode programs); the rest stay interpreter-only."""
    from paper_2108_02692_amd.batching import ProgramCache
    cache = ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=38, native_keys=[(6, 3, ())], native=E.NATIVE_WHOLE)
    assert cache.get(6, 3).info["native"] == E.NATIVE_WHOLE
    assert cache.get(6, 3, (1,)).info["native"] == 0
    assert cache.get(10, 4).info["native"] == 0
    assert cache.get(6, 3) is cache.get(6, 3, ())
