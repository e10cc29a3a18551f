"""The C ABI library on the CPU: it loads, exports every entry point that
include/ec.h declares, and its gfx950 kernels were built the way the
executor's design requires (checked on the assembly of the library built here)."""
import os
import re
import subprocess

import pytest

import paper_2108_02692_amd as E
from paper_2108_02692_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:ec_status|void|const char\s*\*)\s*\*?\s*(ec_\w+)\s*\(",
                                 src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "ec_compile_slp" in names and "ec_encode" in names and "ec_decode" in names
    out = subprocess.run(["nm", "-D", "--defined-only", E.lib()._name], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ec_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert getattr(E.lib(), n) is not None


def test_status_strings():
    assert E.ec_status_str(0) == "ok"
    for s in range(1, 9):
        assert E.ec_status_str(s) and E.ec_status_str(s) != "unknown status"


SLOT_BUDGETS = [24, 32, 36, 38, 40, 44, 48, 56, 60]
OBJDUMP = os.path.join(os.path.dirname(_build.HIPCC), "..", "llvm", "bin", "llvm-objdump")


def assemble(d, name):
    """Assembly and disassembly of csrc/<name>.hip built here (gfx950)."""
    base = [_build.HIPCC, "-x", "hip"] + _build.DEVICE_FLAGS + ["-O3", "-std=c++17", "--cuda-device-only",
                                                                "-I", os.path.join(ROOT, "include")]
    src = os.path.join(_build.CSRC, name + ".hip")
    subprocess.run(base + ["-S", src, "-o", str(d / (name + ".s"))], check=True, capture_output=True)
    subprocess.run(base + ["--no-gpu-bundle-output", "-c", src, "-o", str(d / (name + ".co"))], check=True,
                   capture_output=True)
    dis = subprocess.run([OBJDUMP, "-d", "--no-show-raw-insn", str(d / (name + ".co"))], check=True,
                         capture_output=True, text=True).stdout
    return (d / (name + ".s")).read_text(), dis


@pytest.fixture(scope="module")
def built(tmp_path_factory):
    """The direct executor (exec.hip)."""
    return assemble(tmp_path_factory.mktemp("isa"), "exec")


@pytest.fixture(scope="module")
def built_staged(tmp_path_factory):
    """The staged executor (staged.hip)."""
    return assemble(tmp_path_factory.mktemp("isa_staged"), "staged")


def kernel_names():
    for K in SLOT_BUDGETS:
        yield K, "_ZN2ec%d%s_kernel_%dENS_%d%sE" % (18, "slp_exec", K, 8, "ExecArgs")
        yield K, "_ZN2ec%d%s_kernel_%dENS_%d%sE" % (19, "slp_batch", K, 9, "BatchArgs")


def staged_names():
    for K in SLOT_BUDGETS:
        yield K, "_ZN2ec%d%s_kernel_%dENS_%d%sE" % (20, "slp_staged", K, 8, "ExecArgs")


def test_generated_sources_are_current(tmp_path):
    """exec.hip and staged.hip are what gen_exec.py writes now."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen_exec", os.path.join(_build.CSRC, "gen_exec.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    gen.main(str(tmp_path))
    for name in ("exec.hip", "staged.hip"):
        with open(os.path.join(_build.CSRC, name)) as a, open(tmp_path / name) as b:
            assert a.read() == b.read(), name + " is stale: run gen_exec.py"


def instructions(dis, name):
    m = re.search(r"<%s>:\n(.*?)s_endpgm" % re.escape(name), dis, re.S)
    assert m, name
    out = {}
    for line in m.group(1).splitlines():
        mm = re.match(r"\s+(\S.*?)\s+//\s+([0-9A-F]+):", line)
        if mm:
            out[int(mm.group(2), 16)] = mm.group(1).strip()
    return out


def test_executor_isa(built):
    asm, _ = built
    meta = dict(re.findall(r"\.name:\s+(\S+)\n(?:.*\n)*?\s+\.vgpr_count:\s+(\d+)", asm))
    scratch = dict(re.findall(r"\.name:\s+(\S+)\n(?:.*\n)*?\s+\.private_segment_fixed_size:\s+(\d+)", asm))
    for K, name in kernel_names():
        body = re.search(r"^%s:[^\n]*\n(.*?)s_endpgm" % re.escape(name), asm, re.S | re.M).group(1)
        assert scratch[name] == "0", name  # no spills
        # m0 carries the VGPR index; only the executor's own asm may touch it
        outside = re.sub(r";;#ASMSTART.*?;;#ASMEND", "", body, flags=re.S)
        assert not re.search(r"\bm0\b", outside), name
        vgprs = int(meta[name])
        assert 4 + 4 * K + 1 <= vgprs <= 256, (name, vgprs)
        # the occupancy the batch launcher assumes (granules of 8 of 512)
        waves = 512 // (-(-vgprs // 8) * 8)
        assert waves >= (4 if K <= 24 else 3 if K <= 38 else 2), (name, vgprs)


def test_interpreter_layout(built):
    """The host encodes byte offsets into the executor's tables; check them
    against the built executor: handlers 512 bytes apart, 20-byte run steps reading
    window words 15..2, 16-byte load entries, 8-byte wait entries."""
    _, dis = built
    for K, name in kernel_names():
        ins = instructions(dis, name)
        addrs = sorted(ins)
        gp = [a for a in addrs if ins[a] == "s_getpc_b64 s[82:83]"]
        assert len(gp) == 1, name
        i = addrs.index(gp[0])
        base = {}
        for a in addrs[i + 1:i + 13:2]:
            reg, lit = re.match(r"s_add_u32 s(\d+), s82, (0x[0-9a-f]+)", ins[a]).groups()
            base[int(reg)] = gp[0] + 4 + int(lit, 16)
        for h, W in ((base[84], 36), (base[86], 52)):
            assert h % 512 == 0
            for kind in range(8):
                want = "s_branch" if kind == 6 else "s_bfe_u32 s74, s%d, 0x7000c" % W
                assert ins.get(h + 512 * kind, "").startswith(want), (name, kind)
        for r, W in ((base[88], 36), (base[90], 52)):
            for step in range(14):
                assert ins.get(r + 20 * step) == "s_set_gpr_idx_on s%d, gpr_idx(SRC0,DST)" % (W + 15 - step)
            assert ins.get(r + 280) == "s_set_gpr_idx_off"
        for k in range(K):
            assert ins.get(base[92] + 16 * k, "").startswith("global_load_dwordx4 v[%d:%d]" % (4 + 4 * k, 7 + 4 * k))
            assert ins[base[92] + 16 * k].endswith(" nt")
        for k in range(64):
            assert ins.get(base[94] + 8 * k, "").startswith("s_waitcnt vmcnt(%d)" % k)
        # the prefetch handler writes only the pinned scratch register
        pf = [ins[a] for a in addrs if base[84] + 7 * 512 <= a < base[84] + 8 * 512 and "global_load" in ins[a]]
        assert pf == ["global_load_dword v%d, v%s, s[72:73]" % (4 + 4 * K, pf[0].split(", v")[1].split(",")[0])]


def test_staged_isa(built_staged):
    """The staged kernels: no spills; the interpreter's s_set_gpr_idx_on
    writes m0, which the LDS-DMA loads read as their LDS address, so m0 is
    set again after the last interpreter block before every such load; the
    loads are non-temporal; the occupancy the launcher assumes holds."""
    asm, _ = built_staged
    meta = dict(re.findall(r"\.name:\s+(\S+)\n(?:.*\n)*?\s+\.vgpr_count:\s+(\d+)", asm))
    scratch = dict(re.findall(r"\.name:\s+(\S+)\n(?:.*\n)*?\s+\.private_segment_fixed_size:\s+(\d+)", asm))
    for K, name in staged_names():
        body = re.search(r"^%s:[^\n]*\n(.*?)s_endpgm" % re.escape(name), asm, re.S | re.M).group(1)
        assert scratch[name] == "0", name
        lines = re.sub(r";;#ASMSTART.*?;;#ASMEND", ";;ASM", body, flags=re.S).splitlines()
        dma, m0_set = 0, False
        for ln in lines:
            if ";;ASM" in ln:
                m0_set = False
            elif re.search(r"s_mov_b32 m0,", ln):
                m0_set = True
            elif "global_load_lds_dwordx4" in ln:
                dma += 1
                assert m0_set, (name, ln)
                assert ln.rstrip().endswith(" nt"), (name, ln)
        assert dma >= 1, name
        vgprs = int(meta[name])
        assert 4 + 4 * K + 1 <= vgprs <= 256, (name, vgprs)
        waves = 512 // (-(-vgprs // 8) * 8)
        assert waves >= (4 if K <= 24 else 3 if K <= 38 else 2), (name, vgprs)


def test_staged_interpreter_layout(built_staged):
    """The staged interpreter keeps the direct one's tables (handlers 512
    bytes apart, 20-byte run steps), with its 16-byte load entries reading
    LDS into the slot from the address in the spare register."""
    _, dis = built_staged
    for K, name in staged_names():
        ins = instructions(dis, name)
        addrs = sorted(ins)
        gp = [a for a in addrs if ins[a] == "s_getpc_b64 s[82:83]"]
        assert len(gp) == 1, name
        i = addrs.index(gp[0])
        base = {}
        for a in addrs[i + 1:i + 13:2]:
            reg, lit = re.match(r"s_add_u32 s(\d+), s82, (0x[0-9a-f]+)", ins[a]).groups()
            base[int(reg)] = gp[0] + 4 + int(lit, 16)
        for h, W in ((base[84], 36), (base[86], 52)):
            assert h % 512 == 0
            for kind in range(8):
                want = "s_branch" if kind == 6 else "s_bfe_u32 s74, s%d, 0x7000c" % W
                assert ins.get(h + 512 * kind, "").startswith(want), (name, kind)
        for r, W in ((base[88], 36), (base[90], 52)):
            for step in range(14):
                assert ins.get(r + 20 * step) == "s_set_gpr_idx_on s%d, gpr_idx(SRC0,DST)" % (W + 15 - step)
        for k in range(K):
            assert ins.get(base[92] + 16 * k) == "ds_read_b128 v[%d:%d], v%d" % (4 + 4 * k, 7 + 4 * k, 4 + 4 * K)
        # no global loads into the slots and no waits on the vector memory counter inside the interpreter
        table = [ins[a] for a in addrs if base[84] <= a < base[92] + 16 * K]
        assert not any(t.startswith("global_load") or "vmcnt" in t for t in table), name


def test_launch_argument_errors_need_no_device():
    """Every argument check of ec_encode / ec_decode happens before any HIP
    call, so it is reported on a host without a GPU too (pointers here are
    plain integers, never dereferenced)."""
    gen = E.ec_matrix_cauchy(10, 4)
    enc = E.ec_compile_slp(10, 4, gen)
    dec = E.ec_compile_slp(10, 4, gen, [3])
    S = 1 << 16
    ins = [0x100000 + k * S for k in range(10)]
    outs = [0x10000000 + k * S for k in range(4)]
    cases = [
        (lambda: E.ec_encode(enc, ins, outs, 0), "EC_ERR_ALIGN"),
        (lambda: E.ec_encode(enc, ins, outs, S + 64), "EC_ERR_ALIGN"),
        (lambda: E.ec_encode(enc, ins[:-1] + [ins[-1] + 8], outs, S), "EC_ERR_ALIGN"),
        (lambda: E.ec_encode(enc, ins, outs[:-1] + [ins[0] + 128], S), "EC_ERR_ARG"),  # output overlaps an input
        (lambda: E.ec_encode(enc, ins, outs[:-1] + [outs[0] + 128], S), "EC_ERR_ARG"),  # outputs overlap
        (lambda: E.ec_encode(enc, ins[:-1] + [0], outs, S), "EC_ERR_ARG"),
        (lambda: E.ec_encode(enc, ins, outs, 8 << 29), "EC_ERR_UNSUPPORTED"),  # strips of 512 MiB: too long
        (lambda: E.ec_decode(enc, ins, outs, S), "EC_ERR_ARG"),
        (lambda: E.ec_encode(dec, ins, outs[:1], S), "EC_ERR_ARG"),
    ]
    for call, name in cases:
        with pytest.raises(E.EcError) as e:
            call()
        assert e.value.name == name


def test_compile_limits_and_degenerate_codecs():
    from bytecode_sim import simulate
    import numpy as np
    import oracle
    from oracle import slp as S
    for n, p, er in ((1, 1, ()), (1, 3, ()), (1, 3, (0,)), (1, 3, (0, 2, 3)), (2, 0, ()), (28, 4, ()),
                     (28, 4, (0, 5, 27, 31)), (31, 1, (30,)), (4, 12, ())):
        gen = E.ec_matrix_cauchy(n, p)
        G = np.array(gen, dtype=np.uint8)
        D = oracle.decode_matrix(G, n, p, list(er))[0] if er else G[n:]
        rows = S.rows_from_bitmatrix(oracle.bitmatrix(D)) if len(D) else []
        for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
            prog = E.ec_compile_slp(n, p, gen, list(er), level=level)
            got = simulate(prog.bytecode(), prog.info["slots"], n, len(prog.out_blocks))
            assert [got[o] for o in range(len(rows))] == rows, (n, p, er, level)
    with pytest.raises(E.EcError) as e:
        E.ec_compile_slp(29, 4, E.ec_matrix_cauchy(29, 4))  # 33 blocks > the 32-entry table
    assert e.value.name == "EC_ERR_ARG"
