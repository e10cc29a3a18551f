"""The C ABI library on the CPU: it loads, exports every entry point that
include/ec.h declares, and its gfx950 kernels were built the way the
executor's design requires (checked on the assembly of this build)."""
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


@pytest.fixture(scope="module")
def kernel_asm(tmp_path_factory):
    out = tmp_path_factory.mktemp("isa") / "exec.s"
    cmd = [_build.HIPCC, "-x", "hip"] + _build.DEVICE_FLAGS + ["-O3", "-std=c++17", "--cuda-device-only", "-S",
                                                               os.path.join(_build.CSRC, "exec.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def kernels(asm):
    return re.findall(r"^(_ZN2ec15slp_exec_kernelILi(\d+)EEEvNS_8ExecArgsE):[^\n]*\n(.*?)s_endpgm", asm, flags=re.S | re.M)


def test_executor_isa(kernel_asm):
    ks = kernels(kernel_asm)
    assert sorted(int(k) for _, k, _ in ks) == [16, 24, 32, 40, 48]
    for name, K, body in ks:
        # no scratch (spills) in the executor
        assert "scratch_" not in body, name
        # m0 carries the VGPR index; only the executor's own asm may touch it
        outside = re.sub(r";;#ASMSTART.*?;;#ASMEND", "", body, flags=re.S)
        assert not re.search(r"\bm0\b", outside), name
        # every strip load/store uses a scalar base address
        for m in re.finditer(r"global_(load|store)_dwordx4 .*", body):
            assert re.search(r", s\[\d+:\d+\]", m.group(0)), m.group(0)
    meta = dict(re.findall(r"\.name:\s+(_ZN2ec15slp_exec_kernelILi\d+EEEvNS_8ExecArgsE)\n(?:.*\n)*?\s+\.vgpr_count:\s+(\d+)",
                           kernel_asm))
    for name, K, _ in ks:
        if name in meta:
            assert int(meta[name]) <= 4 + 4 * int(K) + 16, (name, meta[name])
