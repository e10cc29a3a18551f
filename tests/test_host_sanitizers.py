"""Host code under AddressSanitizer, UndefinedBehaviorSanitizer and
LeakSanitizer, on the CPU: the library's C++ compile path through its C ABI
(tests/sanitize/lib_driver.cpp; device launchers stubbed, no HIP call made)
and the C oracle (tests/sanitize/oracle_driver.c).  Both are built with the
system g++/gcc into a temporary directory."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2108_02692_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ASAN_OPTIONS="detect_leaks=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs the system g++ and gcc")


def run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r.stdout + r.stderr


def run_driver(exe, cwd):
    r = subprocess.run([exe], cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    if "LeakSanitizer has encountered a fatal error" in out:  # no ptrace here: leaks unchecked
        r = subprocess.run([exe], cwd=cwd, capture_output=True, text=True, timeout=600,
                           env=dict(ENV, ASAN_OPTIONS="detect_leaks=0"))
        out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


@pytest.mark.slow
def test_library_host_code_sanitized(tmp_path):
    srcs = ["gf.cpp", "slp.cpp", "push.cpp", "capi.cpp", "batch.cpp", "serve.cpp", "program_pool.cpp", "native.cpp"]
    inc = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    jobs = [(["g++"] + inc + SAN + ["-c", os.path.join(CSRC, s), "-o", s + ".o"]) for s in srcs]
    jobs.append(["g++"] + inc + SAN + ["-c", os.path.join(HERE, "sanitize", "lib_driver.cpp"), "-o", "drv.o"])
    with ThreadPoolExecutor(max_workers=6) as ex:
        list(ex.map(lambda c: run(c, tmp_path), jobs))
    run(["g++"] + SAN + ["-o", "lib_driver", "drv.o"] + [s + ".o" for s in srcs] +
        ["-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"], tmp_path)
    out = run_driver(str(tmp_path / "lib_driver"), tmp_path)
    assert "0 check failures" in out


def test_oracle_sanitized(tmp_path):
    run(["gcc", "-std=c11"] + SAN + ["-o", "oracle_driver", os.path.join(HERE, "sanitize", "oracle_driver.c"),
                                     os.path.join(ROOT, "oracle", "rs_oracle.c")], tmp_path)
    out = run_driver(str(tmp_path / "oracle_driver"), tmp_path)
    assert "0 check failures" in out
