"""Build of libec.so (host compiler + gfx950 executor) with hipcc.

The library is built in-tree, next to this file, so that it travels with the
source tree.  ``build()`` always recompiles; ``ensure_built()`` only builds
when the library is missing.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libec.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["gf.cpp", "slp.cpp", "push.cpp", "capi.cpp", "batch.cpp", "serve.cpp", "program_pool.cpp", "native.cpp", "exec.hip", "staged.hip", "noalloc.hip", "ceiling.hip"]
# Packed FP32 instructions are disabled for all device code (none is used).
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    objs = []
    with tempfile.TemporaryDirectory(prefix="ecbuild") as tmp:
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            # hipcc gives .cpp files a device pass too: gfx950 (they hold no kernels)
            cmd = [HIPCC] + DEVICE_FLAGS + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
            if src.endswith(".hip"):
                cmd = [HIPCC, "-x", "hip"] + DEVICE_FLAGS + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        for cmd, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out.decode(errors="replace")))
            if verbose and out:
                print(out.decode(errors="replace"))
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        link = [HIPCC] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp_lib] + objs + ["-lhiprtc"]
        r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(tmp_lib, LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
