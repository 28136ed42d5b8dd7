"""Builds libdapt.so, the C-ABI library of gfx950 HIP kernels, in-tree.

    python -m paper_1806_08815_amd.build

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are
disabled for all device code, and floating-point contraction is off (the one
floating-point decision on the device, the replica-exchange test, is a single
IEEE multiply and compare).  Loops start on 64-byte boundaries, so the step
loops' speed does not shift with the length of the code in front of them.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdapt.so")
SOURCES = ["da_kernels.hip", "da_probe.hip", "da_tables.cpp", "da_api.cpp", "da_server.cpp",
           "da_noalloc.hip"]
HEADERS = ["da_internal.h", "da_runtime.h"]


def source_hash() -> str:
    """SHA-256 over the library's sources and headers (and include/da.h), in a
    fixed order.  The built library reports the hash it was built from
    (da_build_id), so a binary older than its sources is detected at load."""
    import hashlib
    h = hashlib.sha256()
    for name in SOURCES + HEADERS:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(INCLUDE, "da.h"), "rb") as f:
        h.update(b"da.h\0" + f.read())
    return h.hexdigest()


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build_library(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-falign-loops=64",
              "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]
    build_id = source_hash()

    def compile_one(src):
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *common, "-c", os.path.join(CSRC, src), "-o", obj]
        if src == "da_api.cpp":
            cmd.insert(1, f'-DDAPT_BUILD_ID="{build_id}"')
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in r.stderr.splitlines()
                        if "packed-fp32-ops' is not a recognized feature" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
        return obj

    # the sources compile independently: all at once
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
