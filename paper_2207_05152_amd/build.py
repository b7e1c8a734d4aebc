"""Build libdlic.so for gfx950 in-tree with hipcc.

Each source compiles to its own object in parallel, then one hipcc line links
them into the shared library.

Usage: python -m paper_2207_05152_amd.build   (or build() from Python)
       python -m paper_2207_05152_amd.build --sanitize-host   (host code under ASan + UBSan:
       LD_PRELOAD=<clang>/lib/linux/libclang_rt.asan-x86_64.so DLIC_LIB=<the library>
       python -m pytest tests -m "not gpu")
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libdlic.so")

SOURCES = ["dlic_api.hip", "dlic_encode.hip", "dlic_decode.hip", "dlic_train.hip", "dlic_probe.hip",
           "dlic_deep.hip", "dlic_deep12.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # encoder and decoder must round identically: no contraction into FMA
    "-ffp-contract=off",
    # packed FP32 ops stay off (only scalar VALU FP32 and MFMA are used)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


# Host-side sanitizers for the CPU checks of the library's host code (argument
# checks, weight conversion, header parsing, batch plans); the device code is
# compiled as usual.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    """Compile every source for gfx950 and link libdlic.so (or, with sanitize, a
    library whose host code runs under AddressSanitizer and UBSan, to be loaded
    with the ASan runtime preloaded, DLIC_LIB pointing at it)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = out or (os.path.join(HERE, "libdlic_hostsan.so") if sanitize else LIB)
    extra = SANITIZE_HOST if sanitize else []
    with tempfile.TemporaryDirectory(prefix="dlic_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[hipcc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
        if any(rcs):
            raise RuntimeError("hipcc failed compiling libdlic sources")
        tmp = lib + ".tmp"
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if sanitize:
            link[3:3] = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
        if _run(link, verbose):
            raise RuntimeError("hipcc failed linking " + os.path.basename(lib))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize-host" in sys.argv))
