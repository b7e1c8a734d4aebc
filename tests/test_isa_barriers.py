"""Workgroup barriers in the compiled kernels sit at most one loop deep.

A loop around a barrier whose exit condition the compiler takes as divergent
may be restructured into a loop nested inside another: the lanes that leave
the inner loop early wait while the rest of their wave runs around it, so one
wave reaches the barrier with part of its lanes ahead of the others.  In the
persistent batch decoder that let lanes 1..63 of wave 0 re-read the work item
before lane 0 had taken the next ticket, and the kernel never finished.  Our
kernels have at most one loop around their barriers (the persistent work loop,
the encoder's chunk loop), so a barrier two loops deep in the device assembly
can only come from such a split.  The assembly's block comments give each
block's loop depth."""
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2207_05152_amd import build as B

SOURCES = ["dlic_decode.hip", "dlic_encode.hip", "dlic_train.hip"]


def _device_asm(src, outdir):
    out = os.path.join(outdir, src + ".s")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [hipcc, *flags, "-I", B.INCLUDE, "--cuda-device-only", "-S",
           os.path.join(B.CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return out


def barrier_depths(asm_text):
    """{kernel: [loop depth of each s_barrier]} from device assembly."""
    res, kern, depth = {}, None, 0
    for ln in asm_text.split("\n"):
        m = re.match(r"^(_Z\w+):", ln)
        if m:
            kern, depth = m.group(1), 0
            res[kern] = []
            continue
        if kern is None:
            continue
        if re.match(r"^(\.LBB\w+|; %bb\.\d+):", ln):
            # a block inside loops names its innermost loop's depth; a loop
            # header names its parent first and its own depth on the next line
            d = re.search(r"Depth=(\d+)", ln)
            depth = int(d.group(1)) if d else 0
        h = re.search(r"Loop Header: Depth=(\d+)", ln)
        if h:
            depth = int(h.group(1))
        s = ln.strip()
        if s.startswith("s_barrier"):
            res[kern].append(depth)
        if s.startswith(".Lfunc_end"):
            kern = None
    return res


def test_depth_parser_on_a_hand_example():
    asm = "\n".join([
        "_Zkernel:", "\ts_barrier",
        ".LBB0_1:   ; =>This Loop Header: Depth=1", "\ts_barrier",
        ".LBB0_2:   ;   Parent Loop BB0_1 Depth=1", "; =>  This Inner Loop Header: Depth=2",
        "\ts_barrier",
        "; %bb.3:   ;   in Loop: Header=BB0_1 Depth=1", "\ts_barrier",
        ".LBB0_4:", "\ts_barrier", ".Lfunc_end0:",
    ])
    # block 2 is the header of a loop inside loop 1: its own depth is on the
    # comment line after its label
    assert barrier_depths(asm) == {"_Zkernel": [0, 1, 2, 1, 0]}


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_no_barrier_two_loops_deep(tmp_path):
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        outs = list(ex.map(lambda s: _device_asm(s, str(tmp_path)), SOURCES))
    seen = 0
    for out in outs:
        with open(out) as fh:
            depths = barrier_depths(fh.read())
        for kern, ds in depths.items():
            seen += len(ds)
            assert all(d <= 1 for d in ds), (kern, ds)
    assert seen > 0
    # the persistent batch decoder keeps its barriers inside its one work loop
    with open(outs[0]) as fh:
        dec = barrier_depths(fh.read())
    batch = [ds for k, ds in dec.items() if "batch_decode_kernel" in k]
    assert batch and all(max(ds) == 1 for ds in batch)
