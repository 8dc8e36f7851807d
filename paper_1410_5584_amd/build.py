"""Build the HIP library libfmlb.so in-tree for gfx950 with hipcc.

Every source is compiled to an object with the common flags plus its own
(SOURCE_FLAGS), in parallel, and the objects are linked into libfmlb.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmlb.so")
SOURCES = ["runtime.hip", "fused_bf16.hip", "batch.hip", "multi.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=on", "-Wall", "-Wno-unused-function",
]

# The BF16 fused step is ALU-bound; the instruction-level-parallelism
# scheduler runs it faster (it slows the FP32 and FP16 forms, which stay in
# runtime.hip with the default scheduler).
SOURCE_FLAGS = {"fused_bf16.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def compile_commands(objdir: str, out: str) -> tuple[list[list[str]], list[str]]:
    """(per-source compile commands, link command)."""
    objs, cmds = [], []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        cmds.append([hipcc(), *FLAGS, *SOURCE_FLAGS.get(s, []), "-c", "-o", obj, os.path.join(CSRC, s)])
        objs.append(obj)
    link = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out, *objs]
    return cmds, link


def build(verbose: bool = False) -> str:
    """Compile every source into libfmlb.so (always recompiles)."""
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=HERE)
    os.close(fd)
    try:
        with tempfile.TemporaryDirectory() as objdir:
            cmds, link = compile_commands(objdir, tmp)
            if verbose:
                for c in cmds + [link]:
                    print(" ".join(c), flush=True)
            with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
                for r in list(ex.map(lambda c: subprocess.run(c), cmds)):
                    if r.returncode != 0:
                        raise subprocess.CalledProcessError(r.returncode, r.args)
            subprocess.run(link, check=True)
        os.replace(tmp, LIB)
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
