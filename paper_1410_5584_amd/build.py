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
SOURCES = ["runtime.hip", "fused_ilp.hip", "batch.hip", "multi.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=on", "-Wall", "-Wno-unused-function",
]

# The instruction-level-parallelism scheduler runs the D3Q19 fused steps (and
# the BF16 D2Q9 one) and the N-species steps faster (three species at 256^3:
# 2.06-2.09 -> 2.005-2.008 ms, four 2.75 -> 2.70, two unchanged); it slows the
# D2Q9 FP32 step and the batched kernels gain nothing from it, so those keep
# the default.
_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
SOURCE_FLAGS = {"fused_ilp.hip": _ILP, "multi.hip": _ILP}


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (CPU checks of the
# host runtime only; the device code is built as usual).  Each flag goes to
# the host compilation alone.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def compile_commands(objdir: str, out: str, sanitize_host: bool = False) -> tuple[list[list[str]], list[str]]:
    """(per-source compile commands, link command)."""
    objs, cmds = [], []
    extra = (["-O1", "-g"] + HOST_SANITIZE) if sanitize_host else []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        cmds.append([hipcc(), *FLAGS, *SOURCE_FLAGS.get(s, []), *extra, "-c", "-o", obj, os.path.join(CSRC, s)])
        objs.append(obj)
    link = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *(HOST_SANITIZE if sanitize_host else []),
            "-o", out, *objs]
    return cmds, link


def build(verbose: bool = False, sanitize_host: bool = False, out: str | None = None) -> str:
    """Compile every source into libfmlb.so (always recompiles), or with
    sanitize_host into `out`: the same library with the host code built
    under AddressSanitizer and UndefinedBehaviorSanitizer (load it into a
    process that preloads the compiler's ASan runtime)."""
    target = out or LIB
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=os.path.dirname(target))
    os.close(fd)
    try:
        with tempfile.TemporaryDirectory() as objdir:
            cmds, link = compile_commands(objdir, tmp, sanitize_host)
            if verbose:
                for c in cmds + [link]:
                    print(" ".join(c), flush=True)
            with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
                for r in list(ex.map(lambda c: subprocess.run(c), cmds)):
                    if r.returncode != 0:
                        raise subprocess.CalledProcessError(r.returncode, r.args)
            subprocess.run(link, check=True)
        os.replace(tmp, target)
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
    return target


def sources() -> list[str]:
    """Every file the library is compiled from."""
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)) + [os.path.join(HERE, "..", "include", "fmlb.h")]


def asan_runtime() -> str:
    """The compiler's AddressSanitizer runtime (to preload for a host-sanitized library)."""
    out = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang"),
                          "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("no clang ASan runtime found")
    return found[-1]


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
