"""CPU sanitizer leg.

1. The C oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer,
   runs every entry point over its largest per-site cases (D3Q19 with four
   species: 69 normals per site) through tests/sanitize_oracle.c.  A planted
   overflow in a copy of the oracle (its normals buffer cut to 64 entries)
   must be reported, which shows that the leg catches that class of error.
2. The HIP library with its host code built under the same sanitizers passes
   the ABI tests (tests/test_abi.py: parameter validation, buffer sizing,
   error paths; no GPU is needed) in a process that preloads the ASan runtime.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = [os.path.join(ROOT, "oracle", n) for n in ("flbe_oracle.c", "flbe_multi.c")]
DRIVER = os.path.join(HERE, "sanitize_oracle.c")
BUILD_DIR = os.path.join(HERE, "_sanitize_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _gcc(out, sources, include=None):
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-Wall", "-Wno-unknown-pragmas", *SAN]
    if include:
        cmd += ["-I", include]
    cmd += ["-o", out, *sources, "-lm"]
    subprocess.run(cmd, check=True)


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    _gcc(exe, [DRIVER, *ORACLE])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout


def test_planted_overflow_is_reported(tmp_path):
    src = open(ORACLE[0]).read()
    planted = src.replace("double u[ORC_MAX_NORMALS];", "double u[64];")
    assert planted != src
    path = tmp_path / "flbe_oracle_planted.c"
    path.write_text(planted)
    exe = str(tmp_path / "planted")
    _gcc(exe, [DRIVER, str(path), ORACLE[1]], include=os.path.join(ROOT, "oracle"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "stack-buffer-overflow" in r.stderr


def _sanitized_library():
    from paper_1410_5584_amd import build
    os.makedirs(BUILD_DIR, exist_ok=True)
    lib = os.path.join(BUILD_DIR, "libfmlb_host_asan.so")
    newest = max(os.path.getmtime(f) for f in build.sources() + [os.path.abspath(build.__file__)])
    if not os.path.exists(lib) or os.path.getmtime(lib) < newest:
        build.build(sanitize_host=True, out=lib)
    return lib, build.asan_runtime()


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_abi_under_host_sanitizers():
    lib, rt = _sanitized_library()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0", FMLB_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi.py")], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout and "error" not in r.stdout.lower().split("passed")[-1]
