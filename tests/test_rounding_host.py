"""Host build of the stochastic-rounding conversions of the 16-bit storage
(paper_1410_5584_amd/csrc/storage.h, the source the kernels compile): every
value of the hash bits they use is tried, and the mean of the rounded values
must equal the input (unbiased rounding), with both neighbouring
representable values occurring; this includes FP16 subnormals, whose spacing
2^-24 is coarser than the 13 bits dithered in the normal range.  The hash
must depend on the site, the value index, the step and both seed words."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(_hipcc()), reason="needs hipcc")
def test_stochastic_rounding_is_unbiased(tmp_path):
    exe = str(tmp_path / "sr_check")
    subprocess.run([_hipcc(), "-O2", "-std=c++17", "--offload-host-only", "-o", exe,
                    os.path.join(HERE, "sr_rounding_check.cpp")], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip().endswith("ok")
