"""Pins of the oracle's random numbers.

- Philox4x32-10 against rocRAND's independent implementation of the same
  published bijection (Salmon et al., SC'11), on many (counter, key) tuples;
- the 23-bit uniform extraction convention;
- Box-Muller normals: moments, Kolmogorov-Smirnov against scipy's normal CDF,
  independence of the pairs (Sec. VI A asks for independent Gaussian noise per
  mode and site, drawn with Box-Muller).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand_ref.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(7)
    tuples = rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64)
    tuples[:8] = 0
    tuples[1, 0] = 1
    tuples[2, 4] = 1
    tuples[3] = 2 ** 32 - 1
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in tuples) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(tuples)
    for row, r in zip(tuples, ref):
        got = orc.philox(row[:4], row[4:])
        assert got == r, (row, got, r)


def test_uniform_extraction(orc):
    """Word w of block j gives the pair (u_2w', u_2w'+1) from its high and
    low 16 bits, u = (2U + 1) / 2^17."""
    seed, site, step = 0x1234_5678_9ABC, 77, 3_000_000_123
    u = orc.uniforms(seed, site, step, 24)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for j in range(3):
        x = orc.philox([site, step & 0xFFFFFFFF, j, step >> 32], key)
        for t in range(4):
            k = 8 * j + 2 * t
            assert u[k] == (2 * (x[t] >> 16) + 1) / 2.0 ** 17
            assert u[k + 1] == (2 * (x[t] & 0xFFFF) + 1) / 2.0 ** 17
    assert np.all(u > 0) and np.all(u < 1)


def test_normal_tail_bound_and_variance_bias(orc):
    """16-bit uniforms cap |z| at sqrt(2 ln 2^17) = 4.85; the variance of the
    discrete Box-Muller radius differs from 2 by less than 1e-4 (midpoint sum
    of -2 ln u over the 2^16 grid values)."""
    z = np.concatenate([orc.normals(3, s, 1, 33) for s in range(3000)])
    assert np.max(np.abs(z)) <= np.sqrt(2 * np.log(2.0 ** 17)) + 1e-12
    U = np.arange(2 ** 16)
    mean_r2 = np.mean(-2 * np.log((2 * U + 1) / 2.0 ** 17))
    assert abs(mean_r2 - 2.0) < 1e-4


def _many_normals(orc, n_sites=20000, K=14, seed=9, step=5):
    return np.array([orc.normals(seed, s, step, K) for s in range(n_sites)])


def test_box_muller_statistics(orc):
    z = _many_normals(orc)
    flat = z.ravel()
    n = flat.size
    assert abs(flat.mean()) < 5 / np.sqrt(n)
    assert abs(flat.var() - 1) < 5 * np.sqrt(2 / n)
    kurt = stats.kurtosis(flat, fisher=False)
    assert abs(kurt - 3) < 5 * np.sqrt(24 / n)
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    # each normal index separately is N(0, 1)
    for k in range(z.shape[1]):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-5, k
    # independence: correlation matrix across indices (incl. the cos/sin pair)
    C = np.corrcoef(z.T)
    off = C[~np.eye(C.shape[0], dtype=bool)]
    assert np.max(np.abs(off)) < 6 / np.sqrt(z.shape[0])


def test_normals_differ_by_site_step_seed(orc):
    a = orc.normals(1, 10, 4, 33)
    assert not np.allclose(a, orc.normals(1, 11, 4, 33))
    assert not np.allclose(a, orc.normals(1, 10, 5, 33))
    assert not np.allclose(a, orc.normals(2, 10, 4, 33))
    assert np.array_equal(a, orc.normals(1, 10, 4, 33))
    # a prefix of the stream does not depend on how many normals are drawn
    assert np.array_equal(orc.normals(1, 10, 4, 14), a[:14])
