"""Pins of the oracle's site-wise entry points, which the full-size GPU parity
tests use as their checker.

- orc_collide_site: the post-collision populations of one site (the
  right-hand side of Eq. (84) before streaming).  Streamed to r + c_i they
  must be the next state of orc_step, with the thermal noise of Eq. (74) on,
  the lattice force of Eq. (87) on and every relaxation rate different, on
  both lattices.
- orc_health: counts of sites with a non-positive density and of sites with a
  non-finite population; pinned on states built by hand whose counts are
  known.
- orc_normals: the number of normals per site is bounded; a count outside
  the bound is an error, never a silent fill.
"""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("lattice_id, shape", [(0, (1, 6, 7)), (1, (4, 3, 5))])
def test_collide_site_is_the_step(orc, lattice_id, shape):
    nz, ny, nx = shape
    s = orc.Sim(orc.Params(lattice=lattice_id, nx=nx, ny=ny, nz=nz, tau=(0.8, 1.3), tau_d=0.9, G=0.6,
                           kT=1e-4, seed=11))
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=4, amplitude=0.05)
    s.init_density(r1, r2)
    s.step(3)
    fs = np.stack([s.collide_site(r) for r in range(s.nsites)], axis=-1)  # [2, Q, sites]
    s.step(1)
    f1 = s.populations().reshape(2, s.Q, -1)
    c = s.c
    moved = 0.0
    for r in range(s.nsites):
        x, y, z = r % nx, (r // nx) % ny, r // (nx * ny)
        for i in range(s.Q):
            dst = (x + c[i, 0]) % nx + nx * ((y + c[i, 1]) % ny + ny * ((z + c[i, 2]) % nz))
            assert np.allclose(f1[:, i, dst], fs[:, i, r], rtol=0, atol=1e-15)
            moved = max(moved, float(np.max(np.abs(fs[:, i, r] - s.w[i] * np.array([r1.flat[r], r2.flat[r]])))))
    assert moved > 1e-4  # the step did something (noise and force act)


def test_collide_site_rejects_bad_sites(orc):
    s = orc.Sim(orc.Params(lattice=0, nx=4, ny=3, nz=1))
    s.init_density(1.0, 1.0)
    for bad in (-1, 12):
        with pytest.raises(RuntimeError):
            s.collide_site(bad)


def test_health_counts(orc):
    """Known states: the rest state has no bad site; one site with a negative
    density of species 1, one with a NaN population of species 2 (its density
    is then NaN, so not positive either), one with an infinite population whose
    density stays positive."""
    s = orc.Sim(orc.Params(lattice=0, nx=8, ny=8, nz=1))
    s.init_density(1.0, 1.0)
    assert s.health() == (0, 0)
    f = s.populations()
    f[0, :, 0, 2, 3] = -0.1
    f[1, 4, 0, 5, 5] = np.nan
    s.set_populations(f, 0)
    assert s.health() == (2, 1)
    f[0, 1, 0, 7, 0] = np.inf
    s.set_populations(f, 0)
    assert s.health() == (2, 2)
    # zero density is not positive
    f = s.populations()
    f[:, :, 0, 1, 1] = np.nan_to_num(f[:, :, 0, 1, 1])
    f[1, :, 0, 1, 1] = 0.0
    s.set_populations(f, 0)
    assert s.health() == (3, 2)


def test_health_d3q19_brute_force(orc):
    """The counts equal a direct evaluation of the definition on a random state."""
    shape = (3, 4, 5)
    s = orc.Sim(orc.Params(lattice=1, nx=5, ny=4, nz=3))
    rng = np.random.default_rng(1)
    f = rng.normal(0.05, 0.05, size=(2, 19) + shape)
    f[0, 3, 1, 2, 2] = np.inf
    f[1, 0, 0, 0, 4] = np.nan
    s.set_populations(f, 0)
    rho = f.sum(axis=1)
    with np.errstate(invalid="ignore"):
        nonpos = int(np.sum(~((rho[0] > 0) & (rho[1] > 0))))
    nonfinite = int(np.sum(~np.isfinite(f).all(axis=(0, 1))))
    assert nonpos > 0 and nonfinite == 2
    assert s.health() == (nonpos, nonfinite)


def test_normals_count_bound(orc):
    assert orc.normals(1, 0, 0, 0).shape == (0,)
    z = orc.normals(3, 7, 9, orc.MAX_NORMALS)
    assert z.shape == (orc.MAX_NORMALS,) and np.all(np.isfinite(z))
    # the first normals of a longer request are the same numbers
    assert np.array_equal(orc.normals(3, 7, 9, 33), z[:33])
    for bad in (orc.MAX_NORMALS + 1, -1):
        with pytest.raises(ValueError):
            orc.normals(3, 7, 9, bad)
