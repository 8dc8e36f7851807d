"""One-GPU stand-in for the slab decomposition of a lattice across GPUs.

A D3Q19 lattice of NZ planes is split into two z-slabs.  Each slab runs as
its own lattice of nz/2 + 4 planes: two halo planes on each side, because
the force on a slab's boundary plane needs the pre-collision densities of
the next plane outward, and that plane's densities are pulled from one
plane further out.  After every step the halo planes are refreshed with the
owning slab's post-collision populations (here through host copies of the
raw state; across GPUs a send/receive per face).  The slabs' own planes must
then equal the undivided lattice bit for bit.

With thermal noise on, each slab sets its noise-counter site offset
(fmlb_set_counter_offset: the undivided lattice's index of its first site
minus its own), so every site draws the noise it draws in the undivided
run.  Checked: the streaming, the density ring and the force across the
cut, the halo depth, and the noise keying.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NX, NY, NZ = 16, 8, 12
HALO = 2


@pytest.fixture(scope="module")
def fm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1410_5584_amd as fm
    fm.lib()
    return fm


def _say(*a):
    print(*a, flush=True)


def _params(fm, nz, storage, kT=0.0, flags=0):
    return fm.Params(lattice="d3q19", storage=storage, nx=NX, ny=NY, nz=nz, tau=(0.8, 1.2), tau_d=0.9, G=0.9,
                     kT=kT, seed=3, flags=flags)


def _planes(raw, storage, nz):
    """Raw state as [2 * Q, nz, ny * nx] words of the storage type."""
    dt = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[storage]
    return raw.view(dt).reshape(-1, nz, NY * NX)


@pytest.mark.parametrize("storage,kT,flags", [("f64", 0.0, 0), ("f32", 0.0, 0), ("f64", 1e-4, 0), ("f32", 1e-4, 0),
                                              ("bf16", 1e-4, 4)])
def test_two_slabs_equal_the_undivided_lattice(fm, storage, kT, flags):
    """flags 4 = stochastic 16-bit rounding, whose offsets hash the global
    site index too."""
    import workloads
    _say("case two z-slabs with halo exchange,", storage, "kT", kT, "flags", flags)
    r1, r2 = workloads.initial_density((NZ, NY, NX), "perturbed", seed=12, amplitude=0.05)
    whole = fm.Lattice(_params(fm, NZ, storage, kT, flags))
    whole.init_density(r1, r2)
    raw0, step0 = whole.save_raw()
    g0 = _planes(raw0, storage, NZ)

    half = NZ // 2
    nze = half + 2 * HALO
    offsets = (0, half)                          # first global plane owned by each slab
    glob = [[(z0 - HALO + e) % NZ for e in range(nze)] for z0 in offsets]   # extended plane -> global plane
    slabs = []
    for k, z0 in enumerate(offsets):
        lat = fm.Lattice(_params(fm, nze, storage, kT, flags))
        # extended site s holds global site s + (z0 - HALO) * NX * NY on the slab's own planes
        lat.set_counter_offset(((z0 - HALO) * NX * NY) % 2 ** 32)
        ext = np.ascontiguousarray(g0[:, glob[k], :])
        lat.load_raw(ext.view(np.uint8).reshape(-1), step0)
        slabs.append(lat)

    steps = 8
    for _ in range(steps):
        whole.step(1)
        for lat in slabs:
            lat.step(1)
        raws = [_planes(lat.save_raw()[0].copy(), storage, nze) for lat in slabs]
        own = {}                                 # global plane -> (slab, extended plane) of its owner
        for k, z0 in enumerate(offsets):
            for e in range(HALO, HALO + half):
                own[glob[k][e]] = (k, e)
        for k, lat in enumerate(slabs):
            ext = raws[k].copy()
            for e in list(range(HALO)) + list(range(HALO + half, nze)):
                ok, oe = own[glob[k][e]]
                ext[:, e, :] = raws[ok][:, oe, :]
            lat.load_raw(np.ascontiguousarray(ext).view(np.uint8).reshape(-1), whole.step_count)

    want = _planes(whole.save_raw()[0], storage, NZ)
    for k, z0 in enumerate(offsets):
        got = _planes(slabs[k].save_raw()[0], storage, nze)[:, HALO:HALO + half, :]
        assert np.array_equal(got, want[:, z0:z0 + half, :]), (storage, k)
    whole.close()
    for lat in slabs:
        lat.close()


def test_counter_offset_range_and_default(fm):
    """Offsets outside [0, 2^32) are rejected; offset 0 (the default) leaves
    a run unchanged, and a nonzero offset changes the noise and nothing else
    (with the noise off the bits are the same)."""
    lat = fm.Lattice(_params(fm, 4, "f32"))
    lat.set_counter_offset(0)
    lat.set_counter_offset(2 ** 32 - 1)
    for bad in (-1, 2 ** 32):
        with pytest.raises(fm.FmlbError) as e:
            lat.set_counter_offset(bad)
        assert e.value.status == fm.FMLB_E_INVALID
    lat.close()
    runs = {}
    for kT, off in ((1e-4, 0), (1e-4, None), (1e-4, 12345), (0.0, 0), (0.0, 12345)):
        g = fm.Lattice(_params(fm, 6, "f32", kT))
        if off is not None:
            g.set_counter_offset(off)
        g.init_density(1.0, 0.9)
        g.step(3)
        runs[(kT, off)] = g.save_raw()[0]
        g.close()
    assert np.array_equal(runs[(1e-4, 0)], runs[(1e-4, None)])
    assert not np.array_equal(runs[(1e-4, 0)], runs[(1e-4, 12345)])
    assert np.array_equal(runs[(0.0, 0)], runs[(0.0, 12345)])


def test_one_halo_plane_is_not_enough(fm):
    """With a single halo plane per side the densities of that plane are
    pulled from beyond the slab (here: the far halo after the wrap), so the
    slab's boundary planes go wrong after the first step."""
    import workloads
    _say("case two z-slabs, one halo plane")
    storage, halo = "f64", 1
    r1, r2 = workloads.initial_density((NZ, NY, NX), "perturbed", seed=12, amplitude=0.05)
    whole = fm.Lattice(_params(fm, NZ, storage))
    whole.init_density(r1, r2)
    raw0, step0 = whole.save_raw()
    g0 = _planes(raw0, storage, NZ)
    half = NZ // 2
    nze = half + 2 * halo
    glob = [(0 - halo + e) % NZ for e in range(nze)]
    lat = fm.Lattice(_params(fm, nze, storage))
    lat.load_raw(np.ascontiguousarray(g0[:, glob, :]).view(np.uint8).reshape(-1), step0)
    whole.step(1)
    lat.step(1)
    want = _planes(whole.save_raw()[0], storage, NZ)[:, 0:half, :]
    got = _planes(lat.save_raw()[0], storage, nze)[:, halo:halo + half, :]
    assert not np.array_equal(got[:, 0, :], want[:, 0, :])
    assert np.array_equal(got[:, 2:half - 2, :], want[:, 2:half - 2, :])
    whole.close()
    lat.close()
