"""The allocation-free structure-factor accumulation (fmlb_sk_accumulate_static,
work arrays in a static device array of the library) against the context's
fmlb_sk_accumulate on the same state, bit for bit (same kernels, same
summation order), on two calls in a row: a larger lattice first, then a
smaller one, so the second call runs on work arrays that still hold the
first call's data.  Sizes above the static array are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1410_5584_amd as fm
    fm.lib()
    return fm


def _say(*a):
    print(*a, flush=True)


def _compare(fm, torch, lattice, storage, shape, G):
    import workloads
    nz, ny, nx = shape
    _say("case static S(k)", lattice, storage, shape)
    p = fm.Params(lattice=lattice, storage=storage, nx=nx, ny=ny, nz=nz, tau=(0.8, 1.2), tau_d=1.0, G=G,
                  kT=1e-4, seed=3)
    lat = fm.Lattice(p)
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=4, amplitude=0.05)
    lat.init_density(r1, r2)
    lat.step(20)
    lat.reset_accumulators()
    lat.sk_accumulate()
    ref = np.stack([lat.sk(k)[0] for k in range(7)])
    raw, _ = lat.save_raw()
    pops = torch.from_numpy(np.ascontiguousarray(raw).copy()).to("cuda")
    n = nx * ny * nz
    acc = torch.zeros(7 * n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    fm.fmlb_sk_accumulate_static(p.c(), pops.data_ptr(), acc.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    got = acc.cpu().numpy().reshape(7, *shape)
    lat.close()
    assert np.max(np.abs(ref)) > 0
    for k in range(7):
        assert np.array_equal(got[k], ref[k]), k


def test_static_sk_matches_the_context(fm):
    import torch
    _compare(fm, torch, "d2q9", "f64", (1, 96, 128), 0.5)    # 12288 sites
    _compare(fm, torch, "d3q19", "f32", (10, 12, 9), 0.4)    # 1080 sites, after the larger call


def test_static_sk_rejects_oversize(fm):
    import torch
    _say("case static S(k) oversize")
    p = fm.Params(lattice="d2q9", storage="f32", nx=1025, ny=1024)
    assert p.nx * p.ny > fm.SK_STATIC_MAX_SITES
    dummy = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_sk_accumulate_static(p.c(), dummy.data_ptr(), dummy.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert e.value.status == fm.FMLB_E_SIZE
