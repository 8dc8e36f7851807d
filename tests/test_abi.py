"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, sizes buffers, and rejects invalid parameters before touching
the GPU.  No compute call is made here."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmlb.h")


@pytest.fixture(scope="module")
def fm():
    import paper_1410_5584_amd as fm
    if not os.path.exists(fm.LIB_PATH):
        from paper_1410_5584_amd import build
        build.build()
    fm.lib()
    return fm


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmlb_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(fm):
    names = _declared()
    assert len(names) >= 30
    out = subprocess.run(["nm", "-D", "--defined-only", fm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\b(fmlb_[a-z0-9_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    for n in names:
        assert n in fm._SIGNATURES, n


def test_required_bytes(fm):
    p = fm.Params(lattice="d3q19", storage="f32", nx=256, ny=256, nz=256)
    n = 256 ** 3
    assert fm.fmlb_required_bytes(p.c(), 0) == 2 * 19 * n * 4
    assert fm.fmlb_required_bytes(p.c(), 1) == 2 * 19 * n * 4
    assert fm.fmlb_required_bytes(p.c(), 2) > 2 * n * 4
    p16 = fm.Params(lattice="d3q19", storage="bf16", nx=256, ny=256, nz=256)
    assert fm.fmlb_required_bytes(p16.c(), 0) == 2 * 19 * n * 2
    p64 = fm.Params(lattice="d2q9", storage="f64", nx=64, ny=64)
    assert fm.fmlb_required_bytes(p64.c(), 0) == 2 * 9 * 64 * 64 * 8


@pytest.mark.parametrize("bad", [
    dict(tau=(0.5, 1.0)), dict(tau=(1.0, 0.4)), dict(tau_d=0.5), dict(kT=-1e-5),
    dict(nx=0), dict(lattice="d2q9", nz=2), dict(G=float("nan")),
    dict(storage="f32", flags=4), dict(storage="f64", flags=4), dict(flags=8),
])
def test_invalid_parameters_rejected(fm, bad):
    p = fm.Params(**bad)
    assert fm.fmlb_required_bytes(p.c(), 0) == 0
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_create(p.c(), 0, [256, 512, 768])
    assert e.value.status == fm.FMLB_E_INVALID


def test_null_and_alignment_errors(fm):
    p = fm.Params()
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_create(p.c(), 0, [0, 512, 768])
    assert e.value.status == fm.FMLB_E_NULL
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_create(p.c(), 0, [256 + 8, 512, 768])
    assert e.value.status == fm.FMLB_E_INVALID
    assert fm.lib().fmlb_status_string(fm.FMLB_E_STATE).decode() == "populations not initialised"


def _rep(fm, **kw):
    d = dict(lattice="d2q9", storage="f32", nx=40, ny=33, kT=1e-5, G=0.3)
    d.update(kw)
    return fm.Params(**d).c()


def test_batch_required_bytes(fm):
    reps = [_rep(fm, nx=40, ny=33), _rep(fm, nx=256, ny=256), _rep(fm, nx=1, ny=1)]
    a = fm.fmlb_batch_required_bytes(reps, 0)
    # each replica block 2 x 9 population arrays of the site count rounded up
    # to 64 floats (every array starts on a 256-byte boundary)
    want = sum(2 * 9 * ((n + 63) // 64) * 64 * 4 for n in (40 * 33, 256 * 256, 1))
    assert a == want
    assert fm.fmlb_batch_required_bytes(reps, 1) == want
    assert fm.fmlb_batch_required_bytes(reps, 2) > 2 * 256 * 256 * 8


@pytest.mark.parametrize("bad", [
    dict(lattice="d3q19", nz=4), dict(storage="f64"), dict(storage="bf16"), dict(nz=2),
    dict(tau=(0.5, 1.0)), dict(kT=-1.0), dict(nx=0), dict(flags=4), dict(flags=8),
])
def test_batch_invalid_replica_rejected(fm, bad):
    reps = [_rep(fm), _rep(fm, **bad)]
    assert fm.fmlb_batch_required_bytes(reps, 0) == 0
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_batch_create(reps, 0, [256, 512, 768])
    assert e.value.status == fm.FMLB_E_INVALID
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_batch_create([_rep(fm)], 0, [256, 0, 768])
    assert e.value.status == fm.FMLB_E_NULL


def test_multi_required_bytes(fm):
    G = ((0.0, 0.3, 0.2), (0.3, 0.0, 0.1), (0.2, 0.1, 0.0))
    p = fm.MultiParams(lattice="d3q19", storage="f32", nspecies=3, nx=64, ny=32, nz=16, G=G)
    n = 64 * 32 * 16
    assert fm.fmlb_multi_required_bytes(p.c(), 0) == 3 * 19 * n * 4
    assert fm.fmlb_multi_required_bytes(p.c(), 1) == 3 * 19 * n * 4
    assert fm.fmlb_multi_required_bytes(p.c(), 2) >= 3 * n * 4 + 4 * n * 8
    p4 = fm.MultiParams(lattice="d2q9", storage="f64", nspecies=4, nx=10, ny=10, tau=(1.0,) * 4,
                        G=tuple((0.0,) * 4 for _ in range(4)))
    assert fm.fmlb_multi_required_bytes(p4.c(), 0) == 4 * 9 * 100 * 8 + (256 - (4 * 9 * 100 * 8) % 256) % 256


@pytest.mark.parametrize("bad", [
    dict(nspecies=1), dict(nspecies=5), dict(storage="bf16"), dict(tau=(1.0, 0.5, 1.0)),
    dict(G=((0.0, 0.3, 0.2), (0.31, 0.0, 0.1), (0.2, 0.1, 0.0))), dict(lattice="d2q9", nz=2), dict(kT=-1.0),
    dict(flags=4), dict(flags=8),
])
def test_multi_invalid_parameters_rejected(fm, bad):
    kw = dict(nspecies=3, G=((0.0, 0.3, 0.2), (0.3, 0.0, 0.1), (0.2, 0.1, 0.0)))
    kw.update(bad)
    if kw["nspecies"] in (1, 5):
        kw["G"] = tuple((0.0,) * 4 for _ in range(4))
    p = fm.MultiParams(**kw)
    for which in range(3):
        assert fm.fmlb_multi_required_bytes(p.c(), which) == 0
    with pytest.raises(fm.FmlbError) as e:
        fm.fmlb_multi_create(p.c(), 0, [256, 512, 768])
    assert e.value.status == fm.FMLB_E_INVALID


def test_multi_set_form_validation(fm):
    """Form selection is host logic: checked without a device (the buffers
    are placeholders that nothing dereferences)."""
    G = ((0.0, 0.3, 0.2), (0.3, 0.0, 0.1), (0.2, 0.1, 0.0))
    ok, bad, unsup = fm.FMLB_OK, fm.FMLB_E_INVALID, fm.FMLB_E_UNSUPPORTED

    def status(m, *args):
        try:
            fm.fmlb_multi_set_form(m, *args)
            return ok
        except fm.FmlbError as e:
            return e.status

    for storage in ("f32", "f64"):
        m = fm.fmlb_multi_create(fm.MultiParams(lattice="d3q19", storage=storage, nspecies=3, nx=64, ny=32, nz=16,
                                                G=G).c(), 0, [256, 512, 768])
        try:
            A, T, F, S = fm.FMLB_MULTI_AUTO, fm.FMLB_MULTI_TWO_PASS, fm.FMLB_MULTI_FUSED, fm.FMLB_MULTI_ASYNC
            assert status(m, A, 0, 0, 0) == ok
            assert status(m, T, 0, 0, 0) == ok
            assert status(m, A, 64, 4, 0) == bad and status(m, T, 0, 0, 8) == bad
            assert status(m, F, 64, 8, 16) == ok and status(m, F, 0, 0, 0) == ok
            assert status(m, F, 32, 4, 0) == bad  # not a register-form tile
            assert status(m, 7, 0, 0, 0) == bad and status(m, -1, 0, 0, 0) == bad
            assert status(m, F, 64, 8, 5000) == bad and status(m, F, 0, 4, 0) == bad
            if storage == "f32":
                for t in ((64, 4, 0), (32, 8, 3), (32, 4, 4096), (0, 0, 0)):
                    assert status(m, S, *t) == ok, t
                # 64x8: its LDS holds two species only
                for t in ((64, 8, 0), (64, 6, 0), (128, 1, 0), (16, 8, 0)):
                    assert status(m, S, *t) == bad, t
            else:
                assert status(m, S, 0, 0, 0) == unsup
            # the shorthand
            fm.fmlb_multi_set_tile(m, 0, 0, 0)
            fm.fmlb_multi_set_tile(m, 1, 0, 0)
            fm.fmlb_multi_set_tile(m, 64, 4, 2)
            for t in ((0, 0, 3), (1, 1, 0), (64, 2, 0)):
                with pytest.raises(fm.FmlbError):
                    fm.fmlb_multi_set_tile(m, *t)
        finally:
            fm.fmlb_multi_destroy(m)


def test_multi_async_tiles_follow_the_lds(fm):
    """64x8 asynchronous tiles fit the LDS with two species, not with three."""
    G2 = ((0.0, 0.3), (0.3, 0.0))
    m = fm.fmlb_multi_create(fm.MultiParams(lattice="d3q19", storage="f32", nspecies=2, nx=64, ny=32, nz=16,
                                            tau=(1.0, 1.0), G=G2, rho_ref=(1.0, 1.0)).c(), 0, [256, 512, 768])
    try:
        fm.fmlb_multi_set_form(m, fm.FMLB_MULTI_ASYNC, 64, 8, 0)
        with pytest.raises(fm.FmlbError):
            fm.fmlb_multi_set_form(m, fm.FMLB_MULTI_ASYNC, 64, 6, 0)
    finally:
        fm.fmlb_multi_destroy(m)
