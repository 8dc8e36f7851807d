"""GPU checks of the batched-replica path through the C ABI.

A batch runs many D2Q9 FP32 lattices with one launch per step.  Each replica
must evolve bit for bit as the same lattice stepped alone (same per-tile code,
own seed and site numbering), whatever the work-list shape and whether the
steps come from a replayed HIP graph or direct launches; and it must agree
with the FP64 oracle to the FP32 bound of the single-lattice parity tests.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (nx, ny, tau, tau_d, G, kT, seed): ragged widths, a 1x1 lattice, one wider
# than the widest tile, and differing physics per replica.
REPLICAS = [
    (32, 32, (1.0, 1.0), 1.0, 0.0, 1e-4, 11),
    (40, 37, (0.8, 1.2), 1.0, 0.5, 1e-5, 12),
    (100, 64, (0.9, 1.1), 0.95, 0.85, 3e-5, 13),
    (64, 130, (1.0, 1.0), 1.0, 0.3, 1e-6, 14),
    (1, 1, (0.9, 1.4), 0.8, 0.5, 1e-3, 15),
    (300, 9, (1.0, 1.0), 1.0, 0.95, 1e-4, 16),
    (17, 5, (0.7, 1.3), 1.0, 0.2, 0.0, 17),
]


@pytest.fixture(scope="module")
def fm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1410_5584_amd as fm
    fm.lib()
    return fm


def _say(*a):
    print(*a, flush=True)


def _params(fm, reps=REPLICAS):
    return [fm.Params(lattice="d2q9", storage="f32", nx=nx, ny=ny, nz=1, tau=tau, tau_d=td, G=G, kT=kT, seed=seed)
            for nx, ny, tau, td, G, kT, seed in reps]


def _densities(p, r):
    import workloads
    return workloads.initial_density((1, p.ny, p.nx), "perturbed", seed=100 + r, amplitude=0.05)


def _batch(fm, reps=REPLICAS):
    ps = _params(fm, reps)
    b = fm.Batch(ps)
    for r, p in enumerate(ps):
        b.init_density(r, *_densities(p, r))
    return b, ps


def test_batch_equals_single_lattices(fm):
    _say("case batch vs single lattices, 7 replicas, 9 steps")
    b, ps = _batch(fm)
    assert b.total_sites == sum(p.nx * p.ny for p in ps)
    b.step(9)
    assert b.step_count == 9
    for r, p in enumerate(ps):
        lat = fm.Lattice(p)
        lat.init_density(*_densities(p, r))
        lat.step(9)
        single = lat.populations()
        lat.close()
        got = b.populations(r)
        assert np.array_equal(got, single), (r, float(np.max(np.abs(got - single))))
    b.close()


def test_batch_against_oracle(fm, orc):
    """Two replicas against the FP64 oracle after 20 steps: FP32 bound as in
    the single-lattice parity tests (2e-5 relative)."""
    _say("case batch vs oracle, 20 steps")
    reps = [REPLICAS[1], REPLICAS[2]]
    b, ps = _batch(fm, reps)
    b.step(20)
    for r, p in enumerate(ps):
        o = orc.Sim(orc.Params(lattice=0, nx=p.nx, ny=p.ny, nz=1, tau=p.tau, tau_d=p.tau_d, G=p.G, kT=p.kT,
                               seed=p.seed))
        o.init_density(*_densities(p, r))
        o.step(20)
        want = o.populations()
        err = float(np.max(np.abs(b.populations(r) - want)) / np.max(np.abs(want)))
        _say("replica", r, "max rel diff", err)
        assert err <= 2e-5
    b.close()


def test_full_size_c4_sampled(fm, orc):
    """The benchmark's batched workload at full size: 512 replicas (sizes
    32^2..256^2, per-replica seed, k_BT and G), work list autotuned, steps
    from one replayed 32-step HIP graph, as the benchmark times them.  Five
    replicas (the smallest, the largest and three drawn with a fixed seed)
    are stepped alone by the FP64 oracle and compared site by site, to the
    FP32 bound of the single-lattice parity tests (2e-5 relative)."""
    import workloads
    reps = workloads.replica_table(512)
    ps = [fm.Params(lattice="d2q9", storage="f32", nx=r["L"], ny=r["L"], nz=1, tau=r["tau"], tau_d=r["tau_d"],
                    G=r["G"], kT=r["kT"], seed=r["seed"]) for r in reps]
    sizes = [p.nx for p in ps]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                    *np.random.default_rng(7).choice(len(ps), 3, replace=False).tolist()})
    _say("case c4 full size, 512 replicas, sampled", picks, [sizes[r] for r in picks])
    b = fm.Batch(ps)
    for r in range(len(ps)):
        b.init_density(r, 1.0, 1.0)
    tile = b.autotune(reps=2)
    _say("autotuned tile", tile)
    b.step(32, use_graph=True)
    assert b.step_count == 32
    for r in picks:
        p = ps[r]
        o = orc.Sim(orc.Params(lattice=0, nx=p.nx, ny=p.ny, nz=1, tau=p.tau, tau_d=p.tau_d, G=p.G, kT=p.kT,
                               seed=p.seed))
        o.init_density(1.0, 1.0)
        o.step(32)
        want = o.populations()
        got = b.populations(r)
        err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        _say("replica", r, "L", p.nx, "G", round(p.G, 3), "kT", p.kT, "max rel diff", err)
        assert err <= 2e-5, (r, err)
    b.close()


@pytest.mark.parametrize("tile,march", [(64, 1), (128, 5), (256, 16), (64, 200), (1, 1), (1, 3), (1, 64), (2, 1),
                                        (2, 5)])
def test_batch_work_list_shape_invariance(fm, tile, march):
    _say("case batch tile", tile, march)
    b0, _ = _batch(fm)
    b1, _ = _batch(fm)
    b1.set_tile(tile, march)
    b0.step(6)
    b1.step(6)
    for r in range(len(REPLICAS)):
        assert np.array_equal(b0.populations(r), b1.populations(r)), r
    b0.close()
    b1.close()


@pytest.mark.parametrize("tile", [1, 2])
def test_batch_packed_widths_at_the_limit(fm, tile):
    """Packed sites reach a neighbour 2 nx - 1 sites away (a row end across
    the x wrap, one row up or down): replicas at and beside the widest packed
    width of each block size (128 for 256 threads, 256 for 512), and wider
    ones on the one-row tiles of the same launch, evolve bit for bit as
    alone; so do replicas narrower or shorter than a block."""
    _say("case batch packed widths, tile", tile)
    reps = [(w, 6, (0.9, 1.1), 1.0, 0.6, 1e-4, 40 + k) for k, w in enumerate((127, 128, 129, 200, 255, 256, 257))]
    # and shapes whose runs of sites wrap around the lattice within a block
    reps += [(1, 50, (1.0, 1.0), 1.0, 0.3, 1e-4, 60), (3, 200, (0.8, 1.2), 0.9, 0.5, 1e-5, 61),
             (7, 1, (1.0, 1.0), 1.0, 0.2, 1e-4, 62), (255, 2, (0.9, 1.1), 1.0, 0.7, 1e-4, 63)]
    b, ps = _batch(fm, reps)
    b.set_tile(tile, 3)
    b.step(5)
    for r, p in enumerate(ps):
        lat = fm.Lattice(p)
        lat.init_density(*_densities(p, r))
        lat.step(5)
        single = lat.populations()
        lat.close()
        assert np.array_equal(b.populations(r), single), (r, p.nx)
    b.close()


def test_batch_graph_replays_equal_direct_launches(fm):
    """Graph replays (32 steps each) with direct launches and host reads
    between them give the same bits as direct launches, at every checkpoint."""
    _say("case batch graph vs eager")
    ge, _ = _batch(fm)
    gg, _ = _batch(fm)
    for n in (70, 5, 64, 33):
        ge.step(n, use_graph=False)
        gg.step(n, use_graph=True)
        ge.synchronize()
        gg.synchronize()
        assert gg.step_count == ge.step_count
        for r in range(len(REPLICAS)):
            assert np.array_equal(ge.populations(r), gg.populations(r)), (n, r)
        gg.mode_accumulate()  # other work on the stream between replays
    ge.close()
    gg.close()


def test_batch_observables_match_single(fm):
    _say("case batch observables")
    b, ps = _batch(fm)
    lats = []
    for r, p in enumerate(ps):
        lat = fm.Lattice(p)
        lat.init_density(*_densities(p, r))
        lats.append(lat)
    for _ in range(4):
        b.step(3)
        b.mode_accumulate()
        for lat in lats:
            lat.step(3)
            lat.mode_accumulate()
    for r, (p, lat) in enumerate(zip(ps, lats)):
        gs = b.global_sums(r)
        np.testing.assert_allclose(gs, lat.global_sums(), rtol=1e-12, atol=1e-12 * p.nx * p.ny)
        if p.kT > 0:
            mv, n = b.mode_variances(r)
            ms, ns = lat.mode_variances()
            assert n == ns == 4
            np.testing.assert_allclose(mv, ms, rtol=1e-9, atol=1e-12)
        lat.close()
    b.close()


def test_batch_conserves_mass_and_momentum(fm):
    """Species masses and total momentum over 200 steps.  The stored FP32
    values are deviations from w_i rho_ref and the update is formed for
    them, so rounding acts at the scale of the density perturbations (5 %
    here), not of w_i rho.  Bound: 2^-30 per step, relative (a 2^-24
    rounding of a 2^-5 deviation, with a margin of 2); momentum the same
    per site."""
    _say("case batch conservation, 200 steps")
    steps = 200
    tol = steps * 2.0 ** -30
    b, ps = _batch(fm)
    before = [b.global_sums(r) for r in range(len(ps))]
    b.step(steps, use_graph=True)
    for r, p in enumerate(ps):
        after = b.global_sums(r)
        n = p.nx * p.ny
        _say(f"  replica {r}: relative mass change {(after[:2] - before[r][:2]) / before[r][:2]}")
        np.testing.assert_allclose(after[:2], before[r][:2], rtol=tol)
        assert np.all(np.abs(after[2:] - before[r][2:]) <= tol * n)
    b.close()


def test_batch_rejects_step_before_init(fm):
    ps = _params(fm, REPLICAS[:2])
    b = fm.Batch(ps)
    b.init_density(0, *_densities(ps[0], 0))
    with pytest.raises(fm.FmlbError) as e:
        b.step(1)
    assert e.value.status == fm.FMLB_E_STATE
    with pytest.raises(fm.FmlbError) as e:
        b.set_tile(96, 4)
    assert e.value.status == fm.FMLB_E_INVALID
    b.close()


def test_batch_autotune_leaves_state_and_results_unchanged(fm):
    _say("case batch autotune")
    b0, _ = _batch(fm)
    b1, _ = _batch(fm)
    b0.step(4)
    b1.step(4)
    before = [b1.populations(r) for r in range(len(REPLICAS))]
    tx, march = b1.autotune(reps=2)
    assert tx in (64, 128, 256) and march in (1, 2, 4, 8, 16, 32, 64)
    assert b1.step_count == 4
    for r in range(len(REPLICAS)):
        assert np.array_equal(b1.populations(r), before[r]), r
    b0.step(5)
    b1.step(5, use_graph=True)
    for r in range(len(REPLICAS)):
        assert np.array_equal(b0.populations(r), b1.populations(r)), r
    b0.close()
    b1.close()
