"""Pins of the N-species oracle (the multicomponent model of Apps. C and D).

What fixes it, other than itself:
  - N = 2 is the binary model: the same sample path as the two-species
    oracle, which has its own pins (test_oracle_physics.py);
  - two identical species with half the density each behave as one species
    of the binary model (deterministic case): this exercises the force sum
    over several partners and every species index above 2;
  - on a single site with lambda_d = 1, the momenta after a step are exactly
    the momentum noises, whose covariance App. D fixes: (2 lambda_d -
    lambda_d^2) k_B T (rho_sigma delta - rho_sigma rho_s' / rho_t);
  - mass of every species and total momentum are conserved;
  - the ideal mixture (G = 0) is equipartitioned at every site:
    <j_sigma j_s'> = k_B T rho_sigma delta and <drho_sigma drho_s'> =
    3 k_B T rho_sigma delta (the Gaussian measure of the binary pin, which is
    invariant under the collision exactly when the momentum noise has the
    covariance above).
"""
import numpy as np
import pytest

import oracle
import workloads

D2Q9, D3Q19 = oracle.D2Q9, oracle.D3Q19


def _binary_pair(lattice, shape, flags=0, kT=1e-4):
    nz, ny, nx = shape
    kw = dict(lattice=lattice, nx=nx, ny=ny, nz=nz, tau_d=0.9, kT=kT, seed=5, flags=flags)
    b = oracle.Sim(oracle.Params(tau=(0.8, 1.2), G=0.6, **kw))
    m = oracle.MultiSim(oracle.MultiParams(nspecies=2, tau=(0.8, 1.2), G=((0.0, 0.6), (0.6, 0.0)), **kw))
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=3, amplitude=0.05)
    b.init_density(r1, r2)
    m.init_density([r1, r2])
    return b, m


@pytest.mark.parametrize("lattice,shape,flags", [(D2Q9, (1, 9, 12), 0), (D2Q9, (1, 7, 5), oracle.NOISE_NO_SDF),
                                                 (D3Q19, (4, 5, 6), 0)])
def test_two_species_is_the_binary_model(lattice, shape, flags):
    b, m = _binary_pair(lattice, shape, flags)
    b.step(30)
    m.step(30)
    fb, fm = b.populations(), m.populations()
    assert np.max(np.abs(fb - fm)) <= 1e-13 * np.max(np.abs(fb))


@pytest.mark.parametrize("lattice,shape", [(D2Q9, (1, 10, 14)), (D3Q19, (5, 4, 6))])
def test_identical_species_merge_into_one(lattice, shape):
    """Species 2 and 3 identical (same tau, same coupling G to species 1, no
    coupling to each other), half the binary species-2 density each: with
    k_B T = 0, f_2 + f_3 follows the binary species 2 and f_1 the binary
    species 1."""
    nz, ny, nx = shape
    G = 0.7
    kw = dict(lattice=lattice, nx=nx, ny=ny, nz=nz, tau_d=0.95, kT=0.0, seed=1)
    b = oracle.Sim(oracle.Params(tau=(0.9, 1.3), G=G, **kw))
    m = oracle.MultiSim(oracle.MultiParams(nspecies=3, tau=(0.9, 1.3, 1.3),
                                           G=((0.0, G, G), (G, 0.0, 0.0), (G, 0.0, 0.0)), **kw))
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=8, amplitude=0.1)
    b.init_density(r1, r2)
    m.init_density([r1, 0.5 * r2, 0.5 * r2])
    b.step(40)
    m.step(40)
    fb, fm = b.populations(), m.populations()
    scale = np.max(np.abs(fb))
    assert np.max(np.abs(fm[0] - fb[0])) <= 1e-13 * scale
    assert np.max(np.abs(fm[1] + fm[2] - fb[1])) <= 1e-13 * scale


@pytest.mark.parametrize("rho", [(1.0, 0.7, 0.4), (1.3, 0.5, 0.9, 0.2)])
def test_single_site_momentum_noise_covariance(rho):
    """1 x 1 lattice, G = 0, lambda_d = 1: the post-collision momenta are
    rho_sigma u + xi_sigma with u = 0 (total momentum zero and conserved),
    so the pre-collision j_bar_sigma of each step is the previous step's
    noise.  Sample covariance over 20000 steps against App. D's covariance
    (per component), within 5 standard errors; total momentum zero to
    roundoff at every step."""
    n = len(rho)
    kT = 1e-3
    m = oracle.MultiSim(oracle.MultiParams(nspecies=n, nx=1, ny=1, tau=(1.0,) * n, tau_d=1.0,
                                           G=tuple((0.0,) * n for _ in range(n)), kT=kT, seed=11))
    m.init_density(list(rho))
    steps = 20000
    J = np.zeros((steps, n, 2))
    for t in range(steps):
        m.step(1)
        J[t] = m.moments()[1][:, :, 0, 0, 0]
    assert np.max(np.abs(J.sum(axis=1))) < 1e-13  # roundoff of a conserved sum over 20000 steps
    r = np.asarray(rho)
    C = kT * (np.diag(r) - np.outer(r, r) / r.sum())
    for al in range(2):
        X = J[:, :, al]
        est = X.T @ X / steps
        se = np.sqrt((np.outer(np.diag(C), np.diag(C)) + C ** 2) / steps)
        assert np.all(np.abs(est - C) <= 5 * se + 1e-18), (al, est, C)


@pytest.mark.parametrize("lattice,shape", [(D2Q9, (1, 14, 20)), (D3Q19, (5, 6, 8))])
def test_multi_conservation(lattice, shape):
    nz, ny, nx = shape
    G = ((0.0, 0.4, 0.3), (0.4, 0.0, 0.6), (0.3, 0.6, 0.0))
    m = oracle.MultiSim(oracle.MultiParams(lattice=lattice, nspecies=3, nx=nx, ny=ny, nz=nz, tau=(0.8, 1.1, 1.4),
                                           tau_d=0.9, G=G, kT=1e-4, seed=3))
    r = [workloads.initial_density(shape, "perturbed", seed=s, amplitude=0.05)[0] * f
         for s, f in ((1, 1.0), (2, 0.7), (3, 0.5))]
    m.init_density(r)
    rho0, j0, _ = m.moments()
    m.step(100)
    rho1, j1, _ = m.moments()
    mass0 = rho0.sum(axis=(1, 2, 3))
    assert np.all(np.abs(rho1.sum(axis=(1, 2, 3)) - mass0) <= 1e-13 * mass0)
    P0, P1 = j0.sum(axis=(0, 2, 3, 4)), j1.sum(axis=(0, 2, 3, 4))
    assert np.all(np.abs(P1 - P0) <= 1e-13 * mass0.sum())


def test_ideal_mixture_equipartition():
    """N = 3, G = 0, 16 x 16, k_B T = 1e-4, different tau per species: per
    site, <j_bar_sigma,alpha j_bar_s',alpha> = k_B T rho_sigma delta and the
    mean-subtracted <drho_sigma drho_s'> = 3 k_B T rho_sigma delta (1 - 1/N_sites),
    over 1500 snapshots 4 steps apart; diagonal within 4 %, off-diagonal
    within 4 % of the geometric mean of the diagonal."""
    n, L, kT = 3, 16, 1e-4
    rho = np.array([1.0, 0.6, 0.3])
    m = oracle.MultiSim(oracle.MultiParams(nspecies=n, nx=L, ny=L, tau=(0.8, 1.0, 1.25), tau_d=1.0,
                                           G=((0.0,) * 3,) * 3, kT=kT, seed=21))
    m.init_density(list(rho))
    m.step(200)
    snaps = 1500
    cj = np.zeros((n, n))
    cr = np.zeros((n, n))
    for _ in range(snaps):
        m.step(4)
        r, j, _ = m.moments()
        jj = j.reshape(n, 2, -1)
        for al in range(2):
            cj += jj[:, al] @ jj[:, al].T / jj.shape[-1]
        dr = r.reshape(n, -1) - r.reshape(n, -1).mean(axis=1, keepdims=True)
        cr += dr @ dr.T / dr.shape[-1]
    cj /= 2 * snaps
    cr /= snaps
    want_j = kT * np.diag(rho)
    want_r = 3 * kT * np.diag(rho) * (1 - 1 / L ** 2)
    for est, want in ((cj, want_j), (cr, want_r)):
        d = np.sqrt(np.diag(want))
        assert np.all(np.abs(est - want) <= 0.04 * np.outer(d, d)), (est, want)


def test_four_species_d3q19_conservation():
    """The largest normal count (D3Q19 with four species: 69 normals per site)."""
    G = ((0.0, 0.45, 0.3, 0.2), (0.45, 0.0, 0.6, 0.1), (0.3, 0.6, 0.0, 0.5), (0.2, 0.1, 0.5, 0.0))
    shape = (3, 4, 5)
    m = oracle.MultiSim(oracle.MultiParams(lattice=D3Q19, nspecies=4, nx=5, ny=4, nz=3, tau=(0.8, 1.1, 1.3, 0.9),
                                           tau_d=0.9, G=G, kT=1e-4, seed=4))
    m.init_density([workloads.initial_density(shape, "perturbed", seed=s, amplitude=0.05)[0] for s in range(4)])
    rho0, j0, _ = m.moments()
    m.step(30)
    rho1, j1, _ = m.moments()
    f = m.populations()
    assert np.all(np.isfinite(f))
    mass0 = rho0.sum(axis=(1, 2, 3))
    assert np.all(np.abs(rho1.sum(axis=(1, 2, 3)) - mass0) <= 1e-13 * mass0)
    assert np.all(np.abs(j1.sum(axis=(0, 2, 3, 4)) - j0.sum(axis=(0, 2, 3, 4))) <= 1e-13 * mass0.sum())


def test_multi_linear_theory_two_species_is_the_binary_theory():
    """The N-species linear theory with two species equals the binary one."""
    from lyapunov import LinearFLBE, LinearMultiFLBE
    kw = dict(rho0=(1.0, 0.7), tau=(0.8, 1.2), tau_d=0.9, kT=1e-5)
    b = LinearFLBE("d2q9", G=0.6, **kw)
    m = LinearMultiFLBE("d2q9", G=((0.0, 0.6), (0.6, 0.0)), **kw)
    for k in ([0.3, 0.0], [1.1, 0.4], [2.5, 2.0]):
        sb = b.structure_factors(k)
        S = m.density_structure(k)
        assert S[0, 0] == pytest.approx(sb["rho1rho1"], rel=1e-10)
        assert S[1, 1] == pytest.approx(sb["rho2rho2"], rel=1e-10)
        assert S[0, 1] == pytest.approx(sb["rho1rho2"], rel=1e-9, abs=1e-16)


def test_multi_linear_theory_limits():
    """Three species.  Ideal mixture (G = 0): S_rho rho = 3 k_B T rho_sigma
    delta and S_jj = k_B T rho_sigma delta at every k (App. C with gamma = 0;
    exact on the lattice).  Coupled and miscible (R^-1 + G positive
    definite): S_rho rho(k) tends to App. C/D's mu (R^-1 + alpha)^-1 and
    S_jj to k_B T rho delta at small k (k = 0.05 along x: within 0.05 % and
    0.01 %; at larger k the lattice values differ from the continuum ones,
    as for two species)."""
    from lyapunov import LinearMultiFLBE, appendix_structure_factor
    rho = (1.0, 0.8, 0.6)
    kT = 1e-5
    ideal = LinearMultiFLBE("d2q9", rho0=rho, tau=(0.9, 1.0, 1.2), tau_d=1.0, kT=kT)
    for kk in ([0.4, 0.0], [1.3, 0.7], [2.9, 0.0]):
        assert np.allclose(ideal.density_structure(kk), 3 * kT * np.diag(rho), rtol=1e-9, atol=1e-9 * kT)
        assert np.allclose(ideal.momentum_structure(kk), kT * np.diag(rho), rtol=1e-9, atol=1e-9 * kT)
    G = ((0.0, 0.4, 0.3), (0.4, 0.0, 0.5), (0.3, 0.5, 0.0))
    th = LinearMultiFLBE("d2q9", rho0=rho, tau=(0.9, 1.0, 1.2), tau_d=1.0, G=G, kT=kT)
    k = 0.05
    S = th.density_structure([k, 0.0])
    want = appendix_structure_factor(k, G, rho, kT)
    assert np.max(np.abs(S - want)) <= 5e-4 * np.max(np.abs(want))
    assert abs(want[0, 1]) > 0.1 * want[0, 0]  # the couplings matter at this k
    Sj = th.momentum_structure([k, 0.0])
    assert np.max(np.abs(Sj - kT * np.diag(rho))) <= 1e-4 * kT


def test_multi_collide_site_is_the_step():
    """The single-site collision, streamed, is the next state."""
    shape = (1, 6, 7)
    m = oracle.MultiSim(oracle.MultiParams(nspecies=3, nx=7, ny=6, tau=(0.8, 1.1, 1.3), tau_d=0.9,
                                           G=((0.0, 0.4, 0.3), (0.4, 0.0, 0.6), (0.3, 0.6, 0.0)), kT=1e-4, seed=3))
    m.init_density([workloads.initial_density(shape, "perturbed", seed=s, amplitude=0.05)[0] for s in range(3)])
    m.step(2)
    fs = np.stack([m.collide_site(r) for r in range(m.nsites)], axis=-1)  # [N, Q, sites]
    m.step(1)
    f1 = m.populations().reshape(3, m.Q, -1)
    c = m.c
    for r in range(m.nsites):
        x, y = r % 7, r // 7
        for i in range(m.Q):
            dst = (x + c[i, 0]) % 7 + 7 * ((y + c[i, 1]) % 6)
            assert np.allclose(f1[:, i, dst], fs[:, i, r], rtol=0, atol=1e-15)
