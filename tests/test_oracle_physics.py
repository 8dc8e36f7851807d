"""Pins of the oracle's time stepping against what the paper and the
mathematics fix.

Invariants: mass of each species and total momentum conserved to roundoff
(R_0 = 0, Sec. V A; opposite momentum noise and common lambda_d, Eqs. (37),
(74); the i / -i terms of Eq. (87) cancel on a periodic lattice).
Special cases: the uniform rest state without noise is stationary; a 1x1
lattice turns every mode into an AR(1) process whose stationary variance the
noise amplitude of Eq. (74) fixes; textbook shear-wave decay with
nu = c_s^2 (tau - 1/2).
Closed forms: equipartition <m_a^2> = N_a mu rho0 (Eq. (50)); ideal-mixture
structure factors S_rho_rho = k_BT rho0 / c_s^2, S_rho_rho' = 0,
S_jj = k_BT rho0, S_vbvb = k_BT / rho_t0 (Eqs. (55)-(57)).
Lattice linear theory (tests/lyapunov.py): the oracle's linearised step equals
the tool's M(k), and its measured S(k) at G > 0 matches the discrete Lyapunov
solution; its small-k limit is Eq. (57) with alpha = G sin k / k.
Worked values: G_c = 1 for rho_t0 = 2 (Sec. VI A); flat-interface bulk
densities 2.3 / 0.06 and width about 6 at G = 1.5 (Sec. VI B).
"""
import os

import numpy as np
import pytest

from lyapunov import LinearFLBE, eq57, lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def _sim(orc, **kw):
    p = orc.Params(**kw)
    return orc.Sim(p)


def _totals(s):
    rho, j, F = s.moments()
    return rho.reshape(2, -1).sum(1), j.reshape(2, s.D, -1).sum(2).sum(0)


@pytest.mark.parametrize("lattice_id,shape,steps", [(0, (1, 24, 20), 150), (1, (6, 5, 7), 40)])
def test_conservation_roundoff(orc, lattice_id, shape, steps):
    nz, ny, nx = shape
    s = _sim(orc, lattice=lattice_id, nx=nx, ny=ny, nz=nz, tau=(0.8, 1.2), tau_d=0.9, G=0.7,
             kT=1e-4, seed=4)
    rng = np.random.default_rng(0)
    s.init_density(1 + 0.05 * rng.uniform(-1, 1, shape), 1 + 0.05 * rng.uniform(-1, 1, shape))
    m0, J0 = _totals(s)
    s.step(steps)
    m1, J1 = _totals(s)
    scale = m0.sum()
    assert np.all(np.abs(m1 - m0) <= 1e-13 * scale)
    assert np.all(np.abs(J1 - J0) <= 1e-13 * scale)
    assert J0.max() == 0.0


@pytest.mark.parametrize("lattice_id,shape", [(0, (1, 8, 8)), (1, (4, 4, 4))])
def test_rest_state_stationary_without_noise(orc, lattice_id, shape):
    nz, ny, nx = shape
    s = _sim(orc, lattice=lattice_id, nx=nx, ny=ny, nz=nz, tau=(0.7, 1.3), G=0.9, kT=0.0)
    s.init_density(1.3, 0.7)
    f0 = s.populations()
    s.step(100)
    assert np.max(np.abs(s.populations() - f0)) <= 1e-15


@pytest.mark.parametrize("lattice_id", [0, 1])
def test_single_site_ar1_variances(orc, lattice_id):
    """On a 1x1(x1) lattice streaming is the identity and the force vanishes,
    so each non-momentum mode follows m' = (1 - lambda) m + xi with
    <xi^2> = (2 lambda - lambda^2) N_a mu rho (Eq. (74)): stationary variance
    N_a mu rho.  Total momentum stays 0 and j_1 = d relaxes with lambda_d to
    variance k_BT rho rho' / rho_t."""
    kT = 1e-4
    rho = (1.4, 0.6)
    s = _sim(orc, lattice=lattice_id, nx=1, ny=1, nz=1, tau=(0.8, 1.25), tau_d=0.7, kT=kT, seed=3)
    s.init_density(rho[0], rho[1])
    Q = s.Q
    n = 40000
    ms = np.empty((n, 2, Q))
    for t in range(n // 1000):
        for k in range(1000):
            s.step(1)
            ms[t * 1000 + k] = s.mode_moments().reshape(2, Q)
    var = ms[1000:].var(axis=0)
    mu = 3 * kT
    for sp in range(2):
        for a in range(s.D + 1, Q):
            target = s.N[a] * mu * rho[sp]
            assert var[sp, a] == pytest.approx(target, rel=0.05), (sp, a)
        for al in range(s.D):
            assert var[sp, 1 + al] == pytest.approx(kT * rho[0] * rho[1] / sum(rho), rel=0.05)
    assert np.max(np.abs(ms[:, 0, 1:1 + s.D] + ms[:, 1, 1:1 + s.D])) < 1e-13


def test_single_site_deterministic_relaxation(orc):
    """No noise, 1x1 lattice: one step multiplies ghost modes by 1 - lambda."""
    c, w, T, N, D = orc.basis(0)
    rng = np.random.default_rng(2)
    f = np.empty((2, 9, 1, 1, 1))
    for sp in range(2):
        f[sp, :, 0, 0, 0] = w * (1 + 0.2 * rng.uniform(-1, 1, 9))
    s = _sim(orc, lattice=0, nx=1, ny=1, nz=1, tau=(0.8, 1.6), kT=0.0)
    s.set_populations(f)
    m0 = s.mode_moments().reshape(2, 9)
    s.step(1)
    m1 = s.mode_moments().reshape(2, 9)
    for sp, tau in enumerate((0.8, 1.6)):
        lam = 1 / tau
        assert m1[sp, 6:] == pytest.approx((1 - lam) * m0[sp, 6:], abs=1e-15)
        assert m1[sp, 0] == pytest.approx(m0[sp, 0], abs=1e-15)


def _collect(s, burn, snaps, every):
    s.step(burn)
    out = []
    for _ in range(snaps):
        s.step(every)
        out.append(s)
        yield s


@pytest.mark.parametrize("lattice_id,shape", [(0, (1, 32, 32)), (1, (6, 6, 6))])
def test_equipartition(orc, lattice_id, shape):
    """<m_a^2> - <m_a>^2 = N_a mu rho0 for every mode (Eq. (50)), sampled from
    the stored (barred) populations after burn-in (C0 physics)."""
    nz, ny, nx = shape
    kT = 1e-4
    s = _sim(orc, lattice=lattice_id, nx=nx, ny=ny, nz=nz, kT=kT, seed=1)
    s.init_density(1.0, 1.0)
    Q = s.Q
    acc = np.zeros((2, Q))
    acc2 = np.zeros((2, Q))
    n = 0
    for snap in _collect(s, 200, 400, 1):
        m = snap.mode_moments().reshape(2, Q, -1)
        acc += m.mean(2)
        acc2 += (m ** 2).mean(2)
        n += 1
    var = acc2 / n - (acc / n) ** 2
    ratio = var / (s.N * 3 * kT * 1.0)
    assert np.all(np.abs(ratio - 1) < 0.03), ratio


def test_ideal_structure_factors(orc):
    """G = 0 (C0 physics on 32x32): S_rho_rho = 3 k_BT rho0 at every k,
    S_rho1rho2 = 0, S_jj = k_BT rho0, S_vbvb = k_BT / rho_t0 (Eqs. (55)-(57))."""
    kT = 1e-4
    s = _sim(orc, lattice=0, nx=32, ny=32, nz=1, kT=kT, seed=1)
    s.init_density(1.0, 1.0)
    acc = {k: 0.0 for k in ("11", "22", "12", "jj", "vb")}
    n = 0
    for snap in _collect(s, 300, 500, 2):
        rho, j, F = snap.moments()
        acc["11"] = acc["11"] + orc.structure_factor(rho[0, 0], rho[0, 0])
        acc["22"] = acc["22"] + orc.structure_factor(rho[1, 0], rho[1, 0])
        acc["12"] = acc["12"] + orc.structure_factor(rho[0, 0], rho[1, 0])
        acc["jj"] = acc["jj"] + 0.5 * sum(orc.structure_factor(j[0, a, 0]) for a in range(2))
        vb = (j[0] + j[1] + 0.5 * (F[0] + F[1])) / (rho[0] + rho[1])
        acc["vb"] = acc["vb"] + 0.5 * sum(orc.structure_factor(vb[a, 0]) for a in range(2))
        n += 1
    S = {k: v / n for k, v in acc.items()}
    mask = np.ones((32, 32), bool)
    mask[0, 0] = False
    target = {"11": 3 * kT, "22": 3 * kT, "jj": kT, "vb": kT / 2}
    for key, t in target.items():
        assert S[key][mask].mean() == pytest.approx(t, rel=0.02), key
        # flat: quadrant averages agree
        kk = np.fft.fftfreq(32)
        kmag = np.sqrt(kk[:, None] ** 2 + kk[None, :] ** 2)
        for lo, hi in ((0.0, 0.25), (0.25, 0.5), (0.5, 0.75)):
            sel = mask & (kmag > lo) & (kmag <= hi)
            assert S[key][sel].mean() == pytest.approx(t, rel=0.06), (key, lo)
    assert abs(S["12"][mask].mean()) < 0.02 * 3 * kT


def _k_grid(shape):
    ks = [2 * np.pi * np.fft.fftfreq(n) for n in shape]
    return np.meshgrid(*ks, indexing="ij")


@pytest.mark.parametrize("lattice_id,dims", [(0, 2), (1, 3)])
def test_linear_step_matches_lyapunov_operator(orc, lattice_id, dims):
    """Deterministic step of a small-amplitude Fourier mode equals M(k) x."""
    name = "d2q9" if lattice_id == 0 else "d3q19"
    cl, wl = lattice(name)
    oc, ow, oT, oN, D = orc.basis(lattice_id)
    Q = len(ow)
    perm = [[tuple(cl[j].astype(int)) for j in range(Q)].index(tuple(int(v) for v in oc[i, :dims]))
            for i in range(Q)]
    shape = (1, 1, 12) if dims == 2 else (4, 1, 12)
    nz, ny, nx = shape
    G, tau, tau_d = 0.55, (0.8, 1.3), 0.9
    eps = 1e-7
    for kvec in ([2 * np.pi / 12, 0.0, 0.0], [2 * np.pi * 5 / 12, 0.0, np.pi / 2]):
        kx, ky, kz = kvec
        L = LinearFLBE(name, G=G, kT=0.0, tau=tau, tau_d=tau_d)
        kk = [kx, ky] if dims == 2 else [kx, ky, kz]
        if dims == 2 and kz != 0:
            continue
        M, _ = L.operators(kk)
        rng = np.random.default_rng(1)
        v = rng.normal(size=2 * Q) + 1j * rng.normal(size=2 * Q)
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ph = np.exp(1j * (kx * x + ky * y + kz * z))
        f = np.zeros((2, Q, nz, ny, nx))
        for sp in range(2):
            for i in range(Q):
                f[sp, i] = ow[i] + eps * np.real(v[sp * Q + perm[i]] * ph)
        s = _sim(orc, lattice=lattice_id, nx=nx, ny=ny, nz=nz, G=G, tau=tau, tau_d=tau_d, kT=0.0)
        s.set_populations(f)
        s.step(1)
        v2 = M @ v
        pred = np.zeros_like(f)
        for sp in range(2):
            for i in range(Q):
                pred[sp, i] = ow[i] + eps * np.real(v2[sp * Q + perm[i]] * ph)
        assert np.max(np.abs(s.populations() - pred)) < 1e-4 * eps


def test_nonideal_structure_factors_vs_lattice_theory(orc):
    """C1 physics (G = 0.5, tau = 0.8 / 1.2, k_BT = 1e-5) on 32x32: measured
    S_rho_rho, S_rho_rho', S_vbvb against the discrete Lyapunov solution,
    averaged over k bands (statistical tolerance)."""
    kT = 1e-5
    G = 0.5
    n = 32
    s = _sim(orc, lattice=0, nx=n, ny=n, nz=1, G=G, tau=(0.8, 1.2), tau_d=1.0, kT=kT, seed=1)
    s.init_density(1.0, 1.0)
    acc = {k: 0.0 for k in ("11", "22", "12", "vb")}
    cnt = 0
    for snap in _collect(s, 3000, 600, 3):
        rho, j, F = snap.moments()
        acc["11"] = acc["11"] + orc.structure_factor(rho[0, 0])
        acc["22"] = acc["22"] + orc.structure_factor(rho[1, 0])
        acc["12"] = acc["12"] + orc.structure_factor(rho[0, 0], rho[1, 0])
        vb = (j[0] + j[1] + 0.5 * (F[0] + F[1])) / (rho[0] + rho[1])
        acc["vb"] = acc["vb"] + 0.5 * sum(orc.structure_factor(vb[a, 0]) for a in range(2))
        cnt += 1
    S = {k: v / cnt for k, v in acc.items()}
    L = LinearFLBE("d2q9", G=G, kT=kT, tau=(0.8, 1.2), tau_d=1.0)
    KY, KX = _k_grid((n, n))
    th = {k: np.zeros((n, n)) for k in ("11", "22", "12", "vb")}
    mask = np.zeros((n, n), bool)
    for iy in range(n):
        for ix in range(n):
            ky, kx = KY[iy, ix], KX[iy, ix]
            if (ix == 0 and iy == 0) or abs(abs(kx) - np.pi) < 1e-12 or abs(abs(ky) - np.pi) < 1e-12:
                continue
            if kx < 0 or (kx == 0 and ky < 0):   # use the half plane; S(-k) = S(k)
                continue
            t = L.structure_factors([kx, ky])
            th["11"][iy, ix], th["22"][iy, ix] = t["rho1rho1"], t["rho2rho2"]
            th["12"][iy, ix], th["vb"][iy, ix] = t["rho1rho2"], t["vbvb"]
            mask[iy, ix] = True
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    for lo, hi in ((0.0, 1.2), (1.2, 2.4), (2.4, 4.5)):
        sel = mask & (kmag > lo) & (kmag <= hi)
        for key in ("11", "22", "vb"):
            meas = (S[key][sel] + S[key][(-np.argwhere(sel)[:, 0]) % n, (-np.argwhere(sel)[:, 1]) % n]).mean() / 2
            assert meas == pytest.approx(th[key][sel].mean(), rel=0.04), (key, lo)
        d12 = S["12"][sel].mean() - th["12"][sel].mean()
        assert abs(d12) < 0.04 * th["11"][sel].mean(), lo
    # the lattice theory tends to Eq. (57) with alpha = G sin k/k at small k
    a, b = eq57(0.05, G, kT)
    t = L.structure_factors([0.05, 0.0])
    assert t["rho1rho1"] == pytest.approx(a, rel=2e-3)
    assert t["rho1rho2"] == pytest.approx(b, rel=2e-3)


def test_no_sdf_breaks_cross_correlation(orc):
    """Without momentum noise (Sec. VI A, "no-sdf") the ideal mixture no longer
    reaches S_rho_rho' = 0: measured and predicted by the linear theory."""
    kT = 1e-4
    n = 32
    s = _sim(orc, lattice=0, nx=n, ny=n, nz=1, kT=kT, seed=2, flags=orc.NOISE_NO_SDF)
    s.init_density(1.0, 1.0)
    acc12 = 0.0
    cnt = 0
    for snap in _collect(s, 600, 300, 2):
        rho, j, F = snap.moments()
        acc12 = acc12 + orc.structure_factor(rho[0, 0], rho[1, 0])
        cnt += 1
    S12 = acc12 / cnt
    L = LinearFLBE("d2q9", G=0.0, kT=kT, sdf=False)
    k = 2 * np.pi * 8 / n
    t = L.structure_factors([k, 0.0])
    assert t["rho1rho2"] > 0.1 * 3 * kT     # theory: clearly non-zero
    meas = 0.5 * (S12[0, 8] + S12[0, n - 8])
    assert meas == pytest.approx(t["rho1rho2"], rel=0.25)


def test_critical_coupling(orc):
    """G_c = 1 at rho0 = rho0' = 1 (Sec. VI A): the longest wave of a 64-site
    box decays for G = 0.95 and grows for G = 1.05 in the deterministic
    scheme, at the rate the linear theory gives."""
    gold = _golden("critical_coupling.txt")
    n = 64
    k = 2 * np.pi / n
    for G, grows in ((gold["G_c"] - 0.05, False), (gold["G_c"] + 0.05, True)):
        L = LinearFLBE("d2q9", G=G, kT=0.0)
        assert (L.spectral_radius([k, 0.0]) > 1.0) == grows
        s = _sim(orc, lattice=0, nx=n, ny=1, nz=1, G=G, kT=0.0)
        x = np.arange(n)
        d = 1e-6 * np.cos(k * x)
        s.init_density((1 + d).reshape(1, 1, n), (1 - d).reshape(1, 1, n))
        s.step(3000)
        r = s.moments()[0][0, 0, 0]
        a0 = np.abs(np.fft.fft(r - r.mean())[1])
        s.step(2000)
        r = s.moments()[0][0, 0, 0]
        a1 = np.abs(np.fft.fft(r - r.mean())[1])
        rate = (a1 / a0) ** (1 / 2000)
        ev = L.eigenvalues([k, 0.0])
        lead = np.max(np.abs(ev))
        assert (a1 > a0) == grows
        assert rate == pytest.approx(lead, abs=2e-6)


def test_shear_wave_viscosity(orc):
    """Deterministic shear wave u_y(x) = A sin(kx): its amplitude decays as
    exp(-nu k^2 t) with nu = c_s^2 (tau - 1/2), the textbook LB viscosity."""
    n = 64
    tau = 0.9
    s = _sim(orc, lattice=0, nx=n, ny=1, nz=1, tau=(tau, tau), tau_d=tau, kT=0.0)
    c, w, T, N, D = orc.basis(0)
    k = 2 * np.pi / n
    A = 1e-5
    x = np.arange(n)
    uy = A * np.sin(k * x)
    f = np.empty((2, 9, 1, 1, n))
    for sp in range(2):
        for i in range(9):
            f[sp, i, 0, 0] = w[i] * (1 + 3 * c[i, 1] * uy)
    s.set_populations(f)
    s.step(50)
    amp0 = np.abs(np.fft.fft(s.moments()[1][:, 1, 0, 0].sum(0))[1])
    t = 400
    s.step(t)
    amp1 = np.abs(np.fft.fft(s.moments()[1][:, 1, 0, 0].sum(0))[1])
    nu = (tau - 0.5) / 3
    assert amp1 / amp0 == pytest.approx(np.exp(-nu * k * k * t), rel=2e-3)


def test_flat_interface_g15(orc):
    """Sec. VI B: G = 1.5, all lambda = 1: bulk densities 2.3 / 0.06 (two
    significant digits as printed) and an interface about 6 sites wide."""
    import workloads
    gold = _golden("interface_g15.txt")
    n = 100
    r1, r2 = workloads.stripe_density(n, 1, 50, gold["rho_dense"], gold["rho_light"])
    s = _sim(orc, lattice=0, nx=n, ny=1, nz=1, G=gold["G"], kT=0.0)
    s.init_density(r1, r2)
    s.step(15000)
    rho = s.moments()[0][:, 0, 0]
    dense, light = rho[0, n // 2], rho[1, n // 2]
    assert float(f"{dense:.2g}") == gold["rho_dense"]
    assert float(f"{light:.1g}") == gold["rho_light"]
    assert rho[1, 0] == pytest.approx(dense, rel=1e-6) and rho[0, 0] == pytest.approx(light, rel=1e-6)
    # width: sites over which rho_1 goes from 1 % to 99 % of the jump
    prof = rho[0, : n // 2]
    frac = (prof - light) / (dense - light)
    inside = np.where((frac > 0.01) & (frac < 0.99))[0]
    width = inside.max() - inside.min() + 1
    assert abs(width - gold["width"]) <= 2


def _flat_interface(orc, lattice_id, n, width, ny=1, nz=1, steps=20000):
    import workloads
    gold = _golden("interface_g15.txt")
    r1, r2 = workloads.stripe_density(n, ny * nz, width, gold["rho_dense"], gold["rho_light"])
    shape = (nz, ny, n)
    s = _sim(orc, lattice=lattice_id, nx=n, ny=ny, nz=nz, G=gold["G"], kT=0.0)
    s.init_density(r1.reshape(shape), r2.reshape(shape))
    s.step(steps)
    return s, gold["G"]


def _pair_virial(s, G):
    """Volume-summed pair-force virial sum_pairs r_ij (x) f_ij of the lattice
    force of Eq. (87): species 1 at r and species 2 at r + c_i interact with
    the force -G w_i c_i rho_1(r) rho_2(r + c_i) on the first and its
    opposite on the second, so the virial is G sum_r sum_i w_i c_i c_i
    rho_1(r) rho_2(r + c_i) (a D x D tensor)."""
    rho = s.moments()[0]
    V = np.zeros((3, 3))
    for i in range(s.Q):
        shifted = np.roll(rho[1], shift=(-s.c[i, 2], -s.c[i, 1], -s.c[i, 0]), axis=(0, 1, 2))
        V += G * s.w[i] * np.outer(s.c[i], s.c[i]) * np.sum(rho[0] * shifted)
    return V, rho


def test_flat_interface_mechanical_surface_tension(orc):
    """Mechanical surface tension of the flat G = 1.5 interface of Sec. VI B
    (the 100-site box with a 50-site stripe, the capillary run's geometry):
    gamma = sum_x (P_N - P_T) / 2 over the box's two interfaces, with the
    pressure tensor of the pair force of Eq. (87) (its virial) plus the
    kinetic stress sum_i f_i c_i c_i.  Pins: (1) in a uniform phase the
    virial is c_s^2 G rho_1 rho_2 per site, so with the isotropic kinetic
    stress the bulk pressure is c_s^2 (rho_1 + rho_2 + G rho_1 rho_2); the
    two coexisting phases have the same pressure (mechanical equilibrium);
    (2) the kinetic stress of the steady interface is isotropic, so gamma is
    the virial's anisotropy alone; (3) D3Q19 gives the same interface and the
    same gamma (the force's projection on the normal, sum over c_x = +-1 of
    w_i, is 1/6 on both lattices).  Measured: gamma = 0.1614 at bulk densities
    2.350 / 0.0620; the paper quotes 0.174 from a Laplace experiment whose
    radii and fit it does not give."""
    cs2 = 1.0 / 3.0
    gam = {}
    for lattice_id, ny, nz in ((0, 1, 1), (1, 2, 2)):
        s, G = _flat_interface(orc, lattice_id, 100, 50, ny=ny, nz=nz)
        V, rho = _pair_virial(s, G)
        n_sites = s.nsites
        # (2) kinetic stress: isotropic in the plane of the interface and normal to it
        f = s.populations().reshape(2, s.Q, -1)
        K = np.einsum("ia,ib,sin->ab", s.c.astype(float), s.c.astype(float), f)
        assert abs(K[0, 0] - K[1, 1]) <= 1e-8 * K[0, 0]
        gam[lattice_id] = (V[0, 0] - V[1, 1]) / 2 / (n_sites / 100)  # per unit interface length
        # (1) bulk pressures from the closed form are equal on both sides; the
        # virial per site in the middle of a phase matches c_s^2 G rho_1 rho_2
        r1, r2 = rho[0].reshape(-1, 100)[0], rho[1].reshape(-1, 100)[0]
        p = cs2 * (r1 + r2 + G * r1 * r2)
        assert p[50] == pytest.approx(p[0], rel=1e-9)
        local = sum(G * s.w[i] * s.c[i, 1] ** 2 * r1[50] * np.roll(r2, -s.c[i, 0])[50] for i in range(s.Q))
        assert local == pytest.approx(cs2 * G * r1[50] * r2[50], rel=1e-9)
    assert gam[0] == pytest.approx(gam[1], rel=1e-6)
    assert gam[0] == pytest.approx(0.1614, abs=5e-4)
    # against the paper's Laplace value: within 10 % (7.3 % below it)
    assert gam[0] == pytest.approx(0.174, rel=0.10)
