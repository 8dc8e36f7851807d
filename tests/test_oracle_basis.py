"""Pins of the oracle's lattices and mode bases against the paper.

- D2Q9 modes and norms against Table I as printed (golden fixture);
- isotropy relations of Eq. (77) and the discrete orthogonality and
  completeness of Eq. (79), in exact rational arithmetic;
- D3Q19 modes 0..9 against the Hermite modes of Eq. (26);
- m_eq of Table I and the projections of the second-order forcing of Eq. (31)
  through one deterministic step of the oracle on tiny lattices.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_d2q9.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, T, N, meq = [t.strip() for t in line.split("|")]
            rows.append((int(a), T, Fraction(N), meq))
    return rows


def _frac(x):
    return Fraction(x).limit_denominator(1000)


def test_d2q9_matches_table1(orc):
    c, w, T, N, D = orc.basis(orc.D2Q9)
    assert D == 2 and T.shape == (9, 9)
    for a, expr, Na, _ in _table1():
        for i in range(9):
            cx, cy = int(c[i, 0]), int(c[i, 1])
            val = eval(expr, {}, dict(cx=cx, cy=cy, c2=cx * cx + cy * cy))
            assert T[a, i] == val, (a, i)
        assert _frac(N[a]) == Na, a


@pytest.mark.parametrize("lattice,Q", [(0, 9), (1, 19)])
def test_isotropy_eq77(orc, lattice, Q):
    c, w, T, N, D = orc.basis(lattice)
    wf = [_frac(x) for x in w]
    assert abs(sum(w) - 1.0) < 1e-15
    cs2 = Fraction(1, 3)
    # second order: sum w c_a c_b = c_s^2 delta
    for al in range(D):
        for be in range(D):
            s = sum(wf[i] * int(c[i, al]) * int(c[i, be]) for i in range(Q))
            assert s == (cs2 if al == be else 0)
    # fourth order: sum w c_a c_b c_g c_d = c_s^4 (dd + dd + dd)
    for idx in np.ndindex(*(D,) * 4):
        a, b, g, d = idx
        s = sum(wf[i] * int(c[i, a]) * int(c[i, b]) * int(c[i, g]) * int(c[i, d]) for i in range(Q))
        expect = cs2 ** 2 * ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
        assert s == expect, idx
    # odd moments vanish
    for al in range(D):
        assert sum(wf[i] * int(c[i, al]) for i in range(Q)) == 0


@pytest.mark.parametrize("lattice,Q", [(0, 9), (1, 19)])
def test_orthogonality_completeness_eq79(orc, lattice, Q):
    c, w, T, N, D = orc.basis(lattice)
    wf = [_frac(x) for x in w]
    Tf = [[_frac(T[a, i]) for i in range(Q)] for a in range(Q)]
    Nf = []
    for a in range(Q):
        for b in range(Q):
            s = sum(wf[i] * Tf[a][i] * Tf[b][i] for i in range(Q))
            if a == b:
                Nf.append(s)
                assert _frac(N[a]) == s
            else:
                assert s == 0, (a, b)
    for i in range(Q):
        for j in range(Q):
            s = wf[i] * sum(Tf[a][i] * Tf[a][j] / Nf[a] for a in range(Q))
            assert s == (1 if i == j else 0), (i, j)


def test_d3q19_hermite_modes_eq26(orc):
    c, w, T, N, D = orc.basis(orc.D3Q19)
    assert D == 3
    third = Fraction(1, 3)
    # theta index after Eq. (25): xx, yy, zz, xy, yz, xz for D = 3
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    for i in range(19):
        ci = [int(v) for v in c[i]]
        assert T[0, i] == 1
        for al in range(3):
            assert T[1 + al, i] == ci[al]
        for k, (al, be) in enumerate(pairs):
            assert _frac(T[4 + k, i]) == ci[al] * ci[be] - (third if al == be else 0)
    # N_theta = c_s^4 (1 + delta) (after Eq. (27))
    for k, (al, be) in enumerate(pairs):
        assert _frac(N[4 + k]) == Fraction(1, 9) * (2 if al == be else 1)


def _one_step_modes(orc, lattice, f_pre, G=0.0, tau=(1.0, 1.0), tau_d=1.0, shape=(1, 1, 1),
                    site=0):
    nz, ny, nx = shape
    p = orc.Params(lattice=lattice, nx=nx, ny=ny, nz=nz, tau=tau, tau_d=tau_d, G=G, kT=0.0)
    s = orc.Sim(p)
    s.set_populations(f_pre)
    fstar = s.collide_site(site)
    return s, fstar


def test_meq_table1_single_site(orc):
    """On a 1x1 lattice with lambda = 1 and no noise, one collision maps the
    transport and ghost modes onto m_eq(rho_sigma, u) with u = v_b_bar (no
    force): Table I's m_eq column."""
    c, w, T, N, D = orc.basis(orc.D2Q9)
    rng = np.random.default_rng(3)
    f = np.empty((2, 9, 1, 1, 1))
    for sp in range(2):
        f[sp, :, 0, 0, 0] = w * (1.0 + 0.3 * rng.uniform(-1, 1, 9))
    rho = f.sum(axis=1)[:, 0, 0, 0]
    j = np.einsum("ia,sixyz->sa", c[:, :2].astype(float), f)
    u = j.sum(0) / rho.sum()
    s, fstar = _one_step_modes(orc, orc.D2Q9, f)
    m_post = fstar @ T.T
    rows = _table1()
    for sp in range(2):
        env = dict(rho=rho[sp], vx=u[0], vy=u[1])
        for a, _, _, meq in rows:
            expect = eval(meq, {}, env)
            assert m_post[sp, a] == pytest.approx(expect, abs=1e-14), (sp, a)


def test_lattice_force_1d_reduction(orc):
    """For a profile varying along x only, Eq. (87) on D2Q9 reduces to
    a(x) = -G/6 [rho'(x+1) - rho'(x-1)] (Sec. VI A)."""
    nx = 7
    G = 0.37
    rng = np.random.default_rng(5)
    r1 = 1.0 + 0.2 * rng.uniform(-1, 1, nx)
    r2 = 1.0 + 0.2 * rng.uniform(-1, 1, nx)
    p = orc.Params(lattice=orc.D2Q9, nx=nx, ny=3, nz=1, G=G)
    s = orc.Sim(p)
    s.init_density(np.broadcast_to(r1, (1, 3, nx)), np.broadcast_to(r2, (1, 3, nx)))
    rho, j, F = s.moments()
    for x in range(nx):
        a1 = -G / 6.0 * (r2[(x + 1) % nx] - r2[(x - 1) % nx])
        a2 = -G / 6.0 * (r1[(x + 1) % nx] - r1[(x - 1) % nx])
        assert F[0, 0, 0, 1, x] == pytest.approx(r1[x] * a1, abs=1e-15)
        assert F[1, 0, 0, 1, x] == pytest.approx(r2[x] * a2, abs=1e-15)
        assert abs(F[0, 1, 0, 1, x]) < 1e-15 and abs(F[1, 1, 0, 1, x]) < 1e-15


def test_forcing_projections_second_order(orc):
    """Projection of the second-order forcing of Eq. (31) onto Table I's
    transport modes, in closed form (derived by hand from Eq. (31) with
    c_s^2 = 1/3): Phi_e = 6 rho a.v, Phi_Pww = 2 rho (a_x v_x - a_y v_y),
    Phi_Pxy = rho (a_x v_y + a_y v_x), Phi = 0 for ghosts, where v is the
    species velocity rho v = j_bar + R_alpha/2 (Eqs. (65), (71)).  With all
    lambda = 1 and no noise one collision gives m*_a = m_eq_a + Phi_a / 2."""
    c, w, T, N, D = orc.basis(orc.D2Q9)
    nx, ny = 5, 4
    G = 0.6
    rng = np.random.default_rng(11)
    f = np.empty((2, 9, 1, ny, nx))
    for sp in range(2):
        f[sp] = w[:, None, None, None] * (1.0 + 0.25 * rng.uniform(-1, 1, (9, 1, ny, nx)))
    p = orc.Params(lattice=orc.D2Q9, nx=nx, ny=ny, nz=1, G=G)
    s = orc.Sim(p)
    s.set_populations(f)
    rho, j, F = s.moments()
    site = 2 + nx * 1
    y, x = 1, 2
    fstar = s.collide_site(site)
    m_post = fstar @ T.T
    r = rho[:, 0, y, x]
    jb = j[:, :, 0, y, x]
    Fs = F[:, :, 0, y, x]
    a = Fs / r[:, None]
    rt = r.sum()
    u = jb.sum(0) / rt + 0.5 * Fs.sum(0) / rt
    for sp in range(2):
        R_mom = (r[sp] * u - jb[sp]) + 0.5 * Fs[sp]
        v = (jb[sp] + 0.5 * R_mom) / r[sp]
        meq = [3 * r[sp] * (u @ u), r[sp] * (u[0] ** 2 - u[1] ** 2), r[sp] * u[0] * u[1], 0, 0, 0]
        phi = [6 * r[sp] * (a[sp] @ v), 2 * r[sp] * (a[sp, 0] * v[0] - a[sp, 1] * v[1]),
               r[sp] * (a[sp, 0] * v[1] + a[sp, 1] * v[0]), 0, 0, 0]
        for k, mode in enumerate(range(3, 9)):
            assert m_post[sp, mode] == pytest.approx(meq[k] + 0.5 * phi[k], abs=1e-14), (sp, mode)
        # momentum: m*_alpha = j_bar + R_alpha = rho u + F/2 when lambda_d = 1
        assert m_post[sp, 1:3] == pytest.approx(r[sp] * u + 0.5 * Fs[sp], abs=1e-14)
        assert m_post[sp, 0] == pytest.approx(r[sp], abs=1e-14)
