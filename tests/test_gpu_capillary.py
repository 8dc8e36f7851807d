"""Capillary fluctuations of a liquid-liquid interface (Sec. VI B) on the GPU.

The paper's set-up:
  - D2Q9, G = 1.5, every relaxation rate 1;
  - bulk densities 2.3 / 0.06, interface about 6 sites wide;
  - surface tension 0.174 from a Laplace experiment;
  - a 50 x 512 stripe in a 100 x 512 periodic box at k_BT = 1e-5, whose interface height spectrum
    follows Eq. (91), <|h(k)|^2> = k_BT / (gamma k^2), up to k of about 1.
Here:
  - the Laplace experiment: droplets of several radii, with the mechanical pressure of the model
    p = c_s^2 (rho_1 + rho_2) + c_s^2 G rho_1 rho_2 (the continuum limit of Eq. (87) with
    sum_i w_i c_i c_i = c_s^2 I), gamma from dp = gamma / R;
  - the spectrum of both interfaces of the fluctuating stripe against Eq. (91) with that gamma.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

G = 1.5
DENSE, LIGHT = 2.3, 0.06
CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def fm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1410_5584_amd as fm
    fm.lib()
    return fm


def _say(*a):
    print(*a, flush=True)


def _pressure(r1, r2):
    return CS2 * (r1 + r2) + CS2 * G * r1 * r2


def _laplace_gamma(fm):
    n = 128
    y, x = np.mgrid[0:n, 0:n]
    pts = []
    for R in (12.0, 16.0, 22.0, 30.0):
        inside = (x - n / 2 + 0.5) ** 2 + (y - n / 2 + 0.5) ** 2 < R * R
        r1 = np.where(inside, DENSE, LIGHT)[None]
        r2 = np.where(inside, LIGHT, DENSE)[None]
        lat = fm.Lattice(fm.Params(lattice="d2q9", storage="f64", nx=n, ny=n, tau=(1.0, 1.0), tau_d=1.0, G=G,
                                   kT=0.0, seed=1))
        lat.init_density(r1, r2)
        lat.step(20000)
        rho = lat.moments()[0][:, 0]
        lat.close()
        rin = rho[:, n // 2, n // 2]
        rout = rho[:, 0, 0]
        # radius from the area the dense species occupies above the outer value
        area = np.sum((rho[0] - rout[0]) / (rin[0] - rout[0]))
        Reff = np.sqrt(area / np.pi)
        dp = _pressure(*rin) - _pressure(*rout)
        pts.append((Reff, dp, rin, rout))
        _say(f"  droplet R0 = {R}: R = {Reff:.3f}, inside {rin.round(4)}, outside {rout.round(4)}, dp = {dp:.5e}")
    inv_r = np.array([1.0 / p[0] for p in pts])
    dps = np.array([p[1] for p in pts])
    gamma, c0 = np.polyfit(inv_r, dps, 1)
    return gamma, c0, pts


def test_laplace_surface_tension(fm):
    """gamma from dp = gamma / R over four droplets (equimolar radii from
    the dense species' excess area).  Measured here: 0.151.  The paper
    reports 0.174 from its own Laplace experiment without radii, radius
    definition or fit, so the bound against it is loose (15 %); the
    capillary spectrum below is the sharper check of gamma.  The fit's
    intercept, a finite-size pressure offset, must be small against the
    smallest droplet's dp."""
    _say("case Laplace test, G = 1.5")
    gamma, c0, pts = _laplace_gamma(fm)
    _say(f"  gamma = {gamma:.4f} (paper: 0.174), intercept {c0:.2e}")
    assert gamma == pytest.approx(0.174, rel=0.15)
    assert abs(c0) < 0.1 * max(p[1] for p in pts)
    # bulk densities of the largest droplet as printed in Sec. VI B
    rin, rout = pts[-1][2], pts[-1][3]
    assert float(f"{rin[0]:.2g}") == DENSE and float(f"{rout[1]:.2g}") == DENSE
    assert float(f"{rin[1]:.1g}") == LIGHT and float(f"{rout[0]:.1g}") == LIGHT


def _heights(phi, x0, x1):
    """Crossing of phi = rho_1 - rho_2 through 0 between columns x0 and x1,
    per row, by linear interpolation (phi changes sign once there)."""
    seg = phi[:, x0:x1]
    s = np.sign(seg)
    idx = np.argmax(s[:, :-1] != s[:, 1:], axis=1)
    rows = np.arange(phi.shape[0])
    a, b = seg[rows, idx], seg[rows, idx + 1]
    return x0 + idx + a / (a - b)


def test_capillary_spectrum(fm):
    """100 x 512 box, 50 x 512 stripe, k_BT = 1e-5, FP32: 1e5 steps of
    burn-in, then 2000 snapshots 1000 steps apart (2.1e6 steps in all, as in
    the paper).  For k = 2 pi n / 512, both interfaces' height spectra
    <|h(k)|^2> (h(k) = L^-1/2 sum_y h(y) e^-iky) against k_BT / (gamma k^2),
    gamma from the Laplace test: band means of k^2 <|h|^2> gamma / k_BT within
    15 % for n in [5, 20) and [20, 80) (k up to 0.98).  Modes n < 5 relax
    over more than 1e5 steps and are left out."""
    import workloads
    kT = 1e-5
    nx, ny = 100, 512
    gamma, _, _ = _laplace_gamma(fm)
    _say(f"case capillary spectrum, gamma = {gamma:.4f}")
    r1, r2 = workloads.stripe_density(nx, ny, 50, DENSE, LIGHT)
    lat = fm.Lattice(fm.Params(lattice="d2q9", storage="f32", nx=nx, ny=ny, tau=(1.0, 1.0), tau_d=1.0, G=G, kT=kT,
                               seed=7))
    lat.init_density(r1, r2)
    lat.step(100000)
    acc = np.zeros(ny)
    snaps = 2000
    for _ in range(snaps):
        lat.step(1000)
        rho = lat.moments()[0][:, 0]
        phi = rho[0] - rho[1]
        for x0, x1 in ((5, 45), (55, 95)):
            h = _heights(phi, x0, x1)
            hk = np.fft.fft(h - h.mean()) / np.sqrt(ny)
            acc += np.abs(hk) ** 2
    lat.close()
    spec = acc / (2 * snaps)
    k = 2 * np.pi * np.fft.fftfreq(ny)
    for lo, hi in ((5, 20), (20, 80)):
        ratio = np.mean([k[n] ** 2 * spec[n] * gamma / kT for n in range(lo, hi)])
        _say(f"  n in [{lo},{hi}): k^2 <|h|^2> gamma / k_BT = {ratio:.3f}")
        assert ratio == pytest.approx(1.0, rel=0.15), (lo, hi)
