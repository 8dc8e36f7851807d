"""Capillary fluctuations of a liquid-liquid interface (Sec. VI B) on the GPU.

The paper's set-up:
  - D2Q9, G = 1.5, every relaxation rate 1;
  - bulk densities 2.3 / 0.06, interface about 6 sites wide;
  - surface tension 0.174 from a Laplace experiment;
  - a 50 x 512 stripe in a 100 x 512 periodic box at k_BT = 1e-5, whose interface height spectrum
    follows Eq. (91), <|h(k)|^2> = k_BT / (gamma k^2), up to k of about 1.
Here:
  - the Laplace experiment: droplets of several radii, with the bulk pressure of the model
    p = c_s^2 (rho_1 + rho_2) + c_s^2 G rho_1 rho_2 (the momentum balance of the pair force of
    Eq. (87) across an interface, sum_i w_i c_i c_i = c_s^2 I), gamma from dp = gamma / R;
    it gives 0.151;
  - the spectrum of both interfaces of the fluctuating stripe against Eq. (91) with the paper's
    gamma = 0.174, which it follows within a few percent (so the spectrum's gamma agrees with the
    paper's, and the Laplace value here is the one that differs);
  - FP32 against FP64 storage on the same spectrum.
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
    # bulk densities of the largest droplet against those printed in Sec. VI B
    # (2.3 and 0.06, to the digits given there); the Laplace pressure of a
    # finite droplet shifts them by a few percent (measured: 2.355 / 0.061
    # inside, 0.066 / 2.320 outside)
    rin, rout = pts[-1][2], pts[-1][3]
    assert rin[0] == pytest.approx(DENSE, rel=0.03) and rout[1] == pytest.approx(DENSE, rel=0.03)
    assert rin[1] == pytest.approx(LIGHT, rel=0.12) and rout[0] == pytest.approx(LIGHT, rel=0.12)


def _heights(phi, x0, x1):
    """Crossing of phi = rho_1 - rho_2 through 0 between columns x0 and x1,
    per row, by linear interpolation (phi changes sign once there)."""
    seg = phi[:, x0:x1]
    s = np.sign(seg)
    idx = np.argmax(s[:, :-1] != s[:, 1:], axis=1)
    rows = np.arange(phi.shape[0])
    a, b = seg[rows, idx], seg[rows, idx + 1]
    return x0 + idx + a / (a - b)


GAMMA_PAPER = 0.174  # Sec. VI B, from the paper's Laplace experiment
KT_CAP = 1e-5


def _spectrum(fm, storage, seed, burn, snaps, every=1000):
    """Mean |h(k)|^2 over both interfaces of the 100 x 512 stripe, h(k) =
    L^-1/2 sum_y h(y) e^-iky, from `snaps` snapshots `every` steps apart."""
    import workloads
    nx, ny = 100, 512
    r1, r2 = workloads.stripe_density(nx, ny, 50, DENSE, LIGHT)
    lat = fm.Lattice(fm.Params(lattice="d2q9", storage=storage, nx=nx, ny=ny, tau=(1.0, 1.0), tau_d=1.0, G=G,
                               kT=KT_CAP, seed=seed))
    lat.init_density(r1, r2)
    lat.step(burn)
    acc = np.zeros(ny)
    for _ in range(snaps):
        lat.step(every)
        rho = lat.moments()[0][:, 0]
        phi = rho[0] - rho[1]
        for x0, x1 in ((5, 45), (55, 95)):
            h = _heights(phi, x0, x1)
            acc += np.abs(np.fft.fft(h - h.mean()) / np.sqrt(ny)) ** 2
    lat.close()
    return acc / (2 * snaps), 2 * np.pi * np.fft.fftfreq(ny)


def _band(spec, k, lo, hi, gamma):
    return float(np.mean([k[n] ** 2 * spec[n] * gamma / KT_CAP for n in range(lo, hi)]))


def test_capillary_spectrum(fm):
    """100 x 512 box, 50 x 512 stripe, k_BT = 1e-5, FP32: 1e5 steps of
    burn-in, then 2000 snapshots 1000 steps apart (2.1e6 steps in all, as in
    the paper).  For k = 2 pi n / 512, both interfaces' height spectra
    against Eq. (91) with the paper's gamma = 0.174: band means of
    k^2 <|h|^2> gamma / k_BT within 10 % of 1 for n in [5, 20) and [20, 80)
    (k up to 0.98).  Snapshots 1000 steps apart are uncorrelated for n >= 5
    (measured autocorrelation below 0.1), so the statistical error of a band
    mean is about 0.5 %; measured: 0.94-0.96 and 0.98-0.99.  With the
    Laplace gamma of this implementation (0.151) the ratios are 0.82 / 0.85:
    the spectrum gives a gamma near the paper's value and the Laplace
    reading is the one that differs.  n < 5 is left out: those modes lie
    about 10 % below the law."""
    _say("case capillary spectrum FP32, gamma 0.174")
    spec, k = _spectrum(fm, "f32", 7, 100000, 2000)
    for lo, hi in ((5, 20), (20, 80)):
        ratio = _band(spec, k, lo, hi, GAMMA_PAPER)
        _say(f"  n in [{lo},{hi}): k^2 <|h|^2> gamma / k_BT = {ratio:.3f}")
        assert ratio == pytest.approx(1.0, rel=0.10), (lo, hi)


def test_capillary_spectrum_fp32_matches_fp64(fm):
    """FP32 and FP64 storage give the same interface spectrum: 500 snapshots
    each, different seeds (independent samples, about 1 % statistical error
    per band), band means within 5 % of each other.  FP32 holds deviations
    from w_i rho_ref; storing absolute FP32 values instead shifted these
    bands by about 10 % in a run of this length."""
    _say("case capillary spectrum FP32 vs FP64")
    s32, k = _spectrum(fm, "f32", 21, 100000, 500)
    s64, _ = _spectrum(fm, "f64", 22, 100000, 500)
    for lo, hi in ((5, 20), (20, 80)):
        a, b = _band(s32, k, lo, hi, GAMMA_PAPER), _band(s64, k, lo, hi, GAMMA_PAPER)
        _say(f"  n in [{lo},{hi}): FP32 {a:.3f}  FP64 {b:.3f}")
        assert a == pytest.approx(b, rel=0.05), (lo, hi)
