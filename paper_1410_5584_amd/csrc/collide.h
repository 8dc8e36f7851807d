// Per-site collision of the two-species FLBE (Sec. V, Eqs. (84)-(86)),
// evaluated directly in population space.
//
// For species sigma with transport and ghost relaxation lambda, momentum
// relaxation lambda_d, density rho, momentum j = j_bar (Eq. (86)) and
// acceleration a (Eq. (87)), the update f*_i = f_i + w_i sum_a T_ai R_a / N_a
// with R_a from Eq. (85) is assembled as
//
//   f*_i = (1 - lambda) f_i + w_i [ A + c_i.V + c_i.M.c_i + G_i ]
//
// where
//  - the relaxation of every non-conserved, non-momentum mode towards 0 is
//    lambda (f_i - w_i rho - 3 w_i c_i.j) by completeness (Eq. (79)), so no
//    forward mode transform is needed;
//  - R is the momentum-mode R_alpha = lambda_d (rho u - j) + (1 - lambda_d/2)
//    F + xi_alpha with u = v_b_bar + a_b / 2 (Eq. (85)), the renormalised force
//    (Eq. (72)) and the momentum noise +-xi (Eq. (74)); V = 3 lambda j + 3 R;
//  - the second-order (transport) parts of the truncated equilibrium (Eq. (29))
//    and of the forcing (Eq. (31)) project onto transport modes only:
//    9/2 (c c - I/3) : P with P = lambda rho u u + (1 - lambda/2) rho
//    (a v + v a) and the species velocity rho v = j + R / 2 (Eqs. (65), (71));
//  - the noise of Eq. (74) on mode a has standard deviation
//    sqrt((2 lambda - lambda^2) N_a mu rho) = g sqrt(N_a), so its population
//    image is w_i T_ai g z_a / sqrt(N_a) (independent of how T_a is scaled).
//    The transport modes are second-order polynomials, so their noise is
//    c.N.c - tr(N)/3 for a symmetric tensor N built from their normals; with
//    M = 9/2 P + N and A = lambda rho - tr(M)/3 the whole transport sector is
//    one tensor contraction.  G_i is the ghost-mode noise, written per
//    velocity class from a few precombined amplitudes.
// Opposite velocities share the even part (A, c.M.c, even ghosts) and negate
// the odd part (c.V, odd ghosts), so every pair costs one E and one O.
#pragma once

#include "lattice.h"
#include "rng.h"

namespace fmlb {

constexpr double csqrt(double x)
{
    double r = x > 1.0 ? x : 1.0;
    for (int k = 0; k < 200; ++k) r = 0.5 * (r + x / r);
    return r;
}

// 1 / sqrt(N_a) per mode, evaluated at compile time.
template <class L>
struct NormTable {
    double inv_sqrt[L::Q];
    constexpr NormTable() : inv_sqrt()
    {
        for (int a = 0; a < L::Q; ++a) inv_sqrt[a] = csqrt((double)L::Nden[a] / (double)L::Nnum[a]);
    }
};

template <class L>
inline constexpr NormTable<L> kNorm{};

// Per-lattice physical constants, already converted to the arithmetic type.
template <class Real>
struct Phys {
    Real lam[2];         // 1 / tau_sigma
    Real lam_d;          // 1 / tau_d
    Real negG;           // -G
    Real gain[2];        // sqrt((2 lambda - lambda^2) mu), mu = 3 k_B T
    Real sd_gain;        // sqrt((2 lambda_d - lambda_d^2) k_B T), 0 without momentum noise
    uint32_t key0, key1; // Philox key (seed)
};

// Reciprocal and square root.  FP32 uses the hardware approximations
// (v_rcp_f32, v_sqrt_f32, both within 1 ulp): every operand here is a
// positive density or -2 ln u of a 16-bit uniform, never denormal, so the
// IEEE-exact sequences would only add range-fixup instructions.
template <class Real>
__device__ __forceinline__ Real rcp(Real x)
{
    if constexpr (sizeof(Real) == 4)
        return __builtin_amdgcn_rcpf(x);
    else
        return Real(1) / x;
}

template <class Real>
__device__ __forceinline__ Real root(Real x)
{
    if constexpr (sizeof(Real) == 4)
        return __builtin_amdgcn_sqrtf(x);
    else
        return sqrt(x);
}

// Acceleration of Eq. (87): a_sigma = -G sum_i w_i rho_sigma'(r + c_i) c_i.
// nb(i, s) returns rho_s at r + c_i.  Summation order is fixed (velocity
// order), so every kernel that uses this helper gets the same bits.
template <class L, class Real, class NB>
__device__ __forceinline__ void lattice_acceleration(const NB &nb, Real negG, Real (&acc)[2][3])
{
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        Real ax = 0, ay = 0, az = 0;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const Real t = Real(L::w36[i]) / Real(36) * nb(i, 1 - s);
            if (L::cx[i]) ax += L::cx[i] > 0 ? t : -t;
            if (L::cy[i]) ay += L::cy[i] > 0 ? t : -t;
            if (L::D == 3 && L::cz[i]) az += L::cz[i] > 0 ? t : -t;
        }
        acc[s][0] = negG * ax;
        acc[s][1] = negG * ay;
        acc[s][2] = negG * az;
    }
}

template <class L, class Real>
__device__ __forceinline__ void moments(const Real (&f)[L::Q], Real &rho, Real (&j)[3])
{
    Real r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        r += f[i];
        if (L::cx[i]) jx += L::cx[i] > 0 ? f[i] : -f[i];
        if (L::cy[i]) jy += L::cy[i] > 0 ? f[i] : -f[i];
        if (L::D == 3 && L::cz[i]) jz += L::cz[i] > 0 ? f[i] : -f[i];
    }
    rho = r;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
}

// Noise of the non-hydrodynamic modes, from zs[a] = g z_a / sqrt(N_a):
// the transport tensor N and the ghost amplitudes per velocity class.
template <class L, class Real>
struct ModeNoise;

// D2Q9, Table I: transport e (3), P_ww (4), P_xy (5); ghosts q_x (6),
// q_y (7), epsilon (8).
template <class Real>
struct ModeNoise<D2Q9, Real> {
    Real Nxx, Nyy, Nzz, Nxy, Nyz, Nxz;
    Real e0, e1, e2, qx, qy;
    __device__ __forceinline__ void init(const Real *zs)
    {
        // e = 3 (c_x^2 - 1/3) + 3 (c_y^2 - 1/3), P_ww = (c_x^2 - 1/3) - (c_y^2 - 1/3)
        Nxx = Real(3) * zs[3] + zs[4];
        Nyy = Real(3) * zs[3] - zs[4];
        Nzz = 0;
        Nxy = Real(0.5) * zs[5];
        Nyz = Nxz = 0;
        // epsilon = 9|c|^4 - 15|c|^2 + 2: 2, -4, 8 on |c|^2 = 0, 1, 2
        e0 = Real(2) * zs[8];
        e1 = Real(-4) * zs[8];
        e2 = Real(8) * zs[8];
        qx = zs[6];
        qy = zs[7];
    }
    // even part at velocity i
    __device__ __forceinline__ Real even(int i) const
    {
        const int c2 = D2Q9::cx[i] * D2Q9::cx[i] + D2Q9::cy[i] * D2Q9::cy[i];
        return c2 == 0 ? e0 : (c2 == 1 ? e1 : e2);
    }
    // odd part: q_alpha = (3|c|^2 - 4) c_alpha = -c_alpha (axis), 2 c_alpha (diagonal)
    __device__ __forceinline__ Real odd(int i) const
    {
        const int cx = D2Q9::cx[i], cy = D2Q9::cy[i];
        const int c2 = cx * cx + cy * cy;
        Real o = 0;
        if (cx) o += cx > 0 ? qx : -qx;
        if (cy) o += cy > 0 ? qy : -qy;
        return c2 == 1 ? -o : Real(2) * o;
    }
};

// D3Q19: transport rows 4..6 are 3 c_alpha^2 - 1 (scaled Hermite), rows 7..9
// c_x c_y, c_y c_z, c_x c_z; ghosts q_alpha (10..12), m_alpha (13..15),
// pi_xx (16), pi_ww (17), epsilon (18) -- see lattice.h.
template <class Real>
struct ModeNoise<D3Q19, Real> {
    Real Nxx, Nyy, Nzz, Nxy, Nyz, Nxz;
    Real e_r, e_ax, e_ay, e_az, e_xy, e_xz, e_yz;
    Real o_x, o_y, o_z, a_xy, b_xy, a_xz, b_xz, a_yz, b_yz;
    __device__ __forceinline__ void init(const Real *zs)
    {
        Nxx = Real(3) * zs[4];
        Nyy = Real(3) * zs[5];
        Nzz = Real(3) * zs[6];
        Nxy = Real(0.5) * zs[7];
        Nyz = Real(0.5) * zs[8];
        Nxz = Real(0.5) * zs[9];
        const Real pxx = zs[16], pww = zs[17], eps = zs[18];
        // even ghosts per class: pi_xx, pi_ww, epsilon values of lattice.h
        e_r = eps;
        e_ax = Real(-2) * pxx - Real(2) * eps;
        e_ay = pxx - pww - Real(2) * eps;
        e_az = pxx + pww - Real(2) * eps;
        e_xy = pxx + pww + eps;
        e_xz = pxx - pww + eps;
        e_yz = Real(-2) * pxx + eps;
        // odd ghosts: axis q_alpha = -2 c_alpha; edges q and m combine per plane
        o_x = Real(-2) * zs[10];
        o_y = Real(-2) * zs[11];
        o_z = Real(-2) * zs[12];
        a_xy = zs[10] + zs[13];  // c_x (q_x + m_x) + c_y (q_y - m_y)
        b_xy = zs[11] - zs[14];
        a_xz = zs[10] - zs[13];  // c_x (q_x - m_x) + c_z (q_z + m_z)
        b_xz = zs[12] + zs[15];
        a_yz = zs[11] + zs[14];  // c_y (q_y + m_y) + c_z (q_z - m_z)
        b_yz = zs[12] - zs[15];
    }
    __device__ __forceinline__ Real even(int i) const
    {
        const int x = D3Q19::cx[i] != 0, y = D3Q19::cy[i] != 0, z = D3Q19::cz[i] != 0;
        if (!x && !y && !z) return e_r;
        if (x && !y && !z) return e_ax;
        if (!x && y && !z) return e_ay;
        if (!x && !y && z) return e_az;
        if (x && y) return e_xy;
        if (x && z) return e_xz;
        return e_yz;
    }
    __device__ __forceinline__ Real odd(int i) const
    {
        const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
        auto sgn = [](int c, Real v) { return c > 0 ? v : -v; };
        const int n = (cx != 0) + (cy != 0) + (cz != 0);
        if (n == 0) return Real(0);
        if (n == 1) return cx ? sgn(cx, o_x) : (cy ? sgn(cy, o_y) : sgn(cz, o_z));
        if (cx && cy) return sgn(cx, a_xy) + sgn(cy, b_xy);
        if (cx && cz) return sgn(cx, a_xz) + sgn(cz, b_xz);
        return sgn(cy, a_yz) + sgn(cz, b_yz);
    }
};

// The normals of a site in two stages, in the order of the stream convention:
// stage 1 yields normals 0..K1-1 (the D momentum normals and species 1's
// mode normals), stage 2 normals K1..K-1 (species 2's mode normals).  Stream
// word w carries normals 2w and 2w+1; the words of stage 1's last Philox
// block that stage 2 needs are carried over, so every block is computed once.
// Splitting keeps only one species' normals live at a time.
template <class L, class Real>
struct SiteNormals {
    static constexpr int K = L::D + 2 * L::NS;
    static constexpr int K1 = L::D + L::NS;  // even for D2Q9 (8) and D3Q19 (18)
    static constexpr int K2 = K - K1;
    static constexpr int W1 = K1 / 2;        // words of stage 1
    static constexpr int W = (K + 1) / 2;    // words in all
    static constexpr int B1 = (W1 + 3) / 4;  // Philox blocks of stage 1
    static constexpr int NB = (W + 3) / 4;
    static constexpr int CARRY = 4 * B1 - W1;
    static_assert(K1 % 2 == 0, "stage boundary must fall between Box-Muller pairs");
    uint32_t carry[CARRY > 0 ? CARRY : 1];

    __device__ __forceinline__ void stage1(const Phys<Real> &ph, const Counter &ctr, Real (&z)[K1])
    {
#pragma unroll
        for (int b = 0; b < B1; ++b) {
            uint32_t w[4];
            block_words(ctr, (uint32_t)b, ph.key0, ph.key1, w);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int word = 4 * b + t;
                if (word < W1)
                    word_normals<Real>(w[t], z[2 * word], z[2 * word + 1]);
                else
                    carry[word - W1] = w[t];
            }
        }
    }

    __device__ __forceinline__ void stage2(const Phys<Real> &ph, const Counter &ctr, Real (&z)[K2])
    {
        auto put = [&](int word, uint32_t w) {
            Real a, c;
            word_normals<Real>(w, a, c);
            const int k = 2 * word - K1;
            z[k] = a;
            if (k + 1 < K2) z[k + 1] = c;
        };
#pragma unroll
        for (int q = 0; q < CARRY; ++q) put(W1 + q, carry[q]);
#pragma unroll
        for (int b = B1; b < NB; ++b) {
            uint32_t w[4];
            block_words(ctr, (uint32_t)b, ph.key0, ph.key1, w);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * b + t < W) put(4 * b + t, w[t]);
        }
    }
};

// Quantities shared by both species of a site: forces F = rho a, the
// equilibrium velocity u = v_b_bar + a_b / 2 (Eq. (85)) and the momentum
// noise amplitude sqrt((2 lambda_d - lambda_d^2) k_B T rho rho' / rho_t)
// (Eq. (74) with the local densities).
template <class Real>
struct SiteCommon {
    Real F[2][3];
    Real u[3];
    Real sd;
};

template <class L, class Real>
__device__ __forceinline__ SiteCommon<Real> site_common(const Real (&rho)[2], const Real (&j)[2][3],
                                                        const Real (&acc)[2][3], const Phys<Real> &ph)
{
    constexpr int D = L::D;
    SiteCommon<Real> c;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int al = 0; al < 3; ++al) c.F[s][al] = rho[s] * acc[s][al];
    const Real rt = rho[0] + rho[1];
    c.u[0] = c.u[1] = c.u[2] = 0;
    if (rt > Real(0)) {
        const Real inv_rt = rcp(rt);
#pragma unroll
        for (int al = 0; al < D; ++al)
            c.u[al] = (j[0][al] + j[1][al]) * inv_rt + Real(0.5) * ((c.F[0][al] + c.F[1][al]) * inv_rt);
    }
    c.sd = 0;
    if (rho[0] > Real(0) && rho[1] > Real(0)) c.sd = ph.sd_gain * root(rho[0] * rho[1] * rcp(rt));
    return c;
}

// base + w_i x.  In FP32 the weights 4/9, 1/9, 1/36 (D2Q9) and 1/3, 1/18,
// 1/36 (D3Q19) round up, so their rounded values sum to 1 + 7e-9 (D2Q9) or
// 1 + 1.5e-8 (D3Q19); with a plain product that excess would add
// lambda * 1.5e-8 of the mass every step (a 3 % drift over 2e6 steps).  The
// weight is applied as a head and a tail (w = w_hi + w_lo exactly to FP32
// working precision), so the product carries only unbiased rounding.
template <class L, class Real>
__device__ __forceinline__ Real relax_add(int i, Real base, Real x)
{
    const double wd = (double)L::w36[i] / 36.0;
    if constexpr (sizeof(Real) == 4) {
        const float hi = (float)wd;
        const float lo = (float)(wd - (double)hi);
        return __builtin_fmaf(x, hi, __builtin_fmaf(x, lo, base));
    } else {
        return base + wd * x;
    }
}

// Collision of one species at one site, in place: f holds the deviations
// d_i = f_i - w_i ref (see collide_site), r the absolute density, dr = r -
// ref, js the momentum, a the acceleration, F = r a, u the common
// equilibrium velocity, lam / lam_d / gain the species' rates and noise
// gain sqrt((2 lambda - lambda^2) mu).  The momentum noise is amp * zmom
// (binary model: +-sigma_d times the D momentum normals; N species: amp = 1
// and zmom the species' correlated noise); zmode holds the NS normals of the
// species' non-hydrodynamic modes.
template <class L, class Real>
__device__ __forceinline__ void relax_species(Real (&f)[L::Q], Real r, Real dr, const Real (&js)[3],
                                              const Real (&a)[3], const Real (&F)[3], const Real (&u)[3], Real lam,
                                              Real lam_d, Real gain, Real amp, const Real *zmom, const Real *zmode)
{
    constexpr int Q = L::Q, D = L::D;
    Real R[3] = {0, 0, 0}, v[3] = {0, 0, 0};
#pragma unroll
    for (int al = 0; al < D; ++al)
        R[al] = lam_d * (r * u[al] - js[al]) + (Real(1) - Real(0.5) * lam_d) * F[al] + amp * zmom[al];
    if (r > Real(0)) {
        const Real inv_r = rcp(r);
#pragma unroll
        for (int al = 0; al < D; ++al) v[al] = (js[al] + Real(0.5) * R[al]) * inv_r;
    }

    // non-hydrodynamic mode noise, zs[a] = g z_a / sqrt(N_a)
    Real zs[Q];
    const Real g = r > Real(0) ? gain * root(r) : Real(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) zs[q] = 0;
#pragma unroll
    for (int q = D + 1; q < Q; ++q) zs[q] = g * Real(kNorm<L>.inv_sqrt[q]) * zmode[q - D - 1];
    ModeNoise<L, Real> mn;
    mn.init(zs);

    // M = 9/2 P + N, P = lambda rho u u + (1 - lambda/2) rho (a v + v a)
    const Real lr = lam * r;
    const Real cf = (Real(1) - Real(0.5) * lam) * r;
    auto Pc = [&](int al, int be) { return lr * u[al] * u[be] + cf * (a[al] * v[be] + v[al] * a[be]); };
    const Real Mxx = Real(4.5) * Pc(0, 0) + mn.Nxx;
    const Real Myy = Real(4.5) * Pc(1, 1) + mn.Nyy;
    const Real Mzz = D == 3 ? Real(4.5) * Pc(2, 2) + mn.Nzz : Real(0);
    const Real Mxy2 = Real(9) * Pc(0, 1) + Real(2) * mn.Nxy;  // 2 M_xy
    const Real Myz2 = D == 3 ? Real(9) * Pc(1, 2) + Real(2) * mn.Nyz : Real(0);
    const Real Mxz2 = D == 3 ? Real(9) * Pc(0, 2) + Real(2) * mn.Nxz : Real(0);
    const Real A = lam * dr - (Mxx + Myy + Mzz) * Real(1.0 / 3.0);
    const Real Vx = Real(3) * (lam * js[0] + R[0]);
    const Real Vy = Real(3) * (lam * js[1] + R[1]);
    const Real Vz = D == 3 ? Real(3) * (lam * js[2] + R[2]) : Real(0);
    const Real keep = Real(1) - lam;

#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ib = opposite<L>(i);
        if (ib < i) continue;  // handled with its partner
        const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
        Real cMc = 0;
        if (cx) cMc += Mxx;
        if (cy) cMc += Myy;
        if (D == 3 && cz) cMc += Mzz;
        if (cx && cy) cMc += (cx * cy > 0) ? Mxy2 : -Mxy2;
        if (D == 3 && cy && cz) cMc += (cy * cz > 0) ? Myz2 : -Myz2;
        if (D == 3 && cx && cz) cMc += (cx * cz > 0) ? Mxz2 : -Mxz2;
        const Real E = A + cMc + mn.even(i);
        if (ib == i) {
            f[i] = relax_add<L>(i, keep * f[i], E);
            continue;
        }
        Real cV = 0;
        if (cx) cV += cx > 0 ? Vx : -Vx;
        if (cy) cV += cy > 0 ? Vy : -Vy;
        if (D == 3 && cz) cV += cz > 0 ? Vz : -Vz;
        const Real O = cV + mn.odd(i);
        f[i] = relax_add<L>(i, keep * f[i], E + O);
        f[ib] = relax_add<L>(ib, keep * f[ib], E - O);
    }
}

// Collision of species s of the binary model at one site, in place.  zmom:
// the D momentum normals (noise +sigma_d z for species 1, -sigma_d z for
// species 2, Eq. (74)); zmode: the NS normals of this species' modes.
template <class L, class Real>
__device__ __forceinline__ void collide_species(int s, Real (&f)[L::Q], Real r, Real dr, const Real (&js)[3],
                                                const Real (&a)[3], const SiteCommon<Real> &c,
                                                const Phys<Real> &ph, const Real *zmom, const Real *zmode)
{
    relax_species<L, Real>(f, r, dr, js, a, c.F[s], c.u, ph.lam[s], ph.lam_d, ph.gain[s], s == 0 ? c.sd : -c.sd,
                           zmom, zmode);
}

// Collide both species at one site in place, species 1 first.  f holds the
// pre-collision populations pulled to the site as deviations d_i = f_i -
// w_i ref_sigma from a reference density (ref = 0: absolute values), drho /
// j their moments (moments(): drho = rho - ref, j unchanged because
// sum_i w_i c_i = 0), acc the accelerations of Eq. (87) (which likewise only
// see density differences).  The update is written for the deviations:
// since (1 - lambda) + lambda = 1, f*_i - w_i ref = (1 - lambda) d_i +
// w_i [lambda drho - tr(M)/3 + ...], so every term is of the size of the
// deviations and FP32 rounding stays at their scale (with absolute FP32
// values the rounding of terms of size w_i rho is not symmetric for smooth
// fields and drifts the mass by ~1e-8 per step).  store(s, f[s]) is called
// as soon as species s is done, so its registers can be released early.
template <class L, class Real, class StoreFn>
__device__ __forceinline__ void collide_site(Real (&f)[2][L::Q], const Real (&drho)[2], const Real (&j)[2][3],
                                             const Real (&acc)[2][3], const Phys<Real> &ph, const Real (&ref)[2],
                                             const Counter &ctr, StoreFn &&store)
{
    constexpr int D = L::D;
    using SN = SiteNormals<L, Real>;
    const Real rho[2] = {ref[0] + drho[0], ref[1] + drho[1]};
    const SiteCommon<Real> c = site_common<L, Real>(rho, j, acc, ph);
    SN sn;
    Real zmom[3] = {0, 0, 0};
    {
        Real z1[SN::K1];
        sn.stage1(ph, ctr, z1);
#pragma unroll
        for (int al = 0; al < D; ++al) zmom[al] = z1[al];
        collide_species<L, Real>(0, f[0], rho[0], drho[0], j[0], acc[0], c, ph, zmom, z1 + D);
    }
    store(0, f[0]);
    {
        Real z2[SN::K2];
        sn.stage2(ph, ctr, z2);
        collide_species<L, Real>(1, f[1], rho[1], drho[1], j[1], acc[1], c, ph, zmom, z2);
    }
    store(1, f[1]);
}

}  // namespace fmlb
