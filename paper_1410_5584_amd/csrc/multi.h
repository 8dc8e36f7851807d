// N species (2..4): the multicomponent form of the model (Apps. C and D).
//
// Per site and species sigma, with the densities of the same step:
//   a_sigma = -sum_s' G_sigma,s' sum_i w_i rho_s'(r + c_i) c_i   (Eq. (87), one coupling per pair)
//   u       = sum_sigma (j_bar_sigma + rho_sigma a_sigma / 2) / rho_t
//   momentum noise xi_sigma with covariance (2 lambda_d - lambda_d^2) k_B T
//   (rho_sigma delta_sigma,s' - rho_sigma rho_s' / rho_t) per component (App. D,
//   with the lattice factor of Eq. (74)); every row sums to zero, so the
//   total momentum receives none.  It is sampled with the Cholesky factor L
//   of the block of species 1..N-1 (positive definite when every density is
//   positive): xi_sigma,alpha = sum_k L_sigma,k z_(k D + alpha) for sigma < N,
//   and xi_N = -(xi_1 + ... + xi_(N-1)).  For N = 2 this is the binary
//   model's +-sigma_d z on the same normals.
//   The non-momentum modes of species sigma use normals D (N - 1) + sigma NS + ...
//   and relax as in the binary model (relax_species).
//
// Three launch forms with the same arithmetic (so the same bits): two passes
// (the first pulls every population and writes the interaction potential
// phi_sigma = sum_s' G_sigma,s' (rho_s' - rho_ref,s') per site -- the force
// needs only differences, sum_i w_i c_i = 0 -- the second pulls again,
// collides and stores); a single pass with register pulls; and a single
// pass with the next plane pulled into LDS while the current one collides
// (FP32).  Storage FP64 (absolute) or FP32 (deviations from w_i rho_ref, as
// in the binary FP32 path).
#pragma once

#include "fused.h"

namespace fmlb {

constexpr int kMaxSpecies = 4;

// Velocity components along plane axis 0 (x), plane axis 1 (y, 3D only) and
// the march axis (z in 3D, y in 2D).
template <class L>
struct MarchAxesN {
    static constexpr int c0(int i) { return L::cx[i]; }
    static constexpr int c1(int i) { return L::D == 3 ? L::cy[i] : 0; }
    static constexpr int cm(int i) { return L::D == 3 ? L::cz[i] : L::cy[i]; }
};

template <class Real>
struct MultiPhys {
    Real lam[kMaxSpecies];   // 1 / tau_sigma
    Real lam_d;              // 1 / tau_d
    Real gain[kMaxSpecies];  // sqrt((2 lambda - lambda^2) mu), 0 without noise
    Real sd2;                // (2 lambda_d - lambda_d^2) k_B T, 0 without momentum noise
    Real G[kMaxSpecies][kMaxSpecies];
    Real ref[kMaxSpecies];   // rho_ref of the stored deviations (0 for FP64)
    uint32_t key0, key1;
};

template <class S>
struct MultiArgs {
    using Real = typename Storage<S>::Real;
    const S *src;
    S *dst;
    Real *phi;  // [N][sites]
    Geom g;
    MultiPhys<Real> ph;
    uint32_t step_lo, step_hi;
};

// The stored values of the N Q pulled populations of site (x, y, z).
template <class L, class S, int N>
__device__ __forceinline__ void multi_pull(const S *src, const Geom &g, int x, int y, int z,
                                           typename Storage<S>::Real (&f)[N][L::Q])
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap(x, -L::cx[i], g.nx);
        const int ys = wrap(y, -L::cy[i], g.ny);
        const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
        const size_t site = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
#pragma unroll
        for (int s = 0; s < N; ++s) f[s][i] = Storage<S>::load(src, ((size_t)(s * L::Q + i)) * g.pitch + site);
    }
}

template <class L, class S, int N>
__device__ __forceinline__ void multi_potential(const MultiPhys<typename Storage<S>::Real> &ph,
                                                const typename Storage<S>::Real (&f)[N][L::Q],
                                                typename Storage<S>::Real (&phi)[N]);

template <class L, class S, int N>
__global__ __launch_bounds__(256) void multi_potential_kernel(MultiArgs<S> a)
{
    using Real = typename Storage<S>::Real;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= a.g.nx) return;
    Real f[N][L::Q], phi[N];
    multi_pull<L, S, N>(a.src, a.g, x, y, z, f);
    multi_potential<L, S, N>(a.ph, f, phi);
    const size_t site = (size_t)x + (size_t)a.g.nx * ((size_t)y + (size_t)a.g.ny * (size_t)z);
#pragma unroll
    for (int s = 0; s < N; ++s) a.phi[(size_t)s * a.g.nsites + site] = phi[s];
}

// Momentum noise xi[N][3] of one site from the normals z[0 .. D(N-1)-1].
template <class L, class Real, int N>
__device__ __forceinline__ void multi_momentum_noise(const Real (&rho)[N], Real rt, Real sd2, const Real *z,
                                                     Real (&xi)[N][3])
{
    constexpr int D = L::D;
#pragma unroll
    for (int s = 0; s < N; ++s) xi[s][0] = xi[s][1] = xi[s][2] = 0;
    bool positive = rt > Real(0);
#pragma unroll
    for (int s = 0; s < N; ++s) positive = positive && rho[s] > Real(0);
    if (!positive) return;
    // covariance block of species 0..N-2 and its lower Cholesky factor
    const Real inv_rt = rcp(rt);
    Real C[N - 1][N - 1], Lc[N - 1][N - 1];
#pragma unroll
    for (int p = 0; p < N - 1; ++p)
#pragma unroll
        for (int q = 0; q < N - 1; ++q) C[p][q] = sd2 * ((p == q ? rho[p] : Real(0)) - rho[p] * rho[q] * inv_rt);
#pragma unroll
    for (int p = 0; p < N - 1; ++p)
#pragma unroll
        for (int q = 0; q < N - 1; ++q) Lc[p][q] = 0;
#pragma unroll
    for (int p = 0; p < N - 1; ++p) {
#pragma unroll
        for (int q = 0; q <= p; ++q) {
            Real acc = C[p][q];
#pragma unroll
            for (int m = 0; m < q; ++m) acc -= Lc[p][m] * Lc[q][m];
            if (q == p)
                Lc[p][p] = acc > Real(0) ? root(acc) : Real(0);
            else
                Lc[p][q] = Lc[q][q] > Real(0) ? acc * rcp(Lc[q][q]) : Real(0);
        }
    }
#pragma unroll
    for (int al = 0; al < D; ++al) {
        Real total = 0;
#pragma unroll
        for (int p = 0; p < N - 1; ++p) {
            Real v = 0;
#pragma unroll
            for (int k = 0; k <= p; ++k) v += Lc[p][k] * z[k * D + al];
            xi[p][al] = v;
            total += v;
        }
        xi[N - 1][al] = -total;
    }
}

// Normals K0 .. K1-1 of a site's stream into z[0 .. K1-K0) (word w: normals
// 2w, 2w + 1; block b: words 4b .. 4b+3, from words(b, w)).  Stages are
// called in order over consecutive ranges; `carry` holds the words of the
// last block of the previous stage, so a block that two stages share is
// fetched once.
template <class Real, int K0, int K1, class WordsFn>
__device__ __forceinline__ void normals_stage(WordsFn &&words, uint32_t (&carry)[4], Real *z)
{
    constexpr int B0 = K0 / 8, B1 = (K1 - 1) / 8;
#pragma unroll
    for (int b = B0; b <= B1; ++b) {
        uint32_t w[4];
        if (b == B0 && K0 % 8 != 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) w[t] = carry[t];
        } else {
            words((uint32_t)b, w);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 8 * b + 2 * t;  // first normal of word t
            if (k + 1 < K0 || k >= K1) continue;
            Real z0, z1;
            word_normals<Real>(w[t], z0, z1);
            if (k >= K0) z[k - K0] = z0;
            if (k + 1 >= K0 && k + 1 < K1) z[k + 1 - K0] = z1;
        }
        if (b == B1) {
#pragma unroll
            for (int t = 0; t < 4; ++t) carry[t] = w[t];
        }
    }
}

// rho_sigma = ref_sigma + drho_sigma and rho_t = sum_sigma rho_sigma, in
// species order.
template <class Real, int N>
__device__ __forceinline__ void multi_densities(const MultiPhys<Real> &ph, const Real (&dr)[N], Real (&rho)[N], Real &rt)
{
    rt = 0;
#pragma unroll
    for (int s = 0; s < N; ++s) {
        rho[s] = ph.ref[s] + dr[s];
        rt += rho[s];
    }
}

// F_sigma = rho_sigma a_sigma (Eq. (87) times the density).
template <class Real>
__device__ __forceinline__ void species_load(Real rho, const Real (&acc)[3], Real (&F)[3])
{
#pragma unroll
    for (int al = 0; al < 3; ++al) F[al] = rho * acc[al];
}

// u = sum_sigma (j_bar_sigma + F_sigma / 2) / rho_t (zero where rho_t <= 0).
template <class L, class Real, int N>
__device__ __forceinline__ void multi_velocity(const Real (&j)[N][3], const Real (&F)[N][3], Real rt, Real (&u)[3])
{
    u[0] = u[1] = u[2] = Real(0);
    if (rt > Real(0)) {
        const Real inv_rt = rcp(rt);
#pragma unroll
        for (int al = 0; al < L::D; ++al) {
            Real jt = 0, Ft = 0;
#pragma unroll
            for (int s = 0; s < N; ++s) {
                jt += j[s][al];
                Ft += F[s][al];
            }
            u[al] = jt * inv_rt + Real(0.5) * (Ft * inv_rt);
        }
    }
}

// Moments, velocities, noise and collision of one site, species by
// species: everything of the step after the pull and the force (shared by
// the two-pass and the single-pass kernels, so all give the same bits).
// words(b, w) gives block b of the site's stream; store(s, f[s]) is called
// once species s is collided.  The normals come in stages (the D (N-1)
// momentum normals, then each species' NS), so only one species' mode
// normals are live at a time.
template <class L, class Real, int N, class WordsFn, class StoreFn>
__device__ __forceinline__ void multi_collide(const MultiPhys<Real> &ph, Real (&f)[N][L::Q], const Real (&acc)[N][3],
                                              WordsFn &&words, StoreFn &&store)
{
    constexpr int Q = L::Q, D = L::D, NS = Q - D - 1;
    constexpr int KM = D * (N - 1);
    Real dr[N], rho[N], j[N][3], F[N][3], rt, u[3];
#pragma unroll
    for (int s = 0; s < N; ++s) moments<L, Real>(f[s], dr[s], j[s]);
    multi_densities<Real, N>(ph, dr, rho, rt);
#pragma unroll
    for (int s = 0; s < N; ++s) species_load<Real>(rho[s], acc[s], F[s]);
    multi_velocity<L, Real, N>(j, F, rt, u);
    uint32_t carry[4] = {0, 0, 0, 0};
    Real xi[N][3];
    {
        Real zm[KM];
        normals_stage<Real, 0, KM>(words, carry, zm);
        multi_momentum_noise<L, Real, N>(rho, rt, ph.sd2, zm, xi);
    }
    static_for<N>([&](auto sc) {
        constexpr int sp = decltype(sc)::value;
        Real zs[NS];
        normals_stage<Real, KM + sp * NS, KM + (sp + 1) * NS>(words, carry, zs);
        relax_species<L, Real>(f[sp], rho[sp], dr[sp], j[sp], acc[sp], F[sp], u, ph.lam[sp], ph.lam_d, ph.gain[sp],
                               Real(1), xi[sp], zs);
        store(sc, f[sp]);
    });
}

// The collision of one site written to dst at `site` (two-pass and register-form kernels).
template <class L, class S, int N>
__device__ __forceinline__ void multi_collide_store(const MultiArgs<S> &a, typename Storage<S>::Real (&f)[N][L::Q],
                                                    typename Storage<S>::Real (&acc)[N][3], size_t site)
{
    constexpr int Q = L::Q;
    const Counter ctr{(uint32_t)site, a.step_lo, a.step_hi};
    multi_collide<L, typename Storage<S>::Real, N>(a.ph, f, acc,
                                                   [&](uint32_t b, uint32_t (&w)[4]) {
                                                       block_words(ctr, b, a.ph.key0, a.ph.key1, w);
                                                   },
                                                   [&](int s, auto &fs) {
#pragma unroll
                                                       for (int i = 0; i < Q; ++i)
                                                           Storage<S>::store(a.dst, ((size_t)(s * Q + i)) * a.g.pitch + site,
                                                                             fs[i]);
                                                   });
}

// a_sigma = -sum_i w_i c_i phi_sigma(r + c_i), phi read through nb(i, sigma).
// phi_sigma = sum_s' G_sigma,s' drho_s', drho read through dr(s').
template <class Real, int N, class DR>
__device__ __forceinline__ Real species_potential(const MultiPhys<Real> &ph, int s, const DR &dr)
{
    Real v = 0;
#pragma unroll
    for (int t = 0; t < N; ++t) v += ph.G[s][t] * dr(t);
    return v;
}

// One species' a = -sum_i w_i c_i phi(r + c_i), phi read through nb(i).
template <class L, class Real, class NB>
__device__ __forceinline__ void species_force(const NB &nb, Real (&acc)[3])
{
    Real ax = 0, ay = 0, az = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const Real t = Real(L::w36[i]) / Real(36) * nb(i);
        if (L::cx[i]) ax += L::cx[i] > 0 ? t : -t;
        if (L::cy[i]) ay += L::cy[i] > 0 ? t : -t;
        if (L::D == 3 && L::cz[i]) az += L::cz[i] > 0 ? t : -t;
    }
    acc[0] = -ax;
    acc[1] = -ay;
    acc[2] = -az;
}

template <class L, class Real, int N, class NB>
__device__ __forceinline__ void multi_force(const NB &nb, Real (&acc)[N][3])
{
#pragma unroll
    for (int s = 0; s < N; ++s) species_force<L, Real>([&](int i) { return nb(i, s); }, acc[s]);
}

// phi_sigma = sum_s' G_sigma,s' drho_s' from the pulled populations.
template <class L, class S, int N>
__device__ __forceinline__ void multi_potential(const MultiPhys<typename Storage<S>::Real> &ph,
                                                const typename Storage<S>::Real (&f)[N][L::Q],
                                                typename Storage<S>::Real (&phi)[N])
{
    using Real = typename Storage<S>::Real;
    Real dr[N];
#pragma unroll
    for (int s = 0; s < N; ++s) {
        Real j[3];
        moments<L, Real>(f[s], dr[s], j);
    }
#pragma unroll
    for (int s = 0; s < N; ++s) phi[s] = species_potential<Real, N>(ph, s, [&](int t) { return dr[t]; });
}

template <class L, class S, int N>
__global__ __launch_bounds__(256) void multi_step_kernel(MultiArgs<S> a)
{
    using Real = typename Storage<S>::Real;
    constexpr int Q = L::Q, D = L::D;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= a.g.nx) return;
    const Geom g = a.g;
    Real f[N][Q];
    multi_pull<L, S, N>(a.src, g, x, y, z, f);
    Real acc[N][3];
    multi_force<L, Real, N>(
        [&](int i, int s) -> Real {
            const int xn = wrap(x, L::cx[i], g.nx);
            const int yn = wrap(y, L::cy[i], g.ny);
            const int zn = D == 3 ? wrap(z, L::cz[i], g.nz) : 0;
            return a.phi[(size_t)s * g.nsites + (size_t)xn + (size_t)g.nx * ((size_t)yn + (size_t)g.ny * zn)];
        },
        acc);
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    multi_collide_store<L, S, N>(a, f, acc, site);
}

// Single-pass form.  A workgroup owns a T0 x T1 tile of the plane
// orthogonal to the march axis (z in 3D, y in 2D) and walks `chunk` planes.
// For plane m+1 every tile and halo-ring site pulls its populations and
// writes its potentials into a four-plane LDS ring; after one barrier the
// force of plane m comes from the ring, and the tile re-pulls plane m
// (read one plane earlier, so from cache rather than HBM) to collide and
// store it.  Against the two-pass form this saves the HBM read of the whole
// state per step and the potentials' round trip; the arithmetic is the same
// (same helpers, same order), so the results are bit-identical.
template <class L, class S, int N, int T0, int T1>
__global__ __launch_bounds__(T0 *T1) void multi_fused_kernel(MultiArgs<S> a, int chunk)
{
    using Real = typename Storage<S>::Real;
    using A = MarchAxesN<L>;
    constexpr int Q = L::Q;
    constexpr bool D3 = L::D == 3;
    constexpr int H0 = T0 + 2, H1 = D3 ? T1 + 2 : 1, OFF1 = D3 ? 1 : 0;
    constexpr int PLANE = H0 * H1, NT = T0 * T1, NHALO = PLANE - NT;
    static_assert(D3 || T1 == 1, "2D tiles are one row");
    static_assert(NHALO <= NT, "halo ring larger than the tile");
    __shared__ Real ring[4][N][PLANE];

    const Geom g = a.g;
    const int n0 = g.nx, n1 = D3 ? g.ny : 1, nm = D3 ? g.nz : g.ny;
    const int tiles0 = (n0 + T0 - 1) / T0, tiles1 = (n1 + T1 - 1) / T1;
    const int t0 = (int)(blockIdx.x % (unsigned)tiles0);
    const int t1 = (int)((blockIdx.x / (unsigned)tiles0) % (unsigned)tiles1);
    const int ck = (int)(blockIdx.x / ((unsigned)tiles0 * tiles1));
    const int mbeg = ck * chunk, mend = min(mbeg + chunk, nm);

    const int tid = threadIdx.x;
    const int l0 = tid % T0, l1 = tid / T0;
    const int p0raw = t0 * T0 + l0, p1raw = t1 * T1 + l1;
    const bool inside = p0raw < n0 && p1raw < n1;
    const int p0 = p0raw % n0, p1 = p1raw % n1;
    const int box_own = (l1 + OFF1) * H0 + (l0 + 1);
    // halo ring: the rows / columns around the tile, one site per thread
    int hb = -1, hp0 = 0, hp1 = 0;
    if (tid < NHALO) {
        int h0, h1;
        if (!D3) {
            h0 = tid == 0 ? 0 : H0 - 1;
            h1 = 0;
        } else if (tid < H0) {
            h0 = tid;
            h1 = 0;
        } else if (tid < 2 * H0) {
            h0 = tid - H0;
            h1 = H1 - 1;
        } else {
            const int q = tid - 2 * H0;
            h0 = (q & 1) ? H0 - 1 : 0;
            h1 = 1 + (q >> 1);
        }
        hb = h1 * H0 + h0;
        hp0 = ((t0 * T0 - 1 + h0) % n0 + n0) % n0;
        hp1 = D3 ? ((t1 * T1 - OFF1 + h1) % n1 + n1) % n1 : 0;
    }
    auto slot = [&](int m) { return (m - mbeg + 1) & 3; };
    auto wrapm = [&](int m) { return m < 0 ? m + nm : (m >= nm ? m - nm : m); };
    // plane coordinates (q0, q1, m) -> lattice (x, y, z)
    auto pull_at = [&](int q0, int q1, int m, Real (&f)[N][Q]) {
        if constexpr (D3)
            multi_pull<L, S, N>(a.src, g, q0, q1, m, f);
        else
            multi_pull<L, S, N>(a.src, g, q0, m, 0, f);
    };
    auto put_potentials = [&](int m) {
        Real f[N][Q], phi[N];
        pull_at(p0, p1, wrapm(m), f);
        multi_potential<L, S, N>(a.ph, f, phi);
#pragma unroll
        for (int s = 0; s < N; ++s) ring[slot(m)][s][box_own] = phi[s];
        if (hb >= 0) {
            pull_at(hp0, hp1, wrapm(m), f);
            multi_potential<L, S, N>(a.ph, f, phi);
#pragma unroll
            for (int s = 0; s < N; ++s) ring[slot(m)][s][hb] = phi[s];
        }
    };

    put_potentials(mbeg - 1);
    put_potentials(mbeg);
#pragma unroll 1
    for (int m = mbeg; m < mend; ++m) {
        put_potentials(m + 1);
        __syncthreads();
        Real acc[N][3];
        multi_force<L, Real, N>(
            [&](int i, int s) -> Real {
                return ring[slot(m + A::cm(i))][s][box_own + A::c1(i) * H0 + A::c0(i)];
            },
            acc);
        if (inside) {
            Real f[N][Q];
            pull_at(p0, p1, m, f);
            const size_t site = D3 ? (size_t)p0 + (size_t)n0 * ((size_t)p1 + (size_t)n1 * (size_t)m)
                                   : (size_t)p0 + (size_t)n0 * (size_t)m;
            multi_collide_store<L, S, N>(a, f, acc, site);
        }
    }
}

// LDS of the asynchronous form (bytes): the potential ring (4 planes of the
// tile and its halo ring) and one plane of pulled rows for the tile and the
// halo ring, N Q words per site.
constexpr size_t multi_async_lds_bytes(int D, int Q, int N, int T0, int T1)
{
    const int H0 = T0 + 2, H1 = D == 3 ? T1 + 2 : 1;
    const int plane = H0 * H1, nt = T0 * T1, nhalo = plane - nt;
    return 4u * ((size_t)4 * N * plane + (size_t)N * Q * nt + (size_t)N * Q * nhalo);
}
constexpr size_t kMaxLdsBytes = 160 * 1024;  // per workgroup (gfx950)

// Asynchronous single pass (FP32 storage): the tile walk of the form above,
// with plane m+2's populations going from memory straight into LDS (buffer
// loads with the LDS destination bit, one 64-lane row per instruction, no
// registers held while in flight) during the collision of plane m.  Each
// wave reads back only the rows its own loads wrote, so those rows need
// only the wave's own counters; the potential ring is the only LDS shared
// between waves.  Every population is written once per step and read once
// for its own tile; the halo rows are the neighbouring tiles' own rows, from
// the caches while neighbouring tiles march in step.  The loads of plane
// m+2 are spread over the iteration by species (a wave has at most 63
// vector memory operations in flight, loads and stores together): species
// 1's tile and halo rows after the force, species sigma+1's once species
// sigma is collided, ahead of its stores.  After the first row load of an
// iteration no LDS read follows until the vmcnt(0) at the top of the next
// one.  Same helpers in the same order as the two-pass form: the same bits.
// When species s's row pulls of plane m+2 are issued in the plane loop below:
// 0 at the top (once the rows of plane m+1 are read back), 1 after the force,
// 2 + k once species k is collided.  Three or more species: all but the last
// at the top, the last after the force (256^3: three species 2.09 -> 2.06 ms,
// four 2.88 -> 2.74 ms); two species: the first after the force, the second
// after the first species' collision (1.165 ms, against 1.21 with the other
// rule).
template <int N>
constexpr int multi_pull_phase(int s)
{
    return N >= 3 ? (s < N - 1 ? 0 : 1) : (s == 0 ? 1 : 2 + (s - 1));
}
template <int N>
constexpr bool multi_phase_used(int ph)
{
    for (int s = 0; s < N; ++s)
        if (multi_pull_phase<N>(s) == ph) return true;
    return false;
}

template <class L, int N, int T0, int T1>
__global__ __launch_bounds__(T0 *T1) void multi_async_kernel(MultiArgs<float> a, int chunk)
{
    using Real = float;
    using Raw = uint32_t;
    using A = MarchAxesN<L>;
    constexpr int Q = L::Q, NQ = N * Q;
    constexpr bool D3 = L::D == 3;
    constexpr int H0 = T0 + 2, H1 = D3 ? T1 + 2 : 1, OFF1 = D3 ? 1 : 0;
    constexpr int PLANE = H0 * H1, NT = T0 * T1, NHALO = PLANE - NT;
    static_assert(D3 || T1 == 1, "2D tiles are one row");
    static_assert(NHALO <= NT, "halo ring larger than the tile");
    static_assert(NT % 64 == 0, "whole waves");
    static_assert(multi_async_lds_bytes(L::D, Q, N, T0, T1) <= kMaxLdsBytes, "LDS");
    __shared__ Real ring[4][N][PLANE];
    __shared__ Raw own[NQ][NT];      // plane m+1 (then m+2) populations of the tile
    __shared__ Raw halo[NQ][NHALO];  // same for the halo ring

    const Geom g = a.g;
    const int n0 = g.nx, n1 = D3 ? g.ny : 1, nm = D3 ? g.nz : g.ny;
    const int tiles0 = (n0 + T0 - 1) / T0, tiles1 = (n1 + T1 - 1) / T1;
    const int chunks = (nm + chunk - 1) / chunk;
    const unsigned logical = xcd_contiguous(blockIdx.x, (unsigned)tiles0 * tiles1 * chunks);
    const int t0 = (int)(logical % (unsigned)tiles0);
    const int t1 = (int)((logical / (unsigned)tiles0) % (unsigned)tiles1);
    const int ck = (int)(logical / ((unsigned)tiles0 * tiles1));
    const int mbeg = ck * chunk, mend = min(mbeg + chunk, nm);

    const uint32_t s1 = (uint32_t)n0;
    const uint32_t sm = D3 ? (uint32_t)n0 * n1 : (uint32_t)n0;
    const uint32_t pop_bytes = (uint32_t)g.pitch * 4u;
    __amdgpu_buffer_rsrc_t rsrc[N], rdst[N];
#pragma unroll
    for (int s = 0; s < N; ++s) {
        rsrc[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.src + (size_t)s * Q * g.pitch), 0, (int)(Q * pop_bytes),
                                                    kBufferWord3);
        rdst[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.dst + (size_t)s * Q * g.pitch), 0, (int)(Q * pop_bytes),
                                                    kBufferWord3);
    }

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l0 = tid % T0, l1 = tid / T0;
    const int p0raw = t0 * T0 + l0, p1raw = t1 * T1 + l1;
    const bool inside = p0raw < n0 && p1raw < n1;
    const int p0 = p0raw % n0, p1 = p1raw % n1;
    const int box_own = (l1 + OFF1) * H0 + (l0 + 1);
    // Copies of the wave number and the population stride that the plane loop
    // marks as changed (three species and more): the LDS destinations and the
    // population offsets of the row pulls are then recomputed each plane (one
    // scalar instruction each) instead of being held across the loop, where
    // they did not fit the scalar registers and came back from VGPR lanes
    // (three species: 133 v_readlane per plane; 2.129 -> 2.110 ms at 256^3,
    // four 2.928 -> 2.887; two species ran slower with it, 1.176 -> 1.190).
    int wave_v = wave;
    uint32_t popb_v = pop_bytes;
    // halo ring: the rows / columns around the tile, one site per thread
    int hb = -1, hp0 = 0, hp1 = 0;
    if (tid < NHALO) {
        int h0, h1;
        if (!D3) {
            h0 = tid == 0 ? 0 : H0 - 1;
            h1 = 0;
        } else if (tid < H0) {
            h0 = tid;
            h1 = 0;
        } else if (tid < 2 * H0) {
            h0 = tid - H0;
            h1 = H1 - 1;
        } else {
            const int q = tid - 2 * H0;
            h0 = (q & 1) ? H0 - 1 : 0;
            h1 = 1 + (q >> 1);
        }
        hb = h1 * H0 + h0;
        hp0 = ((t0 * T0 - 1 + h0) % n0 + n0) % n0;
        hp1 = D3 ? ((t1 * T1 - OFF1 + h1) % n1 + n1) % n1 : 0;
    }
    auto slot = [&](int m) { return (m - mbeg + 1) & 3; };
    auto wrapm = [&](int m) { return m < 0 ? m + nm : (m >= nm ? m - nm : m); };
    // byte offset of the site that population i of (q0, q1, m) is pulled from
    auto pull_off = [&](int q0, int q1, int m, int i) __attribute__((always_inline)) -> uint32_t {
        const int x = wrap(q0, -A::c0(i), n0);
        const int y = D3 ? wrap(q1, -A::c1(i), n1) : 0;
        const int z = wrap(m, -A::cm(i), nm);
        return ((uint32_t)x + s1 * (uint32_t)y + sm * (uint32_t)z) * 4u;
    };
    // Register pull (prologue only).
    auto pull = [&](int q0, int q1, int m, Real (&f)[N][Q]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const uint32_t voff = pull_off(q0, q1, m, i);
#pragma unroll
            for (int s = 0; s < N; ++s) f[s][i] = BufIO<float>::load(rsrc[s], voff, (uint32_t)i * pop_bytes);
        }
    };
    // Species s's share of the asynchronous pull of plane m into rows [NQ][len]
    // (this wave's 64-lane slice).
    auto dma1 = [&](int s, int q0, int q1, int m, Raw *rows, int len) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            lds_void_t *dst = (lds_void_t *)(rows + (s * Q + i) * len + wave_v * 64);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc[s], dst, 4, pull_off(q0, q1, m, i), (uint32_t)i * popb_v, 0,
                                                     0);
        }
    };
    auto issue = [&](int s, int m) __attribute__((always_inline)) {
        dma1(s, p0, p1, m, &own[0][0], NT);
        if (tid < NHALO) dma1(s, hp0, hp1, m, &halo[0][0], NHALO);
    };
    // The pulls of every species whose phase (multi_pull_phase) is ph.
    auto issue_phase = [&](auto ph, int m) __attribute__((always_inline)) {
        static_for<N>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            if constexpr (multi_pull_phase<N>(t) == decltype(ph)::value) issue(t, m);
        });
    };
    auto read_rows = [&](const Raw *rows, int len, Real (&f)[N][Q]) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < N; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) f[s][i] = __builtin_bit_cast(float, rows[(s * Q + i) * len + tid]);
    };
    auto put_phi = [&](int m, int box, const Real (&f)[N][Q]) __attribute__((always_inline)) {
        Real phi[N];
        multi_potential<L, float, N>(a.ph, f, phi);
#pragma unroll
        for (int s = 0; s < N; ++s) ring[slot(m)][s][box] = phi[s];
    };

    Real cur[N][Q];
    // Prologue: potentials of planes mbeg-1 and mbeg and the populations of
    // plane mbeg (register pulls), then the asynchronous pull of plane mbeg+1.
#pragma unroll 1
    for (int m = mbeg - 1; m <= mbeg; ++m) {
        if (hb >= 0) {
            Real h[N][Q];
            pull(hp0, hp1, wrapm(m), h);
            put_phi(m, hb, h);
        }
        Real f[N][Q];
        pull(p0, p1, wrapm(m), f);
        put_phi(m, box_own, f);
        if (m == mbeg) {
#pragma unroll
            for (int s = 0; s < N; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[s][i] = f[s][i];
        }
    }
#pragma unroll
    for (int s = 0; s < N; ++s) issue(s, wrapm(mbeg + 1));

#pragma unroll 1
    for (int m = mbeg; m < mend; ++m) {
        if constexpr (N >= 3) asm volatile("" : "+s"(wave_v), "+s"(popb_v));
        // Rows of plane m+1 have landed.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        Real nxt[N][Q];
        read_rows(&own[0][0], NT, nxt);
        put_phi(m + 1, box_own, nxt);
        if (hb >= 0) {
            Real h[N][Q];
            read_rows(&halo[0][0], NHALO, h);
            put_phi(m + 1, hb, h);
        }
        // This wave's rows are read back: the pulls of plane m+2 due at the top.
        if constexpr (multi_phase_used<N>(0)) {
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
            __builtin_amdgcn_sched_barrier(0);
            if (m + 2 <= mend) issue_phase(std::integral_constant<int, 0>{}, wrapm(m + 2));
            __builtin_amdgcn_sched_barrier(0);
        }
        // Workgroup barrier for the potential ring only: the ring writes are
        // complete once lgkmcnt drains (row loads in flight write only this
        // wave's own rows, which no other wave reads).
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);

        Real acc[N][3];
        multi_force<L, Real, N>(
            [&](int i, int s) __attribute__((always_inline)) -> Real {
                return ring[slot(m + A::cm(i))][s][box_own + A::c1(i) * H0 + A::c0(i)];
            },
            acc);
        // Every LDS read of this iteration is done: the row loads of plane m+2
        // due after the force.
        const bool more = m + 2 <= mend;
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_sched_barrier(0);
        if (more) issue_phase(std::integral_constant<int, 1>{}, wrapm(m + 2));
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t site = (uint32_t)p0 + s1 * (uint32_t)(D3 ? p1 : 0) + sm * (uint32_t)m;
        const uint32_t voff = site * 4u;
        const Counter ctr{site, a.step_lo, a.step_hi};
        multi_collide<L, Real, N>(
            a.ph, cur, acc,
            [&](uint32_t b, uint32_t (&w)[4]) __attribute__((always_inline)) {
                block_words(ctr, b, a.ph.key0, a.ph.key1, w);
            },
            [&](auto sc, auto &fs) __attribute__((always_inline)) {
                constexpr int s = decltype(sc)::value;
                // (with three or more species the fences stay even where
                // nothing is issued: they keep the scheduler from moving work
                // across the species' stores, about 0.5 %)
                if constexpr (N >= 3 || multi_phase_used<N>(2 + s)) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (more) issue_phase(std::integral_constant<int, 2 + s>{}, wrapm(m + 2));
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (inside) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) BufIO<float>::store(fs[i], rdst[s], voff, (uint32_t)i * popb_v);
                }
            });
#pragma unroll
        for (int s = 0; s < N; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
    }
}

// Rest state of species s: buf_i(r) = w_i rho(r + c_i) - w_i ref (pull layout).
template <class L, class S>
__global__ __launch_bounds__(256) void multi_init_kernel(S *dst, const double *rho, Geom g, int s, double ref)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xn = wrap(x, L::cx[i], g.nx);
        const int yn = wrap(y, L::cy[i], g.ny);
        const int zn = L::D == 3 ? wrap(z, L::cz[i], g.nz) : 0;
        const size_t nsite = (size_t)xn + (size_t)g.nx * ((size_t)yn + (size_t)g.ny * (size_t)zn);
        store_pop_f64<L, S>(dst, g.pitch, s, i, site, (double)L::w36[i] / 36.0 * rho[nsite], ref);
    }
}

// FP64 rho_s and j_bar_s (D components) of the pre-collision state into
// out[0][sites], out[1 + alpha][sites].
template <class L, class S>
__global__ __launch_bounds__(256) void multi_moment_kernel(const S *src, double *out, Geom g, int s, double ref)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    double r = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap(x, -L::cx[i], g.nx);
        const int ys = wrap(y, -L::cy[i], g.ny);
        const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
        const size_t from = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
        const double v = load_pop_f64<L, S>(src, g.pitch, s, i, from, ref);
        r += v;
        if (L::cx[i]) j[0] += L::cx[i] > 0 ? v : -v;
        if (L::cy[i]) j[1] += L::cy[i] > 0 ? v : -v;
        if (L::D == 3 && L::cz[i]) j[2] += L::cz[i] > 0 ? v : -v;
    }
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    out[site] = r;
#pragma unroll
    for (int al = 0; al < L::D; ++al) out[(size_t)(1 + al) * g.nsites + site] = j[al];
}

// Block partial sums (FP64) of rho_s and j_bar_s over the sites:
// partial[block][0] = sum rho, partial[block][1 + alpha] = sum j_alpha.
template <class L, class S>
__global__ __launch_bounds__(256) void multi_sums_kernel(const S *src, double *partial, Geom g, int s, double ref)
{
    __shared__ double red[4][256];
    double v[4] = {0, 0, 0, 0};
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < g.nsites; t += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(t % (size_t)g.nx);
        const size_t rr = t / (size_t)g.nx;
        const int y = (int)(rr % (size_t)g.ny);
        const int z = (int)(rr / (size_t)g.ny);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int xs = wrap(x, -L::cx[i], g.nx);
            const int ys = wrap(y, -L::cy[i], g.ny);
            const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
            const size_t from = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
            const double f = load_pop_f64<L, S>(src, g.pitch, s, i, from, ref);
            v[0] += f;
            if (L::cx[i]) v[1] += L::cx[i] > 0 ? f : -f;
            if (L::cy[i]) v[2] += L::cy[i] > 0 ? f : -f;
            if (L::D == 3 && L::cz[i]) v[3] += L::cz[i] > 0 ? f : -f;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) partial[(size_t)blockIdx.x * 4 + q] = red[q][0];
}

}  // namespace fmlb
