// Fused single-pass FLBE step: pull-stream + moments + lattice force + noise
// + collision + store, one read and one write of every population.
//
// The lattice force of Eq. (87) needs the densities of the same time level at
// the neighbours r + c_i, and those depend on the neighbours' own pulled
// populations.  Each workgroup therefore owns a tile of T0 x T1 columns of the
// plane orthogonal to the march axis (z for D3Q19, y for D2Q9) and walks a
// chunk of planes.  For plane m+1 it pulls the populations of its tile (kept
// in registers, with their moments, for the next iteration) and of a one-site
// halo ring around the tile (densities only), and writes both densities into
// a 4-slot LDS ring of planes; after one barrier it collides plane m with the
// densities of planes m-1, m, m+1.  Four slots make one barrier per plane
// sufficient: the slot written for plane m+1 was last read while plane m-2
// was collided.
//
// The densities are produced by the same moments() and the force by the same
// lattice_acceleration() as the two-pass form, so both forms give the same
// bits.  The halo recomputation costs extra (mostly L2-resident) loads, not
// HBM traffic: every population is still fetched from HBM about once.
//
// Memory is addressed through one buffer resource per species and array
// (32-bit per-lane offsets, uniform per-population offsets), which keeps the
// address arithmetic off the vector ALU.  The fused form is used when a
// species' array fits in 4 GiB; larger lattices run the two-pass form.
//
// Workgroups are numbered so that the 8 XCDs (which take workgroups round
// robin) each receive a contiguous range of tiles; neighbouring tiles then
// share one L2 and the halo loads hit it.
#pragma once

#include <type_traits>
#include <utility>

#include "kernels.h"

namespace fmlb {

// Raw buffer access per storage type (values are bit patterns on the wire).
// Stores carry the non-temporal hint (cache-policy bit 1) by default: the
// populations written now are read only in the next step, so they should not
// evict the lines the neighbouring tiles are about to re-read for their halo
// densities (measured on 256^3 D3Q19: 23 % -> 9 % of re-fetched bytes, 4 %
// faster).  Lattices whose state fits the last-level cache store without it
// (launch_fused_shape).
constexpr int kBufferWord3 = 0x00020000;
constexpr int kStoreNonTemporal = 2;

template <class S>
struct BufIO;

template <>
struct BufIO<float> {
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
    template <int CPOL = kStoreNonTemporal>
    __device__ static void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, CPOL);
    }
};

template <>
struct BufIO<__hip_bfloat16> {
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
        return __builtin_bit_cast(float, (uint32_t)b << 16);
    }
    template <int CPOL = kStoreNonTemporal>
    __device__ static void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        const __hip_bfloat16 h = __float2bfloat16(v);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h), r, voff, soff, CPOL);
    }
};

template <>
struct BufIO<__half> {
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
        return __half2float(__ushort_as_half(b));
    }
    template <int CPOL = kStoreNonTemporal>
    __device__ static void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, voff, soff, CPOL);
    }
};

// Stochastic-rounding formats: the same 16-bit words, stored with a hash
// offset (storage.h).
template <>
struct BufIO<bf16_sr> {
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return BufIO<__hip_bfloat16>::load(r, voff, soff);
    }
    template <int CPOL = kStoreNonTemporal>
    __device__ static void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t h)
    {
        __builtin_amdgcn_raw_buffer_store_b16(bf16_bits_sr(v, h), r, voff, soff, CPOL);
    }
};

template <>
struct BufIO<f16_sr> {
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return BufIO<__half>::load(r, voff, soff);
    }
    template <int CPOL = kStoreNonTemporal>
    __device__ static void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t h)
    {
        __builtin_amdgcn_raw_buffer_store_b16(f16_bits_sr(v, h), r, voff, soff, CPOL);
    }
};

// Store population sp_pop (= species * Q + i) of a site after the step with
// counter `step`: round to nearest, or stochastically for the _sr formats;
// CPOL is the stores' cache policy.
template <class S, int CPOL = kStoreNonTemporal>
__device__ __forceinline__ void store_stepped(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                              uint32_t site, uint32_t sp_pop, uint32_t step, uint32_t k0, uint32_t k1)
{
    if constexpr (Storage<S>::stochastic)
        BufIO<S>::template store<CPOL>(v, r, voff, soff, sr_bits(site, sp_pop, step, k0, k1));
    else
        BufIO<S>::template store<CPOL>(v, r, voff, soff);
}

template <class L>
struct MarchAxes {
    static constexpr bool three_d = L::D == 3;
    // velocity components along plane axis 0 (x), plane axis 1 (y, 3D only)
    // and the march axis (z in 3D, y in 2D)
    static constexpr int c0(int i) { return L::cx[i]; }
    static constexpr int c1(int i) { return three_d ? L::cy[i] : 0; }
    static constexpr int cm(int i) { return three_d ? L::cz[i] : L::cy[i]; }
};

// Workgroup position -> tile number with the 8 XCDs (which take workgroups
// round robin) each given a contiguous range of tiles.
__device__ __forceinline__ unsigned xcd_contiguous(unsigned b, unsigned nblk)
{
    const unsigned per_xcd = (nblk + 7) / 8;
    const unsigned xcd = b % 8, k = b / 8;
    const unsigned full = nblk % 8 == 0 ? 8 : nblk % 8;  // XCDs that get per_xcd blocks
    return xcd < full ? xcd * per_xcd + k : full * per_xcd + (xcd - full) * (per_xcd - 1) + k;
}

// One workgroup's share of the fused step: tile (t0, t1) of the plane, planes
// [mbeg, mend) of the march axis.
template <class L, class S, int T0, int T1>
__device__ __forceinline__ void fused_tile(const StepArgs<L, S> &a, int t0, int t1, int mbeg, int mend)
{
    using Real = typename Storage<S>::Real;
    using A = MarchAxes<L>;
    constexpr int Q = L::Q;
    constexpr bool D3 = A::three_d;
    constexpr int H0 = T0 + 2;
    constexpr int H1 = D3 ? T1 + 2 : 1;
    constexpr int OFF1 = D3 ? 1 : 0;
    constexpr int PLANE = H0 * H1;
    constexpr int NT = T0 * T1;
    constexpr int NHALO = PLANE - NT;
    constexpr uint32_t ES = sizeof(S);
    static_assert(D3 || T1 == 1, "2D tiles are one row");
    static_assert(NHALO <= NT, "halo ring larger than the tile");

    __shared__ Real ring[4][2][PLANE];

    const Geom g = a.g;
    const int n0 = g.nx, n1 = D3 ? g.ny : 1, nm = D3 ? g.nz : g.ny;
    const uint32_t s1 = (uint32_t)n0;                          // site stride along plane axis 1
    const uint32_t sm = D3 ? (uint32_t)n0 * n1 : (uint32_t)n0;  // site stride along the march axis
    const uint32_t pop_bytes = (uint32_t)g.pitch * ES;         // one population array

    __amdgpu_buffer_rsrc_t rsrc[2], rdst[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rsrc[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.src + (size_t)s * Q * g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
        rdst[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.dst + (size_t)s * Q * g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
    }

    const int tid = threadIdx.x;
    const int l0 = tid % T0, l1 = tid / T0;
    const int p0raw = t0 * T0 + l0, p1raw = t1 * T1 + l1;
    const bool inside = p0raw < n0 && p1raw < n1;
    const int p0 = p0raw % n0, p1 = p1raw % n1;  // periodic image for ragged tiles
    const int box_own = (l1 + OFF1) * H0 + (l0 + 1);

    // Halo ring position of this thread (tid < NHALO): border of the H0 x H1 box.
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

    // reference density of the stored deviations (0 for absolute storage)
    const Real ref[2] = {Storage<S>::deviation ? a.ref[0] : Real(0), Storage<S>::deviation ? a.ref[1] : Real(0)};
    auto slot = [&](int m) { return (m - mbeg + 1) & 3; };

    // Pull the 2Q populations of plane-site (q0, q1) on plane m (m wrapped).
    auto pull = [&](int q0, int q1, int m, Real (&f)[2][Q]) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int x = wrap(q0, -A::c0(i), n0);
            const int y = D3 ? wrap(q1, -A::c1(i), n1) : 0;
            const int z = wrap(m, -A::cm(i), nm);
            const uint32_t voff = ((uint32_t)x + s1 * (uint32_t)y + sm * (uint32_t)z) * ES;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Real v = BufIO<S>::load(rsrc[s], voff, (uint32_t)i * pop_bytes);
                f[s][i] = v;
            }
        }
    };
    auto wrapm = [&](int m) { return m < 0 ? m + nm : (m >= nm ? m - nm : m); };

    Real cur[2][Q], rc[2], jc[2][3];
    // Prologue: densities of plane mbeg-1, populations and moments of plane mbeg.
#pragma unroll 1
    for (int m = mbeg - 1; m <= mbeg; ++m) {
        Real r, j[3];
        if (hb >= 0) {
            Real h[2][Q];
            pull(hp0, hp1, wrapm(m), h);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                moments<L, Real>(h[s], r, j);
                ring[slot(m)][s][hb] = r;
            }
        }
        Real f[2][Q];
        pull(p0, p1, wrapm(m), f);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<L, Real>(f[s], r, j);
            ring[slot(m)][s][box_own] = r;
            if (m == mbeg) {
                rc[s] = r;
#pragma unroll
                for (int al = 0; al < 3; ++al) jc[s][al] = j[al];
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[s][i] = f[s][i];
            }
        }
    }

#pragma unroll 1
    for (int m = mbeg; m < mend; ++m) {
        // Plane m+1: halo densities, then own populations and moments (kept).
        const int mn = wrapm(m + 1);
        if (hb >= 0) {
            Real h[2][Q];
            pull(hp0, hp1, mn, h);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Real r, j[3];
                moments<L, Real>(h[s], r, j);
                ring[slot(m + 1)][s][hb] = r;
            }
        }
        Real nxt[2][Q], rn[2], jn[2][3];
        pull(p0, p1, mn, nxt);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<L, Real>(nxt[s], rn[s], jn[s]);
            ring[slot(m + 1)][s][box_own] = rn[s];
        }
        __syncthreads();

        if (inside) {
            auto nb = [&](int i, int s) -> Real {
                const int sl = slot(m + A::cm(i));
                return ring[sl][s][box_own + A::c1(i) * H0 + A::c0(i)];
            };
            Real acc[2][3];
            lattice_acceleration<L, Real>(nb, a.ph.negG, acc);
            const uint32_t site = (uint32_t)p0 + s1 * (uint32_t)(D3 ? p1 : 0) + sm * (uint32_t)m;
            const uint32_t voff = site * ES;
            collide_site<L, Real>(cur, rc, jc, acc, a.ph, ref, Counter{site, a.step_lo, a.step_hi},
                                  [&](int s, auto &fs) {
#pragma unroll
                                      for (int i = 0; i < Q; ++i) {
                                          Real v = fs[i];
                                          store_stepped<S>(v, rdst[s], voff, (uint32_t)i * pop_bytes, site,
                                                           (uint32_t)(s * Q + i), a.step_lo, a.ph.key0, a.ph.key1);
                                      }
                                  });
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            rc[s] = rn[s];
#pragma unroll
            for (int al = 0; al < 3; ++al) jc[s][al] = jn[s][al];
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
        }
    }
}

// ---------------------------------------------------------------------------
// Asynchronous form of the same tile walk.  The pulls of plane m+2 go straight
// from memory into LDS (buffer loads with the LDS destination bit, one 64-lane
// row per instruction, no VGPRs held while in flight) and are issued before
// the collision of plane m, so their latency hides behind the collision
// instead of stalling the wave; the register form above waits for plane m+1
// before it can collide plane m.  Each wave reads back only the rows its own
// loads wrote, so these rows need only the wave's own counters.  Own rows
// of plane m+2 are requested once all of the wave's LDS reads of the
// iteration (rows of plane m+1, the density ring) have completed, halo rows
// after the species-1 stores; no LDS read follows until the top of the next
// iteration, where vmcnt(0) guarantees both have landed (loads and stores
// share that counter and may complete out of order).
// The density ring is the only LDS shared between waves; its barrier waits
// for LDS traffic only.
// Lanes outside the lattice (ragged tiles) collide their periodic image like
// the register form but never store.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

// Row element of the asynchronous pulls.  An LDS-destination buffer load
// writes lane l's data at LDS base + 4 l whatever its width, so every row
// slot is a dword; 16-bit formats use its low half.
template <class S>
struct DmaWord;

template <>
struct DmaWord<float> {
    __device__ static float decode(uint32_t r) { return __builtin_bit_cast(float, r); }
};

template <>
struct DmaWord<__hip_bfloat16> {
    __device__ static float decode(uint32_t r) { return __builtin_bit_cast(float, r << 16); }
};

template <>
struct DmaWord<__half> {
    __device__ static float decode(uint32_t r) { return __half2float(__ushort_as_half((unsigned short)r)); }
};

template <>
struct DmaWord<bf16_sr> : DmaWord<__hip_bfloat16> {
};

template <>
struct DmaWord<f16_sr> : DmaWord<__half> {
};

// s_waitcnt immediates (gfx9 layout: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8],
// vmcnt[5:4] in [15:14]); counters not named are left unconstrained.
constexpr int kWaitVm0 = (0x7 << 4) | (0xf << 8);
constexpr int kWaitLgkm0 = 0xf | (0x7 << 4) | (0x3 << 14);

template <class L, class S, int T0, int T1, int CPOL = kStoreNonTemporal>
__device__ __forceinline__ void fused_tile_async(const StepArgs<L, S> &a, int t0, int t1, int mbeg, int mend)
{
    using Real = typename Storage<S>::Real;
    using Raw = uint32_t;
    using A = MarchAxes<L>;
    constexpr int Q = L::Q;
    constexpr bool D3 = A::three_d;
    constexpr int H0 = T0 + 2;
    constexpr int H1 = D3 ? T1 + 2 : 1;
    constexpr int OFF1 = D3 ? 1 : 0;
    constexpr int PLANE = H0 * H1;
    constexpr int NT = T0 * T1;
    constexpr int NHALO = PLANE - NT;
    constexpr uint32_t ES = sizeof(S);
    static_assert(D3 || T1 == 1, "2D tiles are one row");
    static_assert(NHALO <= NT, "halo ring larger than the tile");
    static_assert(NT % 64 == 0, "whole waves");

    __shared__ Real ring[4][2][PLANE];
    __shared__ Raw own[2 * Q][NT];      // plane m+1 (then m+2) populations of the tile
    __shared__ Raw halo[2 * Q][NHALO];  // same for the halo ring

    const Geom g = a.g;
    const int n0 = g.nx, n1 = D3 ? g.ny : 1, nm = D3 ? g.nz : g.ny;
    const uint32_t s1 = (uint32_t)n0;
    const uint32_t sm = D3 ? (uint32_t)n0 * n1 : (uint32_t)n0;
    const uint32_t pop_bytes = (uint32_t)g.pitch * ES;

    __amdgpu_buffer_rsrc_t rsrc[2], rdst[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rsrc[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.src + (size_t)s * Q * g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
        rdst[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.dst + (size_t)s * Q * g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
    }

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // Copies of the wave number and the population stride that the plane loop
    // marks as changed: the LDS destinations and population offsets of the
    // per-lane row pulls and the stores' offsets are then recomputed each
    // plane (one scalar instruction each) instead of being held across the
    // loop, where they did not fit the scalar registers and came back from
    // VGPR lanes (128x4 FP32: 62 v_readlane per plane; 128^3 0.157 -> 0.152
    // ms, 1024^2 D2Q9 0.0360 -> 0.0357).
    int wave_v = wave;
    uint32_t popb_v = pop_bytes;
    const int l0 = tid % T0, l1 = tid / T0;
    const int p0raw = t0 * T0 + l0, p1raw = t1 * T1 + l1;
    const bool inside = p0raw < n0 && p1raw < n1;
    const int p0 = p0raw % n0, p1 = p1raw % n1;
    const int box_own = (l1 + OFF1) * H0 + (l0 + 1);

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

    // reference density of the stored deviations (0 for absolute storage)
    const Real ref[2] = {Storage<S>::deviation ? a.ref[0] : Real(0), Storage<S>::deviation ? a.ref[1] : Real(0)};
    auto slot = [&](int m) { return (m - mbeg + 1) & 3; };
    auto wrapm = [&](int m) { return m < 0 ? m + nm : (m >= nm ? m - nm : m); };
    auto pull_off = [&](int q0, int q1, int m, int i) -> uint32_t {
        const int x = wrap(q0, -A::c0(i), n0);
        const int y = D3 ? wrap(q1, -A::c1(i), n1) : 0;
        const int z = wrap(m, -A::cm(i), nm);
        return ((uint32_t)x + s1 * (uint32_t)y + sm * (uint32_t)z) * ES;
    };
    // Register pull (prologue only).
    auto pull = [&](int q0, int q1, int m, Real (&f)[2][Q]) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const uint32_t voff = pull_off(q0, q1, m, i);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Real v = BufIO<S>::load(rsrc[s], voff, (uint32_t)i * pop_bytes);
                f[s][i] = v;
            }
        }
    };
    // Offsets (in sites) of the source planes m - c_z, c_z = +1, 0, -1, of
    // plane m's pulls, taken once per plane for all of its row pulls (the
    // wrap inside each load's offset cost 50-70 scalar instructions per
    // plane).
    auto src_planes = [&](int m, uint32_t (&zq)[3]) {
        zq[0] = (uint32_t)wrapm(m - 1) * sm;
        zq[1] = (uint32_t)m * sm;
        zq[2] = (uint32_t)wrapm(m + 1) * sm;
    };
    auto pull_off_z = [&](int q0, int q1, const uint32_t (&zq)[3], int i) -> uint32_t {
        const int x = wrap(q0, -A::c0(i), n0);
        const int y = D3 ? wrap(q1, -A::c1(i), n1) : 0;
        return ((uint32_t)x + s1 * (uint32_t)y + zq[1 - A::cm(i)]) * ES;
    };
    // Asynchronous pull of plane m (source planes zq) into rows [2Q][len]: this
    // wave's 64-lane slice.
    auto dma_pull = [&](int q0, int q1, const uint32_t (&zq)[3], Raw *rows, int len) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const uint32_t voff = pull_off_z(q0, q1, zq, i);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                lds_void_t *dst = (lds_void_t *)(rows + (s * Q + i) * len + wave_v * 64);
                if constexpr (ES == 4)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc[s], dst, 4, voff, (uint32_t)i * popb_v, 0, 0);
                else
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc[s], dst, 2, voff, (uint32_t)i * popb_v, 0, 0);
            }
        }
    };
    auto read_rows = [&](const Raw *rows, int len, int idx, Real (&f)[2][Q]) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                Real v = DmaWord<S>::decode(rows[(s * Q + i) * len + idx]);
                f[s][i] = v;
            }
    };

    // One species' share of dma_pull.
    auto dma_pull1 = [&](int s, int q0, int q1, const uint32_t (&zq)[3], Raw *rows, int len) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            lds_void_t *dst = (lds_void_t *)(rows + (s * Q + i) * len + wave_v * 64);
            if constexpr (ES == 4)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc[s], dst, 4, pull_off_z(q0, q1, zq, i), (uint32_t)i * popb_v,
                                                         0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc[s], dst, 2, pull_off_z(q0, q1, zq, i), (uint32_t)i * popb_v,
                                                         0, 0);
        }
    };

    // Issue schedule of the next plane's loads.  A wave has at most 63
    // vector memory operations in flight, shared by loads and stores.  D3Q19:
    // the first species' rows (and halo) after the force, the second
    // species' once the first species is collided, ahead of its stores
    // (measured at 256^3, 16-bit storage, 64x8 tiles: 1.010 -> 0.960 ms per
    // step against all rows after the force and the halo after the first
    // species' stores).  D2Q9 (two halo sites per row) keeps the latter.
    Real cur[2][Q], rc[2], jc[2][3];
    // Prologue: densities of plane mbeg-1, populations and moments of plane
    // mbeg (register pulls), then the asynchronous pull of plane mbeg+1.
#pragma unroll 1
    for (int m = mbeg - 1; m <= mbeg; ++m) {
        Real r, j[3];
        if (hb >= 0) {
            Real h[2][Q];
            pull(hp0, hp1, wrapm(m), h);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                moments<L, Real>(h[s], r, j);
                ring[slot(m)][s][hb] = r;
            }
        }
        Real f[2][Q];
        pull(p0, p1, wrapm(m), f);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<L, Real>(f[s], r, j);
            ring[slot(m)][s][box_own] = r;
            if (m == mbeg) {
                rc[s] = r;
#pragma unroll
                for (int al = 0; al < 3; ++al) jc[s][al] = j[al];
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[s][i] = f[s][i];
            }
        }
    }
    uint32_t zq1[3];
    src_planes(wrapm(mbeg + 1), zq1);
    dma_pull(p0, p1, zq1, &own[0][0], NT);
    if (tid < NHALO) dma_pull(hp0, hp1, zq1, &halo[0][0], NHALO);

#pragma unroll 1
    for (int m = mbeg; m < mend; ++m) {
        asm volatile("" : "+s"(wave_v), "+s"(popb_v));
        // Rows of plane m+1 have landed.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        Real nxt[2][Q], rn[2], jn[2][3];
        read_rows(&own[0][0], NT, tid, nxt);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<L, Real>(nxt[s], rn[s], jn[s]);
            ring[slot(m + 1)][s][box_own] = rn[s];
        }
        if (hb >= 0) {
            Real h[2][Q];
            read_rows(&halo[0][0], NHALO, tid, h);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Real r, j[3];
                moments<L, Real>(h[s], r, j);
                ring[slot(m + 1)][s][hb] = r;
            }
        }
        // Workgroup barrier for the density ring only: the ring writes are
        // complete once lgkmcnt drains (no row loads are in flight here).
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);

        auto nb = [&](int i, int s) -> Real {
            const int sl = slot(m + A::cm(i));
            return ring[sl][s][box_own + A::c1(i) * H0 + A::c0(i)];
        };
        Real acc[2][3];
        lattice_acceleration<L, Real>(nb, a.ph.negG, acc);
        // Every LDS read of this iteration is done: start the row loads of
        // plane m+2 (no LDS read may follow them before the next vmcnt(0)).
        const bool more = m + 2 <= mend;
        uint32_t zq[3];
        src_planes(wrapm(m + 2), zq);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_sched_barrier(0);
        if (more) {
            if constexpr (D3) {
                dma_pull1(0, p0, p1, zq, &own[0][0], NT);
                if (tid < NHALO) dma_pull1(0, hp0, hp1, zq, &halo[0][0], NHALO);
            } else {
                dma_pull(p0, p1, zq, &own[0][0], NT);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t site = (uint32_t)p0 + s1 * (uint32_t)(D3 ? p1 : 0) + sm * (uint32_t)m;
        const uint32_t voff = site * ES;
        collide_site<L, Real>(cur, rc, jc, acc, a.ph, ref, Counter{site, a.step_lo, a.step_hi}, [&](int s, auto &fs) {
            if constexpr (D3) {
                if (s == 0) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (more) {
                        dma_pull1(1, p0, p1, zq, &own[0][0], NT);
                        if (tid < NHALO) dma_pull1(1, hp0, hp1, zq, &halo[0][0], NHALO);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (inside) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    Real v = fs[i];
                    store_stepped<S, CPOL>(v, rdst[s], voff, (uint32_t)i * popb_v, site, (uint32_t)(s * Q + i),
                                     a.step_lo, a.ph.key0, a.ph.key1);
                }
            }
            if constexpr (!D3) {
                if (s == 0 && more && tid < NHALO) {
                    __builtin_amdgcn_sched_barrier(0);
                    dma_pull(hp0, hp1, zq, &halo[0][0], NHALO);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        });
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            rc[s] = rn[s];
#pragma unroll
            for (int al = 0; al < 3; ++al) jc[s][al] = jn[s][al];
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
        }
    }
}

// ---------------------------------------------------------------------------
// Layout of the 16-byte row pulls of the full-width tiles.  A wave owns 64
// consecutive sites x0 .. x0+63 of one lattice row; population i of that
// slice is pulled from x0 - c_x(i) .. x0 + 63 - c_x(i), which the aligned
// 16-byte chunks (EPC elements each) from x0 - EPC (c_x = +1) or x0 cover in
// 64 / EPC + 1 chunks (64 / EPC when c_x = 0).  The chunks of all 2Q
// populations are packed 64 to a load instruction (lane l of instruction j
// lands at 16 l bytes into that instruction's 1 KB of the wave's LDS
// region), with the populations grouped by their shift c_z along the march
// axis so that every instruction has one z offset, uniform across the wave
// (group 0: c_z = +1, 1: c_z = 0, 2: c_z = -1; each group starts a new
// instruction).  Within a group: species 1's populations, then species 2's,
// in velocity order.
// ---------------------------------------------------------------------------
template <class L, int ES>
struct WideRows {
    static constexpr int EPC = 16 / ES;  // elements per chunk
    static constexpr int Q = L::Q;
    static constexpr int NPOP = 2 * Q;
    static constexpr int group_of(int i) { return 1 - L::cz[i]; }
    static constexpr int chunks_of(int i) { return 64 / EPC + (L::cx[i] != 0 ? 1 : 0); }
    // element offset of site lane 0's source within the population's chunks
    static constexpr int shift_of(int i) { return L::cx[i] > 0 ? EPC - 1 : (L::cx[i] < 0 ? 1 : 0); }
    int gchunks[3];    // chunks of each group
    int first[3];      // first instruction of each group
    int ninstr[3];
    int NI;            // instructions in all
    int chunk0[NPOP];  // first chunk of population s * Q + i within the wave region
    constexpr WideRows() : gchunks(), first(), ninstr(), NI(0), chunk0()
    {
        for (int G = 0; G < 3; ++G) {
            first[G] = NI;
            int c = 0;
            for (int sp = 0; sp < 2; ++sp)
                for (int i = 0; i < Q; ++i)
                    if (group_of(i) == G) {
                        chunk0[sp * Q + i] = 64 * first[G] + c;
                        c += chunks_of(i);
                    }
            gchunks[G] = c;
            ninstr[G] = (c + 63) / 64;
            NI += ninstr[G];
        }
    }
    // instruction j's group, and the number of its lanes that carry a chunk
    constexpr int group_of_instr(int j) const { return j < first[1] ? 0 : (j < first[2] ? 1 : 2); }
    constexpr int lanes_of_instr(int j) const
    {
        const int G = group_of_instr(j);
        const int left = gchunks[G] - 64 * (j - first[G]);
        return left < 64 ? left : 64;
    }
};

// ---------------------------------------------------------------------------
// Full-width tiles (D3Q19, tile width = nx): every row of the tile is a whole
// lattice row, so each population is read as contiguous nx-site rows and the
// x halo is the tile's own periodic image (written into the ring's edge
// columns, no loads).  The halo is then just the rows y0 - 1 and y0 + T1, one
// site per thread.  With 16-bit storage their populations take the same
// 16-byte row pulls as the tile's own rows, into a second LDS region
// (158 KB in all); with FP32 they are pulled into registers, since a second
// region would not fit the CU's 160 KB.  Ordering as in fused_tile_async.
//
// The density ring and the row buffer come in as distinct __restrict__
// pointers: after inlining, the compiler then knows that the ring's LDS
// accesses cannot touch the rows that a buffer-to-LDS load in flight is
// writing, and it does not make them wait for that load.
// ---------------------------------------------------------------------------
template <class L, class S, int T0, int T1>
__device__ __forceinline__ void fused_tile_rows_body(const StepArgs<L, S> &a, int t0, int t1, int mbeg, int mend,
                                                     typename Storage<S>::Real *__restrict__ ring_p,
                                                     uint32_t *__restrict__ own_p, uint32_t *__restrict__ hown_p,
                                                     uint32_t *__restrict__ tab_p)
{
    using Real = typename Storage<S>::Real;
    using A = MarchAxes<L>;
    constexpr int Q = L::Q;
    constexpr bool D3 = A::three_d;
    constexpr int H0 = T0 + 2;
    constexpr int H1 = D3 ? T1 + 2 : 1;
    constexpr int OFF1 = D3 ? 1 : 0;
    constexpr int PLANE = H0 * H1;
    constexpr int NT = T0 * T1;
    constexpr int NHALO = 2 * T0;  // rows y-1 and y+T1; the x halo is the tile's own periodic image
    constexpr uint32_t ES = sizeof(S);
    static_assert(D3 || T1 == 1, "2D tiles are one row");
    static_assert(D3 && NHALO <= NT, "full-width tiles: D3Q19, at least two rows");
    static_assert(NT % 64 == 0, "whole waves");

    auto ring = reinterpret_cast<Real (*)[2][PLANE]>(ring_p);  // [4][2][PLANE]
    // own_p: per wave NI x 1 KB of 16-byte row chunks (WideRows), plane m+1 (then m+2)
    constexpr WideRows<L, ES> W{};
    constexpr int NI = W.NI;

    const Geom g = a.g;
    const int n0 = g.nx, n1 = D3 ? g.ny : 1, nm = D3 ? g.nz : g.ny;
    const uint32_t s1 = (uint32_t)n0;
    const uint32_t sm = D3 ? (uint32_t)n0 * n1 : (uint32_t)n0;
    const uint32_t pop_bytes = (uint32_t)g.pitch * ES;

    __amdgpu_buffer_rsrc_t rsrc[2], rdst[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rsrc[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.src + (size_t)s * Q * g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
        rdst[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.dst + (size_t)s * Q * g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
    }

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l0 = tid % T0, l1 = tid / T0;
    const int p0raw = t0 * T0 + l0, p1raw = t1 * T1 + l1;
    const bool inside = p0raw < n0 && p1raw < n1;
    const int p0 = p0raw % n0, p1 = p1raw % n1;
    const int box_own = (l1 + OFF1) * H0 + (l0 + 1);
    const int lane = tid & 63;

    // One buffer resource over both species for the 16-byte row pulls (the
    // launcher requires 2 Q sites ES < 4 GiB for full-width tiles), and the
    // per-lane source offsets of every row-pull instruction (population,
    // x and y parts), fixed over the march and kept in LDS (tab_p); the
    // plane enters as the scalar offset of the instruction's group.
    const __amdgpu_buffer_rsrc_t rall =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.src, 0, (int)(2u * Q * pop_bytes), kBufferWord3);
    {
        const int x0 = (wave % (T0 / 64)) * 64;
        const int yc[3] = {wrap(p1, -1, n1), p1, wrap(p1, 1, n1)};  // rows p1 - c_y for c_y = +1, 0, -1
        static_for<NI>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            constexpr int G = W.group_of_instr(j);
            const int gc = 64 * (j - W.first[G]) + lane;  // chunk within the group
            // the group's populations occupy consecutive chunk ranges: keep the
            // last one that starts at or before gc (selects, no branches)
            int c0 = 0, cb = 0, y = p1;
            uint32_t pop = 0;
            static_for<2 * Q>([&](auto pc) {
                constexpr int sp = decltype(pc)::value / Q, i = decltype(pc)::value % Q;
                if constexpr (WideRows<L, ES>::group_of(i) == G) {
                    constexpr int start = W.chunk0[sp * Q + i] - 64 * W.first[G];
                    const bool here = gc >= start;
                    c0 = here ? start : c0;
                    cb = here ? (A::c0(i) > 0 ? -W.EPC : 0) : cb;
                    y = here ? yc[1 - A::c1(i)] : y;
                    pop = here ? (uint32_t)(sp * Q + i) * pop_bytes : pop;
                }
            });
            int x = x0 + cb + W.EPC * (gc - c0);
            x = x < 0 ? x + n0 : (x >= n0 ? x - n0 : x);
            tab_p[(wave * NI + j) * 64 + lane] = pop + ((uint32_t)x + s1 * (uint32_t)y) * ES;
        });
    }

    // put(j, offset) for every row-pull instruction j of the wave's slice of
    // lattice row prow: the same offsets as the table above, for the 16-bit
    // halo rows (the own rows keep the code above: routed through this lambda
    // they changed the register allocation of the FP32 kernel)
    auto row_offsets = [&](int prow, auto &&put) {
        const int x0 = (wave % (T0 / 64)) * 64;
        const int yc[3] = {wrap(prow, -1, n1), prow, wrap(prow, 1, n1)};  // rows prow - c_y for c_y = +1, 0, -1
        static_for<NI>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            constexpr int G = W.group_of_instr(j);
            const int gc = 64 * (j - W.first[G]) + lane;  // chunk within the group
            // the group's populations occupy consecutive chunk ranges: keep the
            // last one that starts at or before gc (selects, no branches)
            int c0 = 0, cb = 0, y = prow;
            uint32_t pop = 0;
            static_for<2 * Q>([&](auto pc) {
                constexpr int sp = decltype(pc)::value / Q, i = decltype(pc)::value % Q;
                if constexpr (WideRows<L, ES>::group_of(i) == G) {
                    constexpr int start = W.chunk0[sp * Q + i] - 64 * W.first[G];
                    const bool here = gc >= start;
                    c0 = here ? start : c0;
                    cb = here ? (A::c0(i) > 0 ? -W.EPC : 0) : cb;
                    y = here ? yc[1 - A::c1(i)] : y;
                    pop = here ? (uint32_t)(sp * Q + i) * pop_bytes : pop;
                }
            });
            int x = x0 + cb + W.EPC * (gc - c0);
            x = x < 0 ? x + n0 : (x >= n0 ? x - n0 : x);
            put(jc, pop + ((uint32_t)x + s1 * (uint32_t)y) * ES);
        });
    };

    // halo: the two rows y0 - 1 and y0 + T1, one site per thread
    const int hrow = tid / T0, hx = tid % T0;
    const int hh1 = hrow == 0 ? 0 : H1 - 1;
    const int hb = hh1 * H0 + hx + 1;
    const int hp0 = hx;
    const int hp1 = ((t1 * T1 - 1 + (hrow == 0 ? 0 : T1 + 1)) % n1 + n1) % n1;
    // 16-bit storage pulls the halo rows like the own rows, into hown_p, with
    // their per-lane offsets in registers (FP32 pulls them into registers:
    // the LDS of a 256x2 FP32 tile has no room for their rows)
    uint32_t htab[NI];
    if constexpr (ES == 2) row_offsets(hp1, [&](auto jc, uint32_t v) { htab[decltype(jc)::value] = v; });
    // ring positions of the periodic x images (columns -1 and T0)
    // (second store: the periodic image, or the same cell again)
    auto put_ring = [&](float *row_plane, int box, int lx, float v) {
        row_plane[box] = v;
        row_plane[lx == 0 ? box + T0 : (lx == T0 - 1 ? box - T0 : box)] = v;
    };

    // reference density of the stored deviations (0 for absolute storage)
    const Real ref[2] = {Storage<S>::deviation ? a.ref[0] : Real(0), Storage<S>::deviation ? a.ref[1] : Real(0)};
    auto slot = [&](int m) { return (m - mbeg + 1) & 3; };
    auto wrapm = [&](int m) { return m < 0 ? m + nm : (m >= nm ? m - nm : m); };
    auto pull_off = [&](int q0, int q1, int m, int i) -> uint32_t {
        const int x = wrap(q0, -A::c0(i), n0);
        const int y = D3 ? wrap(q1, -A::c1(i), n1) : 0;
        const int z = wrap(m, -A::cm(i), nm);
        return ((uint32_t)x + s1 * (uint32_t)y + sm * (uint32_t)z) * ES;
    };
    // Register pull (prologue only).
    auto pull = [&](int q0, int q1, int m, Real (&f)[2][Q]) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const uint32_t voff = pull_off(q0, q1, m, i);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Real v = BufIO<S>::load(rsrc[s], voff, (uint32_t)i * pop_bytes);
                f[s][i] = v;
            }
        }
    };
    // The 16-byte row pulls of plane m (wrapped), instructions [jb, je): group
    // G's source plane is m - c_z = m - 1, m, m + 1 for G = 0, 1, 2.
    auto wide_issue = [&](int m, auto jb, auto je) {
        const uint32_t zo[3] = {(uint32_t)wrapm(m - 1) * sm * ES, (uint32_t)m * sm * ES,
                                (uint32_t)wrapm(m + 1) * sm * ES};
        lds_void_t *base = (lds_void_t *)(own_p + wave * NI * 256);
        static_for<NI>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (j >= decltype(jb)::value && j < decltype(je)::value) {
                lds_void_t *dst = (lds_void_t *)((__attribute__((address_space(3))) unsigned char *)base + j * 1024);
                const uint32_t voff = tab_p[(wave * NI + j) * 64 + lane];
                constexpr int lanes = W.lanes_of_instr(j);
                if (lanes == 64 || lane < lanes)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rall, dst, 16, voff, zo[W.group_of_instr(j)], 0, 0);
            }
        });
    };
    // The 16-byte pulls of the halo rows of plane m (16-bit storage),
    // instructions [jb, je).
    auto halo_issue = [&](int m, auto jb, auto je) {
        const uint32_t zo[3] = {(uint32_t)wrapm(m - 1) * sm * ES, (uint32_t)m * sm * ES,
                                (uint32_t)wrapm(m + 1) * sm * ES};
        lds_void_t *base = (lds_void_t *)(hown_p + wave * NI * 256);
        static_for<NI>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (j >= decltype(jb)::value && j < decltype(je)::value) {
                lds_void_t *dst = (lds_void_t *)((__attribute__((address_space(3))) unsigned char *)base + j * 1024);
                constexpr int lanes = W.lanes_of_instr(j);
                if (lanes == 64 || lane < lanes)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rall, dst, 16, htab[j], zo[W.group_of_instr(j)], 0, 0);
            }
        });
    };
    // Density deviations of this thread's halo site, from the wave's halo chunks.
    auto halo_read = [&](Real (&r)[2]) {
        const unsigned short *h = reinterpret_cast<const unsigned short *>(hown_p);
        Real f[2][Q], j[3];
        static_for<2 * Q>([&](auto pc) {
            constexpr int sp = decltype(pc)::value / Q, i = decltype(pc)::value % Q;
            constexpr int e = W.EPC * W.chunk0[sp * Q + i] + WideRows<L, ES>::shift_of(i);
            f[sp][i] = DmaWord<S>::decode(h[wave * NI * 512 + e + lane]);
        });
#pragma unroll
        for (int s = 0; s < 2; ++s) moments<L, Real>(f[s], r[s], j);
    };
    // Read back this thread's 2Q pre-collision populations from the wave's chunks.
    auto wide_read = [&](Real (&f)[2][Q]) {
        static_for<2 * Q>([&](auto pc) {
            constexpr int sp = decltype(pc)::value / Q, i = decltype(pc)::value % Q;
            constexpr int e = W.EPC * W.chunk0[sp * Q + i] + WideRows<L, ES>::shift_of(i);
            if constexpr (ES == 4) {
                f[sp][i] = DmaWord<S>::decode(own_p[wave * NI * 256 + e + lane]);
            } else {
                const unsigned short *h = reinterpret_cast<const unsigned short *>(own_p);
                f[sp][i] = DmaWord<S>::decode(h[wave * NI * 512 + e + lane]);
            }
        });
    };
    // instructions issued at the top of a plane; the rest mid-collision
    using J0 = std::integral_constant<int, 0>;
    using JE = std::integral_constant<int, (NI + 1) / 2>;
    using JN = std::integral_constant<int, NI>;
    // 16-bit halo pulls: instructions [0, JH) after the force, [JH, NI) with
    // the second half of the row pulls (stochastic rounding, with more work
    // in the stores, issues fewer before the collision)
    using JH = std::integral_constant<int, Storage<S>::stochastic ? NI / 2 : (NI + 1) / 2>;

    // Register pull of one species' halo site (FP32).
    auto pull1 = [&](int s, int q0, int q1, int m, Real (&w)[2][Q]) {
#pragma unroll
        for (int i = 0; i < Q; ++i) w[s][i] = BufIO<S>::load(rsrc[s], pull_off(q0, q1, m, i), (uint32_t)i * pop_bytes);
    };
    // Issue schedule of one plane, FP32 (per thread: 38 row loads into LDS,
    // 38 halo loads into registers, 38 stores).  A wave can have at most 63
    // vector memory operations in flight, and loads and stores share that
    // counter, so issuing all 76 loads at once stalls the wave until the
    // first of them returns, and the wait at the top of the next plane also
    // covers the stores.  The loads are therefore spread over the plane by
    // species: the first species' rows as soon as the wave has read back
    // its rows of plane m+1, its halo before the barrier, the second
    // species' halo after the force, the second species' rows once the
    // first species is collided, ahead of its stores (measured at 256^3
    // FP32: 1.118 -> 1.037 ms per step against issuing all loads together
    // after the force, 1.033 -> 1.018-1.024 with the first rows moved from
    // after the force to the top; other orders were slower).  16-bit storage
    // pulls 7 + 7 row chunks per wave instead (own and halo rows): the first
    // half of the own rows at the top, the first part of the halo rows after
    // the force, the rest of both once the first species is collided; the
    // halo rows are read back at the top (256^3 BF16: 0.767 -> 0.702 ms per
    // step against the register halo, FP16 0.756 -> 0.703; all halo rows at
    // the top 0.81 ms, all after the force 0.73).
    Real cur[2][Q], rc[2], jc[2][3];
    // Prologue: densities of plane mbeg-1, populations and moments of plane
    // mbeg (register pulls), then the asynchronous pull of plane mbeg+1.
#pragma unroll 1
    for (int m = mbeg - 1; m <= mbeg; ++m) {
        Real r, j[3];
        {
            Real h[2][Q];
            pull(hp0, hp1, wrapm(m), h);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                moments<L, Real>(h[s], r, j);
                put_ring(ring[slot(m)][s], hb, hx, r);
            }
        }
        Real f[2][Q];
        pull(p0, p1, wrapm(m), f);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<L, Real>(f[s], r, j);
            put_ring(ring[slot(m)][s], box_own, l0, r);
            if (m == mbeg) {
                rc[s] = r;
#pragma unroll
                for (int al = 0; al < 3; ++al) jc[s][al] = j[al];
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[s][i] = f[s][i];
            }
        }
    }
    wide_issue(wrapm(mbeg + 1), J0{}, JN{});
    Real hn[2][Q];
    if constexpr (ES == 4)
        pull(hp0, hp1, wrapm(mbeg + 1), hn);
    else
        halo_issue(wrapm(mbeg + 1), J0{}, JN{});

#pragma unroll 1
    for (int m = mbeg; m < mend; ++m) {
        // Rows of plane m+1 have landed.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        Real nxt[2][Q], rn[2], jn[2][3];
        wide_read(nxt);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_sched_barrier(0);
        if (m + 2 <= mend) wide_issue(wrapm(m + 2), J0{}, JE{});
        __builtin_amdgcn_sched_barrier(0);
        Real hr[2];
        if constexpr (ES == 2) halo_read(hr);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<L, Real>(nxt[s], rn[s], jn[s]);
            put_ring(ring[slot(m + 1)][s], box_own, l0, rn[s]);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Real r, j[3];
            if constexpr (ES == 4)
                moments<L, Real>(hn[s], r, j);
            else
                r = hr[s];
            put_ring(ring[slot(m + 1)][s], hb, hx, r);
        }
        if constexpr (ES == 4) {
            if (m + 2 <= mend) pull1(0, hp0, hp1, wrapm(m + 2), hn);
        }
        // Workgroup barrier for the density ring only: the ring writes are
        // complete once lgkmcnt drains (no row loads are in flight here).
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);

        auto nb = [&](int i, int s) -> Real {
            const int sl = slot(m + A::cm(i));
            return ring[sl][s][box_own + A::c1(i) * H0 + A::c0(i)];
        };
        Real acc[2][3];
        lattice_acceleration<L, Real>(nb, a.ph.negG, acc);
        // The second species' halo of plane m+2 (FP32), the first part of
        // the halo rows (16-bit).
        const bool more = m + 2 <= mend;
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (ES == 4) {
            if (more) pull1(1, hp0, hp1, wrapm(m + 2), hn);
        } else {
            if (more) halo_issue(wrapm(m + 2), J0{}, JH{});
        }
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t site = (uint32_t)p0 + s1 * (uint32_t)(D3 ? p1 : 0) + sm * (uint32_t)m;
        const uint32_t voff = site * ES;
        collide_site<L, Real>(cur, rc, jc, acc, a.ph, ref, Counter{site, a.step_lo, a.step_hi}, [&](int s, auto &fs) {
            if (s == 0) {
                __builtin_amdgcn_sched_barrier(0);
                if (more) wide_issue(wrapm(m + 2), JE{}, JN{});
                if constexpr (ES == 2) {
                    if (more) halo_issue(wrapm(m + 2), JH{}, JN{});
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if (inside) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    Real v = fs[i];
                    store_stepped<S>(v, rdst[s], voff, (uint32_t)i * pop_bytes, site, (uint32_t)(s * Q + i),
                                     a.step_lo, a.ph.key0, a.ph.key1);
                }
            }
        });
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            rc[s] = rn[s];
#pragma unroll
            for (int al = 0; al < 3; ++al) jc[s][al] = jn[s][al];
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
        }
    }
}

template <class L, class S, int T0, int T1>
__device__ __forceinline__ void fused_tile_rows(const StepArgs<L, S> &a, int t0, int t1, int mbeg, int mend)
{
    constexpr int PLANE = (T0 + 2) * (T1 + 2);
    __shared__ typename Storage<S>::Real ring[4][2][PLANE];
    constexpr int NW = T0 * T1 / 64, NI = WideRows<L, sizeof(S)>().NI;
    __shared__ __attribute__((aligned(16))) uint32_t own[NW * NI * 256];  // 16-byte buffer-to-LDS targets
    __shared__ uint32_t tab[NW * NI * 64];
    if constexpr (sizeof(S) == 2) {
        __shared__ __attribute__((aligned(16))) uint32_t hown[NW * NI * 256];  // halo rows, same layout
        fused_tile_rows_body<L, S, T0, T1>(a, t0, t1, mbeg, mend, &ring[0][0][0], &own[0], &hown[0], &tab[0]);
    } else {
        fused_tile_rows_body<L, S, T0, T1>(a, t0, t1, mbeg, mend, &ring[0][0][0], &own[0], nullptr, &tab[0]);
    }
}

template <class L, class S, int T0, int T1, bool ASYNC, int CPOL = kStoreNonTemporal>
__global__ __launch_bounds__(T0 *T1) void fused_step_kernel(StepArgs<L, S> a, int chunk)
{
    constexpr bool D3 = L::D == 3;
    const int n0 = a.g.nx, n1 = D3 ? a.g.ny : 1, nm = D3 ? a.g.nz : a.g.ny;
    const int tiles0 = (n0 + T0 - 1) / T0, tiles1 = (n1 + T1 - 1) / T1;
    const int chunks = (nm + chunk - 1) / chunk;
    const unsigned logical = xcd_contiguous(blockIdx.x, (unsigned)tiles0 * tiles1 * chunks);
    const int t0 = (int)(logical % tiles0);
    const int t1 = (int)((logical / tiles0) % tiles1);
    const int ck = (int)(logical / ((unsigned)tiles0 * tiles1));
    const int mbeg = ck * chunk, mend = min(ck * chunk + chunk, nm);
    if constexpr (L::D == 3 && T0 == 256)
        fused_tile_rows<L, S, T0, T1>(a, t0, t1, mbeg, mend);
    else if constexpr (ASYNC)
        fused_tile_async<L, S, T0, T1, CPOL>(a, t0, t1, mbeg, mend);
    else
        fused_tile<L, S, T0, T1>(a, t0, t1, mbeg, mend);
}

// Supported tile shapes (T0 x T1 threads, chunk = planes per workgroup).
// The fused form is built for the FP32-arithmetic storages only; FP64 storage
// (the parity configuration) runs the two-pass form, where the FP64 collision
// fits the register file without spilling.
template <class L, class S>
bool fused_shape_valid(int tile_x, int tile_y, int march)
{
    if (std::is_same<S, double>::value) return false;
    if (march < 0 || march > 4096) return false;
    if (L::D == 3)
        return (tile_x == 256 && tile_y == 2) || (tile_x == 128 && tile_y == 4) || (tile_x == 64 && (tile_y == 4 || tile_y == 8)) ||
               (tile_x == 32 && (tile_y == 8 || tile_y == 16));
    return tile_y == 1 && (tile_x == 64 || tile_x == 128 || tile_x == 256);
}

template <class L, class S>
void default_fused_shape(const Geom &g, int &tx, int &ty, int &chunk)
{
    if (L::D == 3) {
        // Tiles measured on 256^3 (full-width 256x2 rows for every storage:
        // FP32 1.02 ms against 1.17 for 128x4, BF16 0.89 against 0.95 for
        // 64x4; other widths: FP32 128x4, 16-bit 64x4) and from 16^3 to 128^3
        // (narrower tiles for narrower lattices).  The march is then the
        // longest that still gives one workgroup per CU (256): fewer
        // workgroups leave CUs idle, while more, shorter marches re-read more
        // halo planes (128^3 FP32: 149 us at 256 workgroups, 160 us at 512,
        // 252 us at 128; 256^3 BF16 full-width rows: 0.886 ms at 128 planes,
        // 0.900 at 64, 0.915 at 32).
        if (g.nx == 256) {
            tx = 256;
            ty = 2;
        } else if (sizeof(S) == 4 && g.nx >= 128) {
            tx = 128;
            ty = 4;
        } else if (g.nx >= 64) {
            tx = 64;
            ty = 4;
        } else {
            tx = 32;
            ty = 8;
        }
        const long cols = (long)((g.nx + tx - 1) / tx) * (long)((g.ny + ty - 1) / ty);
        chunk = 2;
        while (chunk < 128 && cols * ((g.nz + 2L * chunk - 1) / (2L * chunk)) >= 256) chunk *= 2;
    } else {
        // Measured from 64x2 to 1024^2 (FP32): a small lattice is bound by
        // the latency of one row, so it wants as many workgroups as it has
        // tile rows; from about 2000 tile rows on, marching several rows per
        // workgroup (re-using the force ring) wins, up to 8 rows at 1024^2.
        tx = g.nx >= 256 ? 256 : (g.nx >= 128 ? 128 : 64);
        ty = 1;
        const long rows = (long)((g.nx + tx - 1) / tx) * (long)g.ny;
        chunk = 1;
        while (chunk < 16 && rows / (2L * chunk) >= 512) chunk *= 2;
        if (chunk < 4) chunk = 1;
    }
}

template <class L, class S>
bool fused_supported(const Geom &g, int tile_x, int tile_y, int march)
{
    if (std::is_same<S, double>::value) return false;
    // one species' array must be addressable by a 32-bit buffer offset
    if ((double)L::Q * (double)g.pitch * (double)sizeof(S) >= 4294967295.0) return false;
    // Any lattice size otherwise: ragged tiles are masked and every plane
    // index wraps periodically (with fewer than 3 planes the ring simply holds
    // copies).
    if (L::D == 3 && tile_x == 256 && g.nx != 256) return false;  // full-width tiles only
    // full-width tiles pull both species through one buffer resource
    if (L::D == 3 && (tile_x == 256 || (tile_x == 0 && g.nx == 256)) &&
        2.0 * (double)L::Q * (double)g.pitch * (double)sizeof(S) >= 4294967295.0)
        return false;
    return tile_x == 0 || fused_shape_valid<L, S>(tile_x, tile_y, march);
}

#ifndef FMLB_FUSED_ASYNC
#define FMLB_FUSED_ASYNC 1
#endif

// Both state buffers (read and written each step) up to this size stay in
// MI355X's 256 MB last-level cache from one step to the next if the stores
// keep it: the tiled kernel then stores without the non-temporal hint (D2Q9
// 1024^2, 151 MB: 0.0364 -> 0.0317 ms per step; D3Q19 64^3, 80 MB: 0.0265 ->
// 0.0258; D3Q19 128^3, 637 MB, would lose 2 % without the hint).
constexpr double kCacheResidentBytes = 192.0 * 1024 * 1024;

template <class L, class S, int T0, int T1, bool ASYNC = FMLB_FUSED_ASYNC>
hipError_t launch_fused_shape(const StepArgs<L, S> &a, int chunk, hipStream_t stream)
{
    const int n0 = a.g.nx, n1 = L::D == 3 ? a.g.ny : 1, nm = L::D == 3 ? a.g.nz : a.g.ny;
    const unsigned nblk = (unsigned)((n0 + T0 - 1) / T0) * (unsigned)((n1 + T1 - 1) / T1) *
                          (unsigned)((nm + chunk - 1) / chunk);
    if constexpr (ASYNC && !(L::D == 3 && T0 == 256)) {
        const double state = 2.0 * 2 * L::Q * (double)a.g.pitch * sizeof(S);
        if (state <= kCacheResidentBytes) {
            hipLaunchKernelGGL((fused_step_kernel<L, S, T0, T1, ASYNC, 0>), dim3(nblk), dim3(T0 * T1), 0, stream, a,
                               chunk);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((fused_step_kernel<L, S, T0, T1, ASYNC>), dim3(nblk), dim3(T0 * T1), 0, stream, a, chunk);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_fused(const StepArgs<L, S> &a, int tile_x, int tile_y, int march, hipStream_t stream)
{
    if constexpr (std::is_same<S, double>::value) {
        return hipErrorNotSupported;
    } else {
        int tx = tile_x, ty = tile_y, chunk = march;
        int dtx, dty, dch;
        default_fused_shape<L, S>(a.g, dtx, dty, dch);
        if (tx == 0) {
            tx = dtx;
            ty = dty;
        }
        if (chunk == 0) chunk = dch;
        if constexpr (L::D == 3) {
            if (tx == 256 && ty == 2) return launch_fused_shape<L, S, 256, 2>(a, chunk, stream);
            if (tx == 128 && ty == 4) return launch_fused_shape<L, S, 128, 4>(a, chunk, stream);
            if (tx == 64 && ty == 4) return launch_fused_shape<L, S, 64, 4>(a, chunk, stream);
            if (tx == 64 && ty == 8) return launch_fused_shape<L, S, 64, 8>(a, chunk, stream);
            if (tx == 32 && ty == 8) return launch_fused_shape<L, S, 32, 8>(a, chunk, stream);
            if (tx == 32 && ty == 16) return launch_fused_shape<L, S, 32, 16>(a, chunk, stream);
        } else {
            if (tx == 64) return launch_fused_shape<L, S, 64, 1>(a, chunk, stream);
            if (tx == 128) return launch_fused_shape<L, S, 128, 1>(a, chunk, stream);
            if (tx == 256) return launch_fused_shape<L, S, 256, 1>(a, chunk, stream);
        }
        return hipErrorInvalidValue;
    }
}

}  // namespace fmlb
