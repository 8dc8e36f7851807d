// Population storage formats in device memory.
//
// The state is kept in the pull layout: buffer entry (sigma, i, r) holds the
// post-collision population of the previous step at r, so the pre-collision
// value of step n is f_bar_i(r, n) = buf_i(r - c_i) (streaming of Eq. (84)
// done by the reader).  Arrays are structure-of-arrays, [2][Q][sites], sites
// x-fastest, so every warp-wide access to one population is contiguous.
//
// FP32 and the 16-bit formats store the deviation d_i = f_i - w_i
// rho_ref_sigma (16-bit: rounded to nearest even, or stochastically for the
// bf16_sr / f16_sr formats below; widened to FP32 on load);
// the step kernels update the deviations directly (collide.h), so FP32
// rounding acts at the scale of the fluctuations, not of w_i rho.  FP64
// stores absolute values.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace fmlb {

template <class S>
struct Storage;

// 16-bit formats whose time steps round the stored deviations
// stochastically: the bits below the kept ones get a uniform offset from an
// integer hash of (site, species * Q + population, step, seed), so every rounding
// is unbiased and the errors of neighbouring sites and of successive steps
// are independent.  Round-to-nearest errs alike at all sites of a domain of
// nearly equal deviations, which drifts the species masses of demixed
// lattices; stochastic rounding does not.  Same bits in memory as BF16 /
// FP16; initial states and host writes still round to nearest.
struct bf16_sr {
    unsigned short x;
};
struct f16_sr {
    unsigned short x;
};

// 32 hash bits for the stochastic rounding of value (site, sp_pop) at step
// of a run with Philox key (k0, k1).  The inputs are combined with the three
// 32-bit primes of xxHash32 (Y. Collet, xxHash specification: PRIME32_1 =
// 0x9E3779B1, PRIME32_2 = 0x85EBCA77, PRIME32_3 = 0xC2B2AE3D) and mixed by
// xxHash32's final avalanche (xor-shift 15, multiply PRIME32_2, xor-shift 13,
// multiply PRIME32_3, xor-shift 16), so runs that differ only in the seed
// round independently.
__host__ __device__ __forceinline__ uint32_t sr_hash(uint32_t site, uint32_t sp_pop, uint32_t step, uint32_t k0, uint32_t k1)
{
    uint32_t h = (site * 0x9E3779B1u) ^ (step * 0x85EBCA77u) ^ (sp_pop * 0xC2B2AE3Du) ^ k0 ^ ((k1 << 16) | (k1 >> 16));
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    h *= 0xC2B2AE3Du;
    h ^= h >> 16;
    return h;
}

// Rounding bits (the top 16 are used) of value (site, sp_pop) at step: one
// hash serves the two values sp_pop = 2m and 2m + 1, its high half for the
// first and its low half for the second.
__host__ __device__ __forceinline__ uint32_t sr_bits(uint32_t site, uint32_t sp_pop, uint32_t step, uint32_t k0, uint32_t k1)
{
    const uint32_t h = sr_hash(site, sp_pop >> 1, step, k0, k1);
    return (sp_pop & 1u) ? h << 16 : h;
}

// FP32 -> BF16 bits, stochastic: 16 random bits below the kept ones.
__host__ __device__ __forceinline__ unsigned short bf16_bits_sr(float v, uint32_t h)
{
    return (unsigned short)((__builtin_bit_cast(uint32_t, v) + (h >> 16)) >> 16);
}

// FP32 -> FP16 bits, stochastic.  Normal FP16 range: 13 random bits below the
// FP16 mantissa, then the (now exact) conversion.  Below 2^-14 the FP16
// values are the multiples of 2^-24 (subnormals), coarser than 13 bits below
// an FP32 mantissa there, so |v| 2^24 gets a uniform offset in [0, 1) and is
// rounded down to an integer k, stored as k 2^-24 with the sign of v.
__host__ __device__ __forceinline__ unsigned short f16_bits_sr(float v, uint32_t h)
{
    const float a = __builtin_fabsf(v);
    if (a < 0x1p-14f) {
        const float k = __builtin_floorf(__builtin_fmaf(a, 0x1p24f, (float)(h >> 16) * 0x1p-16f));
        return __half_as_ushort(__float2half_rn(__builtin_copysignf(k * 0x1p-24f, v)));
    }
    const uint32_t b = (__builtin_bit_cast(uint32_t, v) + (h >> 19)) & ~0x1FFFu;
    return __half_as_ushort(__float2half_rn(__builtin_bit_cast(float, b)));
}

template <>
struct Storage<double> {
    using Real = double;
    static constexpr bool deviation = false;
    static constexpr bool stochastic = false;
    __device__ static double load(const double *p, size_t k) { return p[k]; }
    __device__ static void store(double *p, size_t k, double v) { p[k] = v; }
};

template <>
struct Storage<float> {
    using Real = float;
    static constexpr bool deviation = true;
    static constexpr bool stochastic = false;
    __device__ static float load(const float *p, size_t k) { return p[k]; }
    __device__ static void store(float *p, size_t k, float v) { p[k] = v; }
};

template <>
struct Storage<__hip_bfloat16> {
    using Real = float;
    static constexpr bool deviation = true;
    static constexpr bool stochastic = false;
    __device__ static float load(const __hip_bfloat16 *p, size_t k) { return __bfloat162float(p[k]); }
    __device__ static void store(__hip_bfloat16 *p, size_t k, float v) { p[k] = __float2bfloat16(v); }
};

template <>
struct Storage<__half> {
    using Real = float;
    static constexpr bool deviation = true;
    static constexpr bool stochastic = false;
    __device__ static float load(const __half *p, size_t k) { return __half2float(p[k]); }
    __device__ static void store(__half *p, size_t k, float v) { p[k] = __float2half_rn(v); }
};

template <>
struct Storage<bf16_sr> {
    using Real = float;
    static constexpr bool deviation = true;
    static constexpr bool stochastic = true;
    __device__ static float load(const bf16_sr *p, size_t k) { return __builtin_bit_cast(float, (uint32_t)p[k].x << 16); }
    __device__ static void store(bf16_sr *p, size_t k, float v)
    {
        p[k].x = __builtin_bit_cast(unsigned short, __float2bfloat16(v));
    }
    __device__ static void store_sr(bf16_sr *p, size_t k, float v, uint32_t h) { p[k].x = bf16_bits_sr(v, h); }
};

template <>
struct Storage<f16_sr> {
    using Real = float;
    static constexpr bool deviation = true;
    static constexpr bool stochastic = true;
    __device__ static float load(const f16_sr *p, size_t k) { return __half2float(__ushort_as_half(p[k].x)); }
    __device__ static void store(f16_sr *p, size_t k, float v) { p[k].x = __half_as_ushort(__float2half_rn(v)); }
    __device__ static void store_sr(f16_sr *p, size_t k, float v, uint32_t h) { p[k].x = f16_bits_sr(v, h); }
};

// Geometry of one periodic lattice.
struct Geom {
    int nx, ny, nz;
    size_t nsites;  // nx * ny * nz
    size_t pitch;   // elements from one population array to the next (>= nsites)
    Geom() = default;
    __host__ __device__ constexpr Geom(int x, int y, int z, size_t n, size_t p)
        : nx(x), ny(y), nz(z), nsites(n), pitch(p)
    {
    }
};

// r + d with periodic wrap for |d| <= 1.
__device__ __forceinline__ int wrap(int x, int d, int n)
{
    int v = x + d;
    v = v < 0 ? v + n : v;
    v = v >= n ? v - n : v;
    return v;
}

}  // namespace fmlb
