// Counter-based Gaussian noise for the FLBE collision.
//
// The paper draws an independent Gaussian number per mode and site with the
// Box-Muller method (Sec. VI A).  Here the uniforms come from the counter-based
// bijection Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11: two 32x32->64
// multiplications per round, Weyl key schedule, ten rounds), so a normal is a
// pure function of (seed, site, step, index) and any launch shape, tiling or
// replay order gives the same sample path.
//
// Stream layout (shared with every other implementation of the library's
// convention): block j of a site is Philox(counter = (site, step_lo, j,
// step_hi), key = (seed_lo, seed_hi)) and its four words are words 4j..4j+3
// of the site's stream.  Word w yields the Box-Muller pair of normals
// (z_2w, z_2w+1): U_a = w >> 16, U_b = w & 0xffff, u = (2U + 1) 2^-17 in
// (0, 1) (exact in FP32), z_2w = r cos(2 pi u_b), z_2w+1 = r sin(2 pi u_b),
// r = sqrt(-2 ln u_a).  16-bit uniforms bound |z| by sqrt(2 ln 2^17) = 4.85
// (a tail of probability 1.2e-6) and bias the variance by less than 1e-4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmlb {

struct Counter {
    uint32_t site, step_lo, step_hi;
};

// a ^ b ^ c in one instruction (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The four words of block j.
__device__ __forceinline__ void block_words(const Counter &c, uint32_t j, uint32_t k0, uint32_t k1,
                                            uint32_t (&w)[4])
{
    uint32_t x0 = c.site, x1 = c.step_lo, x2 = j, x3 = c.step_hi;
    philox10(x0, x1, x2, x3, k0, k1);
    w[0] = x0;
    w[1] = x1;
    w[2] = x2;
    w[3] = x3;
}

template <class Real>
__device__ __forceinline__ Real to_uniform16(uint32_t U);

template <>
__device__ __forceinline__ float to_uniform16<float>(uint32_t U)
{
    // U < 2^16, so (float)U, U * 2^-16 and the final sum are exact.
    return __builtin_fmaf((float)U, 0x1p-16f, 0x1p-17f);
}

template <>
__device__ __forceinline__ double to_uniform16<double>(uint32_t U)
{
    return __builtin_fma((double)U, 0x1p-16, 0x1p-17);
}

// Box-Muller pair.  FP32: the hardware log2 / sin / cos (v_log_f32 takes
// log base 2, v_sin_f32 / v_cos_f32 take the angle in revolutions, so
// 2 pi u needs no multiply and no range reduction).  FP64: libm-grade calls.
template <class Real>
__device__ __forceinline__ void box_muller(Real ua, Real ub, Real &z0, Real &z1);

template <>
__device__ __forceinline__ void box_muller<float>(float ua, float ub, float &z0, float &z1)
{
    // -2 ln u = -2 ln 2 log2 u >= 1.5e-5 for u <= 1 - 2^-17, never denormal.
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
    z0 = r * __builtin_amdgcn_cosf(ub);
    z1 = r * __builtin_amdgcn_sinf(ub);
}

template <>
__device__ __forceinline__ void box_muller<double>(double ua, double ub, double &z0, double &z1)
{
    const double r = sqrt(-2.0 * log(ua));
    double s, c;
    sincos(6.283185307179586476925286766559 * ub, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// The pair of normals carried by one stream word.
template <class Real>
__device__ __forceinline__ void word_normals(uint32_t w, Real &z0, Real &z1)
{
    box_muller<Real>(to_uniform16<Real>(w >> 16), to_uniform16<Real>(w & 0xffffu), z0, z1);
}

}  // namespace fmlb
