// Population storage formats in device memory.
//
// The state is kept in the pull layout: buffer entry (sigma, i, r) holds the
// post-collision population of the previous step at r, so the pre-collision
// value of step n is f_bar_i(r, n) = buf_i(r - c_i) (streaming of Eq. (84)
// done by the reader).  Arrays are structure-of-arrays, [2][Q][sites], sites
// x-fastest, so every warp-wide access to one population is contiguous.
//
// FP32 and the 16-bit formats store the deviation d_i = f_i - w_i
// rho_ref_sigma (16-bit: rounded to nearest even, widened to FP32 on load);
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

template <>
struct Storage<double> {
    using Real = double;
    static constexpr bool deviation = false;
    __device__ static double load(const double *p, size_t k) { return p[k]; }
    __device__ static void store(double *p, size_t k, double v) { p[k] = v; }
};

template <>
struct Storage<float> {
    using Real = float;
    static constexpr bool deviation = true;
    __device__ static float load(const float *p, size_t k) { return p[k]; }
    __device__ static void store(float *p, size_t k, float v) { p[k] = v; }
};

template <>
struct Storage<__hip_bfloat16> {
    using Real = float;
    static constexpr bool deviation = true;
    __device__ static float load(const __hip_bfloat16 *p, size_t k) { return __bfloat162float(p[k]); }
    __device__ static void store(__hip_bfloat16 *p, size_t k, float v) { p[k] = __float2bfloat16(v); }
};

template <>
struct Storage<__half> {
    using Real = float;
    static constexpr bool deviation = true;
    __device__ static float load(const __half *p, size_t k) { return __half2float(p[k]); }
    __device__ static void store(__half *p, size_t k, float v) { p[k] = __float2half_rn(v); }
};

// Geometry of one periodic lattice.
struct Geom {
    int nx, ny, nz;
    size_t nsites;  // nx * ny * nz
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
