// Step kernels of the FLBE hot path and the state-transfer kernels.
//
// Two step forms share the per-site collision of collide.h and give the same
// bits:
//  - density_kernel + step_kernel: the density pass writes rho_sigma(r) of the
//    pre-collision state (Eq. (86)); the step kernel pulls the populations,
//    reads the neighbours' densities for the force of Eq. (87), collides and
//    stores.  Simple, any lattice size.
//  - fused_step_kernel (fused.h): one pass; each workgroup recomputes the
//    densities of its tile plus a one-site halo into LDS while marching
//    through planes.
#pragma once

#include <type_traits>
#include <utility>

#include "collide.h"
#include "storage.h"

namespace fmlb {

// f(std::integral_constant<int, k>) for k = 0 .. N-1, so that table lookups
// with k inside f are constant expressions.
template <int N, class F, int... K>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, K...>)
{
    (f(std::integral_constant<int, K>{}), ...);
}

template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

template <class L, class S>
struct StepArgs {
    using Real = typename Storage<S>::Real;
    const S *src;
    S *dst;
    Real *rho;  // [2][sites] densities of the pre-collision state (two-pass form)
    Geom g;
    Phys<Real> ph;
    Real ref[2];  // rho_ref per species (deviation storage)
    uint32_t step_lo, step_hi;
};

template <class L, class S>
__device__ __forceinline__ typename Storage<S>::Real load_pop(const S *buf, size_t pitch, int s, int i,
                                                              size_t site, typename Storage<S>::Real ref)
{
    using Real = typename Storage<S>::Real;
    Real v = Storage<S>::load(buf, ((size_t)(s * L::Q + i)) * pitch + site);
    if (Storage<S>::deviation) v += Real(L::w36[i]) / Real(36) * ref;
    return v;
}

// FP64 value v written to population (s, i) of a site: the deviation from
// w_i ref is formed in FP64, then rounded once to the storage format (host
// I/O and initial states).
template <class L, class S>
__device__ __forceinline__ void store_pop_f64(S *buf, size_t pitch, int s, int i, size_t site, double v, double ref)
{
    using Real = typename Storage<S>::Real;
    if (Storage<S>::deviation) v -= (double)L::w36[i] / 36.0 * ref;
    Storage<S>::store(buf, ((size_t)(s * L::Q + i)) * pitch + site, (Real)v);
}

// Absolute FP64 value of a stored population.
template <class L, class S>
__device__ __forceinline__ double load_pop_f64(const S *buf, size_t pitch, int s, int i, size_t site, double ref)
{
    double v = (double)Storage<S>::load(buf, ((size_t)(s * L::Q + i)) * pitch + site);
    if (Storage<S>::deviation) v += (double)L::w36[i] / 36.0 * ref;
    return v;
}

// Pull the 2Q pre-collision populations of site (x, y, z).
template <class L, class S>
__device__ __forceinline__ void pull_site(const S *src, const Geom &g, int x, int y, int z,
                                          const typename Storage<S>::Real (&ref)[2],
                                          typename Storage<S>::Real (&f)[2][L::Q])
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap(x, -L::cx[i], g.nx);
        const int ys = wrap(y, -L::cy[i], g.ny);
        const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
        const size_t site = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
#pragma unroll
        for (int s = 0; s < 2; ++s) f[s][i] = load_pop<L, S>(src, g.pitch, s, i, site, ref[s]);
    }
}

// Pull the 2Q stored values of site (x, y, z) as they are (deviations from
// w_i rho_ref for deviation storage), for the step kernels.
template <class L, class S>
__device__ __forceinline__ void pull_site_stored(const S *src, const Geom &g, int x, int y, int z,
                                                 typename Storage<S>::Real (&f)[2][L::Q])
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap(x, -L::cx[i], g.nx);
        const int ys = wrap(y, -L::cy[i], g.ny);
        const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
        const size_t site = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
#pragma unroll
        for (int s = 0; s < 2; ++s) f[s][i] = Storage<S>::load(src, ((size_t)(s * L::Q + i)) * g.pitch + site);
    }
}

template <class L, class S>
__global__ __launch_bounds__(256) void density_kernel(StepArgs<L, S> a)
{
    using Real = typename Storage<S>::Real;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= a.g.nx) return;
    Real f[2][L::Q];
    pull_site_stored<L, S>(a.src, a.g, x, y, z, f);
    const size_t site = (size_t)x + (size_t)a.g.nx * ((size_t)y + (size_t)a.g.ny * (size_t)z);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        Real r, j[3];
        moments<L, Real>(f[s], r, j);
        a.rho[(size_t)s * a.g.nsites + site] = r;  // rho - rho_ref for deviation storage
    }
}

// site_off is added (mod 2^32) to the site word of the noise counter (a
// lattice that is one slab of a larger one draws the larger one's noise).
template <class L, class S>
__global__ __launch_bounds__(256) void step_kernel(StepArgs<L, S> a, uint32_t site_off)
{
    using Real = typename Storage<S>::Real;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= a.g.nx) return;
    const Geom g = a.g;
    Real f[2][L::Q];
    pull_site_stored<L, S>(a.src, g, x, y, z, f);
    const Real *rho = a.rho;
    auto nb = [&](int i, int s) -> Real {
        const int xn = wrap(x, L::cx[i], g.nx);
        const int yn = wrap(y, L::cy[i], g.ny);
        const int zn = L::D == 3 ? wrap(z, L::cz[i], g.nz) : 0;
        return rho[(size_t)s * g.nsites + (size_t)xn + (size_t)g.nx * ((size_t)yn + (size_t)g.ny * (size_t)zn)];
    };
    Real acc[2][3];
    lattice_acceleration<L, Real>(nb, a.ph.negG, acc);
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    Real rho_s[2], j_s[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) moments<L, Real>(f[s], rho_s[s], j_s[s]);
    // reference density of the stored deviations (0 for absolute storage)
    const Real ref[2] = {Storage<S>::deviation ? a.ref[0] : Real(0), Storage<S>::deviation ? a.ref[1] : Real(0)};
    collide_site<L, Real>(f, rho_s, j_s, acc, a.ph, ref, Counter{(uint32_t)site + site_off, a.step_lo, a.step_hi},
                          [&](int s, auto &fs) {
#pragma unroll
                              for (int i = 0; i < L::Q; ++i)
                              {
                                  const size_t k = ((size_t)(s * L::Q + i)) * g.pitch + site;
                                  if constexpr (Storage<S>::stochastic)
                                      Storage<S>::store_sr(a.dst, k, fs[i],
                                                           sr_bits((uint32_t)site + site_off, (uint32_t)(s * L::Q + i), a.step_lo,
                                                                   a.ph.key0, a.ph.key1));
                                  else
                                      Storage<S>::store(a.dst, k, fs[i]);
                              }
                          });
}

// Rest state from FP64 densities rho[2][sites]: buf_i(r) = w_i rho(r + c_i),
// i.e. f_bar_i(r, 0) = w_i rho(r) in the pull layout.
template <class L, class S>
__global__ __launch_bounds__(256) void init_kernel(S *dst, const double *rho, Geom g,
                                                   typename Storage<S>::Real ref0,
                                                   typename Storage<S>::Real ref1)
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
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double w = (double)L::w36[i] / 36.0;
            store_pop_f64<L, S>(dst, g.pitch, s, i, site, w * rho[(size_t)s * g.nsites + nsite],
                                (double)(s == 0 ? ref0 : ref1));
        }
    }
}

// Pre-collision population (s, i) of every site to FP64: out[r] = buf_i(r - c_i).
template <class L, class S>
__global__ __launch_bounds__(256) void gather_pop_kernel(const S *src, double *out, Geom g, int s, int i,
                                                         typename Storage<S>::Real ref)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
    const int xs = wrap(x, -cx, g.nx), ys = wrap(y, -cy, g.ny), zs = L::D == 3 ? wrap(z, -cz, g.nz) : 0;
    const size_t src_site = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    out[site] = load_pop_f64<L, S>(src, g.pitch, s, i, src_site, (double)ref);
}

// Inverse of gather_pop_kernel: buf_i(r) = in[r + c_i].
template <class L, class S>
__global__ __launch_bounds__(256) void scatter_pop_kernel(S *dst, const double *in, Geom g, int s, int i,
                                                          typename Storage<S>::Real ref)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
    const int xn = wrap(x, cx, g.nx), yn = wrap(y, cy, g.ny), zn = L::D == 3 ? wrap(z, cz, g.nz) : 0;
    const size_t nsite = (size_t)xn + (size_t)g.nx * ((size_t)yn + (size_t)g.ny * (size_t)zn);
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    store_pop_f64<L, S>(dst, g.pitch, s, i, site, in[nsite], (double)ref);
}

// Roofline reference: the pulls and stores of one step with no arithmetic
// (buf_i(r) of the destination = pre-collision f_bar_i(r)).
template <class L, class S>
__global__ __launch_bounds__(256) void pull_copy_kernel(const S *src, S *dst, Geom g)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const size_t site = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    S v[2][L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap(x, -L::cx[i], g.nx), ys = wrap(y, -L::cy[i], g.ny);
        const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
        const size_t s2 = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
#pragma unroll
        for (int s = 0; s < 2; ++s) v[s][i] = src[((size_t)(s * L::Q + i)) * g.pitch + s2];
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
#pragma unroll
        for (int s = 0; s < 2; ++s) dst[((size_t)(s * L::Q + i)) * g.pitch + site] = v[s][i];
}

// Bandwidth references for the roofline (not part of the method): streaming
// kernels over a whole population buffer viewed as 16-byte words, with the
// launch shapes that measured fastest on MI355X for each access kind.
typedef float float4_v __attribute__((ext_vector_type(4)));

// Read-only: every word of `src` once (grid-stride); a sum is written only
// when it equals an impossible value, so the loads cannot be dropped.
static __global__ __launch_bounds__(256) void stream_read_kernel(const float4_v *__restrict__ src, size_t n,
                                                                  float *__restrict__ sink)
{
    float acc = 0.f;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const float4_v v = __builtin_nontemporal_load(&src[t]);
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == -1.2345e-30f) sink[0] = acc;
}

// Write-only: every word of `dst` once (grid-stride, non-temporal).
static __global__ __launch_bounds__(256) void stream_write_kernel(float4_v *__restrict__ dst, size_t n)
{
    const float4_v z = {0.f, 0.f, 0.f, 0.f};
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(z, &dst[t]);
}

// Copy without the pull shifts: 16-byte words, U in flight per thread.
template <int U>
__global__ __launch_bounds__(256) void stream_copy_kernel(const float4_v *__restrict__ src, float4_v *__restrict__ dst,
                                                          size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; t + (U - 1) * stride < n; t += U * stride) {
        float4_v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[t + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], &dst[t + u * stride]);
    }
    for (; t < n; t += stride) __builtin_nontemporal_store(src[t], &dst[t]);
}

}  // namespace fmlb
