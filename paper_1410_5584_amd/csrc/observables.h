// Observables of the stored pre-collision state: moment fields, FP64 global
// sums, mode statistics and structure factors (Sec. VI A).  Every kernel pulls
// the populations (pull layout, see storage.h) so the results refer to
// f_bar(r, n).
#pragma once

#include "kernels.h"

namespace fmlb {

constexpr int kRedBlock = 256;

template <class L, class S>
__device__ __forceinline__ void pull_site_f64(const S *src, const Geom &g, int x, int y, int z,
                                              const typename Storage<S>::Real (&ref)[2], double (&f)[2][L::Q])
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap(x, -L::cx[i], g.nx);
        const int ys = wrap(y, -L::cy[i], g.ny);
        const int zs = L::D == 3 ? wrap(z, -L::cz[i], g.nz) : 0;
        const size_t site = (size_t)xs + (size_t)g.nx * ((size_t)ys + (size_t)g.ny * (size_t)zs);
#pragma unroll
        for (int s = 0; s < 2; ++s) f[s][i] = load_pop_f64<L, S>(src, g.pitch, s, i, site, (double)ref[s]);
    }
}

// Site coordinates of linear index t (grid-stride helpers).
__device__ __forceinline__ void site_xyz(size_t t, const Geom &g, int &x, int &y, int &z)
{
    x = (int)(t % (size_t)g.nx);
    const size_t r = t / (size_t)g.nx;
    y = (int)(r % (size_t)g.ny);
    z = (int)(r / (size_t)g.ny);
}

// which = 0, 1: rho_sigma; 2 + s * D + alpha: j_bar_sigma,alpha.  FP64.
template <class L, class S>
__global__ __launch_bounds__(256) void moment_field_kernel(const S *src, double *out, Geom g, int which,
                                                           typename Storage<S>::Real ref0,
                                                           typename Storage<S>::Real ref1)
{
    using Real = typename Storage<S>::Real;
    const Real ref[2] = {ref0, ref1};
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < g.nsites; t += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        site_xyz(t, g, x, y, z);
        double f[2][L::Q];
        pull_site_f64<L, S>(src, g, x, y, z, ref, f);
        double v = 0;
        if (which < 2) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i) v += f[which][i];
        } else {
            const int s = (which - 2) / L::D, al = (which - 2) % L::D;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const int c = al == 0 ? L::cx[i] : al == 1 ? L::cy[i] : L::cz[i];
                if (c) v += c > 0 ? f[s][i] : -f[s][i];
            }
        }
        out[t] = v;
    }
}

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double *partial)
{
    __shared__ double sh[kRedBlock];
#pragma unroll 1
    for (int k = 0; k < NV; ++k) {
        sh[threadIdx.x] = v[k];
        __syncthreads();
        for (int w = kRedBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * NV + k] = sh[0];
        __syncthreads();
    }
}

// Per-block partial sums of rho_1, rho_2, (j_bar_1 + j_bar_2)_alpha.
template <class L, class S>
__global__ __launch_bounds__(kRedBlock) void sums_kernel(const S *src, double *partial, Geom g,
                                                         typename Storage<S>::Real ref0,
                                                         typename Storage<S>::Real ref1)
{
    using Real = typename Storage<S>::Real;
    const Real ref[2] = {ref0, ref1};
    constexpr int NV = 2 + L::D;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < g.nsites; t += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        site_xyz(t, g, x, y, z);
        double f[2][L::Q];
        pull_site_f64<L, S>(src, g, x, y, z, ref, f);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                v[s] += f[s][i];
                if (L::cx[i]) v[2] += L::cx[i] * f[s][i];
                if (L::cy[i]) v[3] += L::cy[i] * f[s][i];
                if (L::D == 3 && L::cz[i]) v[NV - 1] += L::cz[i] * f[s][i];
            }
    }
    block_reduce_store<NV>(v, partial);
}

// Fixed-order final reduction: out[k] = sum over blocks of partial[b][k];
// if accum != nullptr, accum[k] += that sum instead.
static __global__ __launch_bounds__(kRedBlock) void finalize_kernel(const double *partial, int nblocks, int nv,
                                                             double *out, double *accum)
{
    __shared__ double sh[kRedBlock];
    for (int k = 0; k < nv; ++k) {
        double v = 0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[(size_t)b * nv + k];
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int w = kRedBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (accum)
                accum[k] += sh[0];
            else
                out[k] = sh[0];
        }
        __syncthreads();
    }
}

// Per-block partial sums of m_a and m_a^2 (m_a = sum_i T_ai f_bar_i, Eq. (80))
// for both species: 4Q values laid out [s][a][moment].
template <class L, class S>
__global__ __launch_bounds__(kRedBlock) void mode_stats_kernel(const S *src, double *partial, Geom g,
                                                               typename Storage<S>::Real ref0,
                                                               typename Storage<S>::Real ref1)
{
    using Real = typename Storage<S>::Real;
    const Real ref[2] = {ref0, ref1};
    constexpr int NV = 4 * L::Q;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < g.nsites; t += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        site_xyz(t, g, x, y, z);
        double f[2][L::Q];
        pull_site_f64<L, S>(src, g, x, y, z, ref, f);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                double m = 0;
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    if (L::T[a][i]) m += (double)L::T[a][i] * f[s][i];
                v[(s * L::Q + a) * 2] += m;
                v[(s * L::Q + a) * 2 + 1] += m * m;
            }
    }
    block_reduce_store<NV>(v, partial);
}

// counts[0]: sites where not (rho_1 > 0 and rho_2 > 0); counts[1]: sites with a
// non-finite population.  Block partials as doubles (exact for counts < 2^53).
template <class L, class S>
__global__ __launch_bounds__(kRedBlock) void health_kernel(const S *src, double *partial, Geom g,
                                                           typename Storage<S>::Real ref0,
                                                           typename Storage<S>::Real ref1)
{
    using Real = typename Storage<S>::Real;
    const Real ref[2] = {ref0, ref1};
    double v[2] = {0, 0};
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < g.nsites; t += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        site_xyz(t, g, x, y, z);
        Real f[2][L::Q];
        pull_site<L, S>(src, g, x, y, z, ref, f);
        bool bad = false;
        Real r[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Real acc = 0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                acc += f[s][i];
                bad |= !isfinite(f[s][i]);
            }
            r[s] = acc;
        }
        if (!(r[0] > Real(0) && r[1] > Real(0))) v[0] += 1;
        if (bad) v[1] += 1;
    }
    block_reduce_store<2>(v, partial);
}

// ---------------------------------------------------------------------------
// Structure factors.  The real fields are transformed two at a time: the
// complex field Z = X + iY is built from the pre-collision state, transformed
// by separable line DFTs along x, y, z, and X_hat, Y_hat are recovered from
// Z_hat(k) and Z_hat(-k) (X real: X_hat(-k) = conj X_hat(k)), so
//   X_hat(k) = (Z_hat(k) + conj Z_hat(-k)) / 2,
//   Y_hat(k) = (Z_hat(k) - conj Z_hat(-k)) / (2i).
// Pairs: 0 (rho_1, rho_2); 1 + alpha (j_bar_1,alpha, j_bar_2,alpha);
// D + 1 the physical barycentric velocity (v_b,x, v_b,y) and, in 3D, D + 2
// (v_b,z, 0), with v_b = (j_bar_1 + j_bar_2 + (F_1 + F_2) / 2) / rho_t and
// the force of Eq. (87) at the same time level.  The populations are pulled
// once per snapshot (sk_moments_kernel); the first line transform reads the
// density and momentum pairs straight from those moments, and the velocity
// pairs' fields are built from them first (sk_field_kernel).
// ---------------------------------------------------------------------------
template <class L>
constexpr int sk_pairs()
{
    return L::D == 2 ? 4 : 6;
}

// Moments of both species, pulled once per snapshot, in FP64:
// mom[q][sites] = rho_q (q = 0, 1) and mom[2 + q D + alpha][sites] =
// j_bar_q,alpha, each summed in velocity order.
template <class L, class S>
__global__ __launch_bounds__(256) void sk_moments_kernel(const S *src, double *mom, Geom g,
                                                         typename Storage<S>::Real ref0,
                                                         typename Storage<S>::Real ref1)
{
    using Real = typename Storage<S>::Real;
    const Real ref[2] = {ref0, ref1};
    constexpr int D = L::D;
    const size_t n = g.nsites;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        site_xyz(t, g, x, y, z);
        double f[2][L::Q];
        pull_site_f64<L, S>(src, g, x, y, z, ref, f);
        double r[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                r[q] += f[q][i];
                if (L::cx[i]) j[q][0] += L::cx[i] > 0 ? f[q][i] : -f[q][i];
                if (L::cy[i]) j[q][1] += L::cy[i] > 0 ? f[q][i] : -f[q][i];
                if (D == 3 && L::cz[i]) j[q][2] += L::cz[i] > 0 ? f[q][i] : -f[q][i];
            }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            mom[(size_t)q * n + t] = r[q];
#pragma unroll
            for (int al = 0; al < D; ++al) mom[(size_t)(2 + q * D + al) * n + t] = j[q][al];
        }
    }
}

// Field of pair `pair` from the moments: Z[t] = X + iY.  In 3D the pass of
// pair D + 1 (v_b,x, v_b,y) also keeps v_b,z in the slot of j_bar_1,x, which
// no later pair reads, and pair D + 2 (v_b,z, 0) takes it from there instead
// of gathering the force's neighbour densities again.
template <class L>
__global__ __launch_bounds__(256) void sk_field_kernel(double *mom, double2 *Z, Geom g, int pair, double negG)
{
    constexpr int D = L::D;
    const size_t n = g.nsites;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double X, Y;
        if (pair == 0) {
            X = mom[t];
            Y = mom[n + t];
        } else if (pair <= D) {
            X = mom[(size_t)(2 + pair - 1) * n + t];
            Y = mom[(size_t)(2 + D + pair - 1) * n + t];
        } else if (pair == D + 2) {
            X = mom[2 * n + t];
            Y = 0.0;
        } else {
            // the barycentric velocity: components x (real part) and y (imaginary part)
            int x, y, z;
            site_xyz(t, g, x, y, z);
            double a[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const int xn = wrap(x, L::cx[i], g.nx), yn = wrap(y, L::cy[i], g.ny);
                const int zn = D == 3 ? wrap(z, L::cz[i], g.nz) : 0;
                const size_t nsite = (size_t)xn + (size_t)g.nx * ((size_t)yn + (size_t)g.ny * (size_t)zn);
                const double w = (double)L::w36[i] / 36.0;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const double ro = mom[(size_t)(1 - q) * n + nsite];
                    a[q][0] += L::cx[i] * w * ro;
                    a[q][1] += L::cy[i] * w * ro;
                    a[q][2] += L::cz[i] * w * ro;
                }
            }
            const double r0 = mom[t], r1 = mom[n + t];
            const double rt = r0 + r1;
            double vb[3] = {0, 0, 0};
#pragma unroll
            for (int al = 0; al < D; ++al) {
                const double Ft = negG * (r0 * a[0][al] + r1 * a[1][al]);
                const double jt = mom[(size_t)(2 + al) * n + t] + mom[(size_t)(2 + D + al) * n + t];
                vb[al] = rt > 0 ? (jt + 0.5 * Ft) / rt : 0.0;
            }
            X = vb[0];
            Y = vb[1];
            if (D == 3) mom[2 * n + t] = vb[2];
        }
        Z[t] = make_double2(X, Y);
    }
}

constexpr int kMaxLine = 2048;  // longest line the transforms accept

__device__ __forceinline__ double2 cadd(double2 a, double2 b)
{
    return make_double2(a.x + b.x, a.y + b.y);
}

__device__ __forceinline__ double2 csub(double2 a, double2 b)
{
    return make_double2(a.x - b.x, a.y - b.y);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Four-point DFT in place: v_r <- sum_s v_s (-i)^(r s).
__device__ __forceinline__ void dft4(double2 v[4])
{
    const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const double2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = make_double2(a1.x + b1.y, a1.y - b1.x);  // a1 - i b1
    v[3] = make_double2(a1.x - b1.y, a1.y + b1.x);  // a1 + i b1
}

// Lines of a power-of-two length L (2 <= L <= 2048): in-place FFT of every
// line along one axis, X[k] = sum_n x[n] e^{-2 pi i k n / L}, P lines per
// workgroup of max(64, P L / 4) threads (P L <= 4096).  Line l's elements
// are base(l) + m * stride as in dft_lines_kernel below, and P > 1 again
// needs inner_stride = 1 and inner a multiple of P.
// Mixed-radix Stockham form: a radix-2 pass first when log2 L is odd, then
// radix-4 passes.  The pass that joins transforms of length h into ones of
// length R h (h = 1, then times each radix) takes slot t = blk h + k (k < h)
// of a line, its inputs a[t + s L / R] (s < R), and writes
//   b[blk R h + k + r h] = sum_s a[t + s L / R] W_{R h}^{s k} W_R^{r s},
// W_n = e^{-2 pi i / n}; after the last pass the line holds X in natural
// order.  Each thread owns one radix-4 slot (two radix-2 slots) per pass;
// the first pass reads the lines from memory, the last writes them back, and
// the passes between exchange through one LDS copy of the lines.  The
// twiddles W_L^j, j < L / 2, are tabulated once per workgroup (a quarter from
// sincospi, the next quarter by the exact rotation W_L^{j + L/4} = -i W_L^j);
// W_L^{j + L/2} = -W_L^j covers the rest.
// With re non-null the input of the first pass is re + i im (two real fields
// of the same layout) instead of A; the result goes to A either way.
// Dynamic LDS: (P (L + 1) + L / 2) double2.
template <int P>
__global__ __launch_bounds__(1024) void fft_lines_kernel(double2 *A, int L, size_t stride, int inner,
                                                        size_t inner_stride, size_t outer_stride, const double *re,
                                                        const double *im)
{
    extern __shared__ double2 lds[];
    const int LP = L + 1;  // padded line pitch in LDS
    double2 *a = lds;
    double2 *tw = lds + P * LP;
    const size_t line0 = (size_t)blockIdx.x * P;
    const size_t base = (line0 % (size_t)inner) * inner_stride + (line0 / (size_t)inner) * outer_stride;
    const int tid = threadIdx.x, nthreads = blockDim.x;
    const int q = L / 4;  // radix-4 slots per line
    auto at = [&](int p, int m) -> double2 & { return A[base + (size_t)p + (size_t)m * stride]; };
    auto in = [&](int p, int m) -> double2 {
        const size_t k = base + (size_t)p + (size_t)m * stride;
        return re ? make_double2(re[k], im[k]) : A[k];
    };
    auto twiddle = [&](int j) -> double2 {
        const int half = L / 2;
        if (j < half) return tw[j];
        const double2 w = tw[j - half];
        return make_double2(-w.x, -w.y);
    };

    // First pass (h = 1, no twiddles), straight from memory.
    int h;
    if ((31 - __clz(L)) & 1) {
        for (int e = tid; e < P * (L / 2); e += nthreads) {
            const int p = e % P, t = e / P;
            const double2 u = in(p, t), v = in(p, t + L / 2);
            const double2 y0 = cadd(u, v), y1 = csub(u, v);
            if (L == 2) {
                at(p, 0) = y0;
                at(p, 1) = y1;
            } else {
                a[p * LP + 2 * t] = y0;
                a[p * LP + 2 * t + 1] = y1;
            }
        }
        if (L == 2) return;
        h = 2;
    } else {
        if (tid < P * q) {
            const int p = tid % P, t = tid / P;
            double2 v[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = in(p, t + s * q);
            dft4(v);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (L == 4)
                    at(p, r) = v[r];
                else
                    a[p * LP + 4 * t + r] = v[r];
            }
        }
        if (L == 4) return;
        h = 4;
    }
    for (int j = tid; j < L / 4; j += nthreads) {
        double sn, cs;
        sincospi(-2.0 * (double)j / (double)L, &sn, &cs);
        tw[j] = make_double2(cs, sn);
        tw[j + L / 4] = make_double2(sn, -cs);
    }
    __syncthreads();

    // Radix-4 passes through LDS; the last one writes to memory.
    const bool active = tid < P * q;
    const int p = active ? tid % P : 0, t = active ? tid / P : 0;
    for (; h < L; h *= 4) {
        const bool final_pass = 4 * h == L;
        double2 v[4];
        if (active) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = a[p * LP + t + s * q];
        }
        __syncthreads();
        if (active) {
            const int k = t & (h - 1), blk = t / h;
            const int j = k * (L / (4 * h));
            v[1] = cmul(v[1], twiddle(j));
            v[2] = cmul(v[2], twiddle(2 * j));
            v[3] = cmul(v[3], twiddle(3 * j));
            dft4(v);
            const int o = blk * 4 * h + k;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (final_pass)
                    at(p, o + r * h) = v[r];
                else
                    a[p * LP + o + r * h] = v[r];
            }
        }
        if (!final_pass) __syncthreads();
    }
}

// Lines of any other length: in-place DFT of every line along one axis,
// X[k] = sum_n x[n] e^{-2 pi i k n / L}, as a direct sum against an LDS
// twiddle table.  Line l's elements are base(l) + m * stride, m < L,
// base(l) = (l % inner) * inner_stride + (l / inner) * outer_stride.  A
// workgroup transforms P lines with consecutive bases (P > 1 needs
// inner_stride = 1 and inner a multiple of P): element m of its P lines is
// then P consecutive values, so the loads and stores of a strided axis are
// contiguous runs instead of scattered 16-byte accesses.  L <= 2048.  re,
// im as for fft_lines_kernel.
// Dynamic LDS: (P (L + 1) + L) double2.
template <int P>
__global__ __launch_bounds__(256) void dft_lines_kernel(double2 *A, int L, size_t stride, int inner,
                                                        size_t inner_stride, size_t outer_stride, const double *re,
                                                        const double *im)
{
    extern __shared__ double2 lds[];
    const int LP = L + 1;  // padded line pitch in LDS
    double2 *a = lds;
    double2 *tw = lds + P * LP;
    const size_t line0 = (size_t)blockIdx.x * P;
    const size_t base = (line0 % (size_t)inner) * inner_stride + (line0 / (size_t)inner) * outer_stride;
    for (int e = threadIdx.x; e < P * L; e += blockDim.x) {
        const int p = e % P, m = e / P;
        const size_t k = base + (size_t)p + (size_t)m * stride;
        a[p * LP + m] = re ? make_double2(re[k], im[k]) : A[k];
    }
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * (double)m / (double)L, &sn, &cs);
        tw[m] = make_double2(cs, sn);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P * L; e += blockDim.x) {
        const int p = e % P, k = e / P;
        double re = 0, im = 0;
        int idx = 0;
        for (int n = 0; n < L; ++n) {
            const double2 x = a[p * LP + n], t = tw[idx];
            re += x.x * t.x - x.y * t.y;
            im += x.x * t.y + x.y * t.x;
            idx += k;
            if (idx >= L) idx -= L;
        }
        A[base + (size_t)p + (size_t)k * stride] = make_double2(re, im);
    }
}

// The products of one transformed pair added to the accumulators acc[7][sites]:
// kind 0 (densities) adds |X_hat|^2, |Y_hat|^2, Re X_hat conj(Y_hat) to
// quantities 0, 1, 2; kind 1 (momenta) to 3, 4, 5; kind 2 (velocities)
// adds |X_hat|^2 + |Y_hat|^2 to 6.  Each product is scaled by `scale`; k = 0
// (the mean, removed by the definition dX = X - <X>) is skipped.
static __global__ __launch_bounds__(256) void sk_pair_accum_kernel(const double2 *Z, double *acc, Geom g, int kind,
                                                                   double scale)
{
    const size_t n = g.nsites;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        if (t == 0) continue;
        int x, y, z;
        site_xyz(t, g, x, y, z);
        const int xm = x == 0 ? 0 : g.nx - x, ym = y == 0 ? 0 : g.ny - y, zm = z == 0 ? 0 : g.nz - z;
        const size_t tm = (size_t)xm + (size_t)g.nx * ((size_t)ym + (size_t)g.ny * (size_t)zm);
        const double2 a = Z[t], c = Z[tm];
        // X_hat = (a + conj c) / 2,  Y_hat = (a - conj c) / (2i) = (Im(a) + Im(c), Re(c) - Re(a)) / 2
        const double xr = 0.5 * (a.x + c.x), xi = 0.5 * (a.y - c.y);
        const double yr = 0.5 * (a.y + c.y), yi = 0.5 * (c.x - a.x);
        const double xx = xr * xr + xi * xi, yy = yr * yr + yi * yi;
        if (kind == 2) {
            acc[6 * n + t] += scale * (xx + yy);
        } else {
            const int q = 3 * kind;
            acc[(size_t)q * n + t] += scale * xx;
            acc[(size_t)(q + 1) * n + t] += scale * yy;
            acc[(size_t)(q + 2) * n + t] += scale * (xr * yr + xi * yi);
        }
    }
}

static __global__ __launch_bounds__(256) void fill_kernel(double *p, size_t n, double v)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) p[t] = v;
}

}  // namespace fmlb
