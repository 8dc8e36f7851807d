// Host runtime of the C ABI declared in include/fmlb.h: parameter validation,
// buffer carving, kernel dispatch over (lattice, storage), host transfers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/fmlb.h"
#include "fused.h"
#include "observables.h"

using namespace fmlb;

// Fused steps instantiated in fused_ilp.hip, which is compiled with its own
// scheduling strategy (D3Q19 in every storage and rounding, D2Q9 in BF16).
namespace fmlb {
extern template hipError_t launch_fused<D3Q19, float>(const StepArgs<D3Q19, float> &, int, int, int, hipStream_t);
extern template hipError_t launch_fused<D3Q19, __half>(const StepArgs<D3Q19, __half> &, int, int, int, hipStream_t);
extern template hipError_t launch_fused<D3Q19, __hip_bfloat16>(const StepArgs<D3Q19, __hip_bfloat16> &, int, int,
                                                               int, hipStream_t);
extern template hipError_t launch_fused<D3Q19, f16_sr>(const StepArgs<D3Q19, f16_sr> &, int, int, int, hipStream_t);
extern template hipError_t launch_fused<D3Q19, bf16_sr>(const StepArgs<D3Q19, bf16_sr> &, int, int, int, hipStream_t);
extern template hipError_t launch_fused<D2Q9, __hip_bfloat16>(const StepArgs<D2Q9, __hip_bfloat16> &, int, int, int,
                                                              hipStream_t);
}  // namespace fmlb

namespace fmlb {
// Last HIP error of any entry point (shared with the batched entry points).
thread_local int32_t g_last_hip = 0;
}  // namespace fmlb

namespace {

#define HIP_TRY(...)                                   \
    do {                                               \
        hipError_t e_ = (__VA_ARGS__);                 \
        if (e_ != hipSuccess) {                        \
            g_last_hip = (int32_t)e_;                  \
            return FMLB_E_HIP;                         \
        }                                              \
    } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int lattice_q(int lattice) { return lattice == FMLB_D2Q9 ? 9 : 19; }
int lattice_d(int lattice) { return lattice == FMLB_D2Q9 ? 2 : 3; }

size_t elem_size(int storage)
{
    switch (storage) {
    case FMLB_F64: return 8;
    case FMLB_F32: return 4;
    default: return 2;
    }
}

size_t real_size(int storage) { return storage == FMLB_F64 ? 8 : 4; }

constexpr int kReduceBlocks = 1024;
constexpr int kSkQuantities = 7;
// FP64 moments per site of the structure-factor work arrays: rho_1, rho_2
// and the D components of j_bar_1 and j_bar_2 (kSkMoments for D = 3).
constexpr int kSkMoments = 2 + 2 * 3;
int sk_moments(int lattice) { return lattice == FMLB_D2Q9 ? 2 + 2 * 2 : kSkMoments; }

bool valid_params(const fmlb_params *p)
{
    if (!p) return false;
    if (p->lattice != FMLB_D2Q9 && p->lattice != FMLB_D3Q19) return false;
    if (p->storage < FMLB_F64 || p->storage > FMLB_F16_DEV) return false;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
    if (p->lattice == FMLB_D2Q9 && p->nz != 1) return false;
    const double n = (double)p->nx * (double)p->ny * (double)p->nz;
    if (n >= 2147483648.0) return false;
    if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5) || !(p->tau_d > 0.5)) return false;
    if (!std::isfinite(p->tau[0]) || !std::isfinite(p->tau[1]) || !std::isfinite(p->tau_d)) return false;
    if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return false;
    if (!std::isfinite(p->G)) return false;
    if (!std::isfinite(p->rho_ref[0]) || !std::isfinite(p->rho_ref[1])) return false;
    if (p->flags & ~(uint32_t)(FMLB_NOISE_OFF | FMLB_NOISE_NO_SDF | FMLB_ROUND_STOCHASTIC)) return false;
    if ((p->flags & FMLB_ROUND_STOCHASTIC) && p->storage != FMLB_BF16_DEV && p->storage != FMLB_F16_DEV) return false;
    return true;
}

struct Layout {
    size_t rho, stage, skA, skmom, skacc, partial, modeacc, misc, total;
};

Layout scratch_layout(const fmlb_params *p)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const int Q = lattice_q(p->lattice);
    Layout l{};
    size_t o = 0;
    l.rho = o;
    o += align256(2 * n * real_size(p->storage));
    l.stage = o;
    o += align256(2 * n * sizeof(double));
    l.skA = o;
    o += align256(n * 2 * sizeof(double));
    l.skmom = o;
    o += align256((size_t)sk_moments(p->lattice) * n * sizeof(double));
    l.skacc = o;
    o += align256((size_t)kSkQuantities * n * sizeof(double));
    l.partial = o;
    o += align256((size_t)kReduceBlocks * 4 * Q * sizeof(double));
    l.modeacc = o;
    o += align256(4 * Q * sizeof(double));
    l.misc = o;
    o += align256(64 * sizeof(double));
    l.total = o;
    return l;
}

}  // namespace

struct fmlb_ctx {
    fmlb_params p;
    hipStream_t stream;
    void *pops[2];
    unsigned char *scratch;
    Layout lay;
    Geom g;
    int Q, D;
    int cur;
    int64_t step;
    bool ready;
    int64_t sk_samples, mode_samples;
    int tile_x, tile_y, march;
    uint32_t site_off;  // noise-counter site offset (two-pass form only)
};

namespace {

template <class T>
T *scr(fmlb_ctx *c, size_t off)
{
    return reinterpret_cast<T *>(c->scratch + off);
}

template <class F>
fmlb_status dispatch(const fmlb_ctx *c, F &&f)
{
    if (c->p.flags & FMLB_ROUND_STOCHASTIC) {
        switch (c->p.lattice * 4 + c->p.storage) {
        case FMLB_D2Q9 * 4 + FMLB_BF16_DEV: return f(D2Q9{}, (bf16_sr *)nullptr);
        case FMLB_D2Q9 * 4 + FMLB_F16_DEV: return f(D2Q9{}, (f16_sr *)nullptr);
        case FMLB_D3Q19 * 4 + FMLB_BF16_DEV: return f(D3Q19{}, (bf16_sr *)nullptr);
        case FMLB_D3Q19 * 4 + FMLB_F16_DEV: return f(D3Q19{}, (f16_sr *)nullptr);
        }
        return FMLB_E_INVALID;
    }
    switch (c->p.lattice * 4 + c->p.storage) {
    case FMLB_D2Q9 * 4 + FMLB_F64: return f(D2Q9{}, (double *)nullptr);
    case FMLB_D2Q9 * 4 + FMLB_F32: return f(D2Q9{}, (float *)nullptr);
    case FMLB_D2Q9 * 4 + FMLB_BF16_DEV: return f(D2Q9{}, (__hip_bfloat16 *)nullptr);
    case FMLB_D2Q9 * 4 + FMLB_F16_DEV: return f(D2Q9{}, (__half *)nullptr);
    case FMLB_D3Q19 * 4 + FMLB_F64: return f(D3Q19{}, (double *)nullptr);
    case FMLB_D3Q19 * 4 + FMLB_F32: return f(D3Q19{}, (float *)nullptr);
    case FMLB_D3Q19 * 4 + FMLB_BF16_DEV: return f(D3Q19{}, (__hip_bfloat16 *)nullptr);
    case FMLB_D3Q19 * 4 + FMLB_F16_DEV: return f(D3Q19{}, (__half *)nullptr);
    }
    return FMLB_E_INVALID;
}

struct SiteGrid {
    dim3 grid, block;
};

SiteGrid site_grid(const Geom &g)
{
    int bx = g.nx >= 256 ? 256 : ((g.nx + 63) / 64) * 64;
    SiteGrid s;
    s.block = dim3(bx);
    s.grid = dim3((g.nx + bx - 1) / bx, g.ny, g.nz);
    return s;
}

int stride_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    return (int)(b < (size_t)kReduceBlocks ? (b ? b : 1) : (size_t)kReduceBlocks);
}

template <class Real>
Phys<Real> make_phys(const fmlb_params &p)
{
    Phys<Real> ph{};
    const double lam0 = 1.0 / p.tau[0], lam1 = 1.0 / p.tau[1], lam_d = 1.0 / p.tau_d;
    const double mu = 3.0 * p.kT;  // mu = k_B T / c_s^2
    ph.lam[0] = (Real)lam0;
    ph.lam[1] = (Real)lam1;
    ph.lam_d = (Real)lam_d;
    ph.negG = (Real)(-p.G);
    // Without noise every amplitude is zero: the normals are still drawn
    // (the kernels carry no noise-off branch) and contribute exact zeros.
    const bool noisy = (p.kT > 0.0) && !(p.flags & FMLB_NOISE_OFF);
    const bool sdf = noisy && !(p.flags & FMLB_NOISE_NO_SDF);
    ph.gain[0] = noisy ? (Real)std::sqrt((2.0 * lam0 - lam0 * lam0) * mu) : (Real)0;
    ph.gain[1] = noisy ? (Real)std::sqrt((2.0 * lam1 - lam1 * lam1) * mu) : (Real)0;
    ph.sd_gain = sdf ? (Real)std::sqrt((2.0 * lam_d - lam_d * lam_d) * p.kT) : (Real)0;
    ph.key0 = (uint32_t)p.seed;
    ph.key1 = (uint32_t)(p.seed >> 32);
    return ph;
}

template <class L, class S>
StepArgs<L, S> step_args(fmlb_ctx *c, int64_t step)
{
    using Real = typename Storage<S>::Real;
    StepArgs<L, S> a{};
    a.src = reinterpret_cast<const S *>(c->pops[c->cur]);
    a.dst = reinterpret_cast<S *>(c->pops[1 - c->cur]);
    a.rho = scr<Real>(c, c->lay.rho);
    a.g = c->g;
    a.ph = make_phys<Real>(c->p);
    a.ref[0] = (Real)c->p.rho_ref[0];
    a.ref[1] = (Real)c->p.rho_ref[1];
    a.step_lo = (uint32_t)(uint64_t)step;
    a.step_hi = (uint32_t)((uint64_t)step >> 32);
    return a;
}

template <class L, class S>
fmlb_status run_steps(fmlb_ctx *c, int64_t n)
{
    const SiteGrid sg = site_grid(c->g);
    for (int64_t t = 0; t < n; ++t) {
        StepArgs<L, S> a = step_args<L, S>(c, c->step);
        if (c->tile_x != 1 && c->site_off == 0 && fused_supported<L, S>(c->g, c->tile_x, c->tile_y, c->march)) {
            HIP_TRY(launch_fused<L, S>(a, c->tile_x, c->tile_y, c->march, c->stream));
        } else {
            hipLaunchKernelGGL((density_kernel<L, S>), sg.grid, sg.block, 0, c->stream, a);
            LAUNCH_CHECK();
            hipLaunchKernelGGL((step_kernel<L, S>), sg.grid, sg.block, 0, c->stream, a, c->site_off);
            LAUNCH_CHECK();
        }
        c->cur = 1 - c->cur;
        c->step += 1;
    }
    return FMLB_OK;
}

template <class S>
typename Storage<S>::Real ref_of(const fmlb_ctx *c, int s)
{
    return (typename Storage<S>::Real)c->p.rho_ref[s];
}

fmlb_status sync(fmlb_ctx *c)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FMLB_OK;
}

// Launch the line transforms of one axis, P lines per workgroup: the FFT for
// power-of-two lengths, the direct sum for the others.
template <int P>
fmlb_status dft_axis(hipStream_t stream, double2 *A, int L, size_t lines, size_t stride, int inner,
                     size_t inner_stride, size_t outer_stride, const double *re, const double *im)
{
    const bool pow2 = (L & (L - 1)) == 0;
    const void *fn = pow2 ? (const void *)fft_lines_kernel<P> : (const void *)dft_lines_kernel<P>;
    const size_t lds = ((size_t)P * (L + 1) + (pow2 ? (size_t)L / 2 : (size_t)L)) * sizeof(double2);
    const unsigned threads = pow2 ? (unsigned)std::max(64, P * L / 4) : 256u;
    if (lds > 65536)  // more than the default limit
        HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (pow2)
        hipLaunchKernelGGL(fft_lines_kernel<P>, dim3((unsigned)(lines / P)), dim3(threads), lds, stream, A, L, stride,
                           inner, inner_stride, outer_stride, re, im);
    else
        hipLaunchKernelGGL(dft_lines_kernel<P>, dim3((unsigned)(lines / P)), dim3(threads), lds, stream, A, L, stride,
                           inner, inner_stride, outer_stride, re, im);
    LAUNCH_CHECK();
    return FMLB_OK;
}

// Forward DFT of a complex lattice field along every axis of length > 1.
// The strided axes (y, z) take several adjacent lines per workgroup (as many
// as divide nx, up to 16, within 4096 elements for the FFT or 148 KB of LDS
// for the direct sum), so their accesses are contiguous runs.  With re
// non-null the field is re + i im and A receives the transform (the lattice
// must then have an axis of length > 1).
fmlb_status dft_field(const Geom &g, hipStream_t stream, double2 *A, const double *re = nullptr,
                      const double *im = nullptr)
{
    const int dims[3] = {g.nx, g.ny, g.nz};
    for (int ax = 0; ax < 3; ++ax) {
        const int L = dims[ax];
        if (L == 1) continue;
        size_t stride, inner, inner_stride, outer_stride, lines;
        if (ax == 0) {
            stride = 1;
            lines = (size_t)g.ny * g.nz;
            inner = lines;
            inner_stride = (size_t)g.nx;
            outer_stride = 0;
        } else if (ax == 1) {
            stride = (size_t)g.nx;
            lines = (size_t)g.nx * g.nz;
            inner = (size_t)g.nx;
            inner_stride = 1;
            outer_stride = (size_t)g.nx * g.ny;
        } else {
            stride = (size_t)g.nx * g.ny;
            lines = (size_t)g.nx * g.ny;
            inner = lines;
            inner_stride = 1;
            outer_stride = 0;
        }
        const bool pow2 = (L & (L - 1)) == 0;
        auto fits = [&](int P) {
            if (ax == 0 ? P != 1 : inner % (size_t)P != 0) return false;
            if (pow2) return (size_t)P * L <= 4096;
            return ((size_t)P * (L + 1) + (size_t)L) * sizeof(double2) <= 148 * 1024;
        };
        fmlb_status st;
        if (fits(16))
            st = dft_axis<16>(stream, A, L, lines, stride, (int)inner, inner_stride, outer_stride, re, im);
        else if (fits(8))
            st = dft_axis<8>(stream, A, L, lines, stride, (int)inner, inner_stride, outer_stride, re, im);
        else if (fits(4))
            st = dft_axis<4>(stream, A, L, lines, stride, (int)inner, inner_stride, outer_stride, re, im);
        else if (fits(2))
            st = dft_axis<2>(stream, A, L, lines, stride, (int)inner, inner_stride, outer_stride, re, im);
        else
            st = dft_axis<1>(stream, A, L, lines, stride, (int)inner, inner_stride, outer_stride, re, im);
        if (st) return st;
        re = im = nullptr;  // later axes transform A in place
    }
    return FMLB_OK;
}

// Bytes of work arrays the structure-factor accumulation needs per site:
// the densities of both species (FP64 at most, for the force in v_b) and one
// complex FP64 field.
// Bytes of work arrays the structure-factor accumulation needs per site: the
// FP64 moments of both species (2 + 2 D values; D = 3 at most) and one
// complex FP64 field.
constexpr size_t kSkWorkBytesPerSite = kSkMoments * sizeof(double) + sizeof(double2);

// The structure-factor accumulation of one snapshot (Sec. VI A): the seven
// quantities of fmlb_sk_accumulate are added to acc[7][sites], two real
// fields per complex transform.  mom and Z are work arrays of (2 + 2 D) *
// sites doubles and sites double2.
template <class L, class S>
fmlb_status sk_accumulate_impl(const fmlb_params &p, const Geom &g, hipStream_t stream, const S *src, double *mom,
                               double2 *Z, double *acc)
{
    using Real = typename Storage<S>::Real;
    const size_t n = g.nsites;
    constexpr int D = L::D;
    const dim3 gb(stride_blocks(n)), tb(256);
    hipLaunchKernelGGL((sk_moments_kernel<L, S>), gb, tb, 0, stream, src, mom, g, (Real)p.rho_ref[0],
                       (Real)p.rho_ref[1]);
    LAUNCH_CHECK();
    const double inv_n = 1.0 / (double)n;
    for (int pair = 0; pair < sk_pairs<L>(); ++pair) {
        // The density and momentum pairs are two moment fields each: the first
        // transform reads them directly.  The velocity pairs are built first.
        const double *re = nullptr, *im = nullptr;
        if (pair <= D && n > 1) {
            re = mom + (pair == 0 ? 0 : (size_t)(2 + pair - 1) * n);
            im = mom + (pair == 0 ? n : (size_t)(2 + D + pair - 1) * n);
        } else {
            hipLaunchKernelGGL((sk_field_kernel<L>), gb, tb, 0, stream, mom, Z, g, pair, -p.G);
            LAUNCH_CHECK();
        }
        if (fmlb_status st = dft_field(g, stream, Z, re, im)) return st;
        const int kind = pair == 0 ? 0 : (pair <= D ? 1 : 2);
        hipLaunchKernelGGL(sk_pair_accum_kernel, gb, tb, 0, stream, (const double2 *)Z, acc, g, kind,
                           kind == 0 ? inv_n : inv_n / D);
        LAUNCH_CHECK();
    }
    return FMLB_OK;
}

constexpr size_t kSkStaticBytes = (size_t)FMLB_SK_STATIC_MAX_SITES * kSkWorkBytesPerSite;

}  // namespace

// Work arrays of fmlb_sk_accumulate_static: one copy per GPU, held until the
// process ends.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device (static_scratch()).
static __device__ __align__(256) unsigned char scratch[kSkStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per device).
fmlb_status static_scratch(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return FMLB_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return FMLB_E_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FMLB_OK;
}

}  // namespace

extern "C" {

size_t fmlb_required_bytes(const fmlb_params *p, int which)
{
    if (!valid_params(p)) return 0;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const int Q = lattice_q(p->lattice);
    switch (which) {
    case FMLB_BUF_POPS_A:
    case FMLB_BUF_POPS_B: return align256(2 * (size_t)Q * n * elem_size(p->storage));
    case FMLB_BUF_SCRATCH: return scratch_layout(p).total;
    }
    return 0;
}

fmlb_status fmlb_create(const fmlb_params *p, void *hip_stream, void *const dev_buf[3], fmlb_ctx **out)
{
    if (!p || !dev_buf || !out) return FMLB_E_NULL;
    if (!dev_buf[0] || !dev_buf[1] || !dev_buf[2]) return FMLB_E_NULL;
    if (!valid_params(p)) return FMLB_E_INVALID;
    for (int k = 0; k < 3; ++k)
        if (reinterpret_cast<uintptr_t>(dev_buf[k]) % 256 != 0) return FMLB_E_INVALID;
    fmlb_ctx *c = new (std::nothrow) fmlb_ctx();
    if (!c) return FMLB_E_INVALID;
    c->p = *p;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->pops[0] = dev_buf[0];
    c->pops[1] = dev_buf[1];
    c->scratch = reinterpret_cast<unsigned char *>(dev_buf[2]);
    c->lay = scratch_layout(p);
    c->g = Geom{p->nx, p->ny, p->nz, (size_t)p->nx * p->ny * p->nz, (size_t)p->nx * p->ny * p->nz};
    c->Q = lattice_q(p->lattice);
    c->D = lattice_d(p->lattice);
    c->cur = 0;
    c->step = 0;
    c->ready = false;
    c->sk_samples = c->mode_samples = 0;
    c->tile_x = c->tile_y = c->march = 0;
    *out = c;
    return fmlb_reset_accumulators(c);
}

void fmlb_destroy(fmlb_ctx *c) { delete c; }

fmlb_status fmlb_init_density(fmlb_ctx *c, const double *rho1, const double *rho2)
{
    if (!c || !rho1 || !rho2) return FMLB_E_NULL;
    const size_t n = c->g.nsites;
    double *stage = scr<double>(c, c->lay.stage);
    HIP_TRY(hipMemcpyAsync(stage, rho1, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(stage + n, rho2, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        const SiteGrid sg = site_grid(c->g);
        hipLaunchKernelGGL((init_kernel<L, S>), sg.grid, sg.block, 0, c->stream, reinterpret_cast<S *>(c->pops[0]),
                           (const double *)stage, c->g, ref_of<S>(c, 0), ref_of<S>(c, 1));
        LAUNCH_CHECK();
        return FMLB_OK;
    });
    if (st) return st;
    c->cur = 0;
    c->step = 0;
    c->ready = true;
    return sync(c);
}

fmlb_status fmlb_step(fmlb_ctx *c, int64_t n)
{
    if (!c) return FMLB_E_NULL;
    if (n < 0) return FMLB_E_INVALID;
    if (!c->ready) return FMLB_E_STATE;
    return dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        return run_steps<L, S>(c, n);
    });
}

int64_t fmlb_current_step(const fmlb_ctx *c) { return c ? c->step : -1; }

fmlb_status fmlb_moments(fmlb_ctx *c, double *rho, double *j)
{
    if (!c) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    const size_t n = c->g.nsites;
    double *stage = scr<double>(c, c->lay.stage);
    const int ncomp = 2 + 2 * c->D;
    for (int k = 0; k < ncomp; ++k) {
        double *dst = k < 2 ? (rho ? rho + (size_t)k * n : nullptr) : (j ? j + (size_t)(k - 2) * n : nullptr);
        if (!dst) continue;
        fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
            using L = decltype(l);
            using S = std::remove_pointer_t<decltype(sp)>;
            hipLaunchKernelGGL((moment_field_kernel<L, S>), dim3(stride_blocks(n)), dim3(256), 0, c->stream,
                               reinterpret_cast<const S *>(c->pops[c->cur]), stage, c->g, k, ref_of<S>(c, 0),
                               ref_of<S>(c, 1));
            LAUNCH_CHECK();
            return FMLB_OK;
        });
        if (st) return st;
        HIP_TRY(hipMemcpyAsync(dst, stage, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (fmlb_status s2 = sync(c)) return s2;
    }
    return FMLB_OK;
}

fmlb_status fmlb_global_sums(fmlb_ctx *c, double *out)
{
    if (!c || !out) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    const size_t n = c->g.nsites;
    const int nb = stride_blocks(n);
    double *partial = scr<double>(c, c->lay.partial);
    double *misc = scr<double>(c, c->lay.misc);
    const int nv = 2 + c->D;
    fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        hipLaunchKernelGGL((sums_kernel<L, S>), dim3(nb), dim3(kRedBlock), 0, c->stream,
                           reinterpret_cast<const S *>(c->pops[c->cur]), partial, c->g, ref_of<S>(c, 0),
                           ref_of<S>(c, 1));
        LAUNCH_CHECK();
        return FMLB_OK;
    });
    if (st) return st;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedBlock), 0, c->stream, (const double *)partial, nb, nv,
                       misc, (double *)nullptr);
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(out, misc, nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

fmlb_status fmlb_mode_accumulate(fmlb_ctx *c)
{
    if (!c) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    const size_t n = c->g.nsites;
    const int nb = stride_blocks(n);
    double *partial = scr<double>(c, c->lay.partial);
    double *acc = scr<double>(c, c->lay.modeacc);
    fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        hipLaunchKernelGGL((mode_stats_kernel<L, S>), dim3(nb), dim3(kRedBlock), 0, c->stream,
                           reinterpret_cast<const S *>(c->pops[c->cur]), partial, c->g, ref_of<S>(c, 0),
                           ref_of<S>(c, 1));
        LAUNCH_CHECK();
        return FMLB_OK;
    });
    if (st) return st;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedBlock), 0, c->stream, (const double *)partial, nb,
                       4 * c->Q, (double *)nullptr, acc);
    LAUNCH_CHECK();
    c->mode_samples += 1;
    return FMLB_OK;
}

fmlb_status fmlb_mode_variances(fmlb_ctx *c, double *out, int64_t *n_samples)
{
    if (!c || !out) return FMLB_E_NULL;
    if (!(c->p.kT > 0.0)) return FMLB_E_INVALID;  // the ratio is defined for k_B T > 0
    if (c->mode_samples == 0) return FMLB_E_STATE;
    std::vector<double> acc(4 * c->Q);
    HIP_TRY(hipMemcpyAsync(acc.data(), scr<double>(c, c->lay.modeacc), acc.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    if (fmlb_status st = sync(c)) return st;
    const double cnt = (double)c->mode_samples * (double)c->g.nsites;
    const double mu = 3.0 * c->p.kT;
    for (int s = 0; s < 2; ++s) {
        // sampled mean density of the species: the mean of mode 0 (m_0 = rho)
        const double rho_mean = acc[(s * c->Q) * 2] / cnt;
        for (int a = 0; a < c->Q; ++a) {
            const double m1 = acc[(s * c->Q + a) * 2] / cnt;
            const double m2 = acc[(s * c->Q + a) * 2 + 1] / cnt;
            const double N = c->p.lattice == FMLB_D2Q9 ? (double)D2Q9::Nnum[a] / D2Q9::Nden[a]
                                                       : (double)D3Q19::Nnum[a] / D3Q19::Nden[a];
            out[s * c->Q + a] = rho_mean > 0.0 ? (m2 - m1 * m1) / (N * mu * rho_mean) : NAN;
        }
    }
    if (n_samples) *n_samples = c->mode_samples;
    return FMLB_OK;
}

fmlb_status fmlb_sk_accumulate(fmlb_ctx *c)
{
    if (!c) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    if (c->g.nx > kMaxLine || c->g.ny > kMaxLine || c->g.nz > kMaxLine) return FMLB_E_UNSUPPORTED;
    double2 *Z = scr<double2>(c, c->lay.skA);
    double *acc = scr<double>(c, c->lay.skacc);
    fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        return sk_accumulate_impl<L, S>(c->p, c->g, c->stream, reinterpret_cast<const S *>(c->pops[c->cur]),
                                        scr<double>(c, c->lay.skmom), Z, acc);
    });
    if (st) return st;
    c->sk_samples += 1;
    return FMLB_OK;
}

fmlb_status fmlb_sk_accumulate_static(const fmlb_params *p, const void *pops, double *acc, void *hip_stream)
{
    if (!p || !pops || !acc) return FMLB_E_NULL;
    if (!valid_params(p)) return FMLB_E_INVALID;
    const size_t nsites = (size_t)p->nx * p->ny * p->nz;
    const Geom g{p->nx, p->ny, p->nz, nsites, nsites};
    if (g.nsites > (size_t)FMLB_SK_STATIC_MAX_SITES) return FMLB_E_SIZE;
    if (g.nx > kMaxLine || g.ny > kMaxLine || g.nz > kMaxLine) return FMLB_E_UNSUPPORTED;
    void *base = nullptr;
    if (fmlb_status st = static_scratch(&base)) return st;
    // work arrays carved from the static array: the moments, then Z
    unsigned char *w = reinterpret_cast<unsigned char *>(base);
    double2 *Z = reinterpret_cast<double2 *>(w + (size_t)sk_moments(p->lattice) * g.nsites * sizeof(double));
    fmlb_ctx tmp{};
    tmp.p = *p;
    return dispatch(&tmp, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        return sk_accumulate_impl<L, S>(*p, g, reinterpret_cast<hipStream_t>(hip_stream),
                                        reinterpret_cast<const S *>(pops), reinterpret_cast<double *>(w), Z, acc);
    });
}

fmlb_status fmlb_sk_get(fmlb_ctx *c, int which, double *out, int64_t *n_samples)
{
    if (!c || !out) return FMLB_E_NULL;
    if (which < 0 || which >= kSkQuantities) return FMLB_E_INVALID;
    const size_t n = c->g.nsites;
    HIP_TRY(hipMemcpyAsync(out, scr<double>(c, c->lay.skacc) + (size_t)which * n, n * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    if (fmlb_status st = sync(c)) return st;
    if (c->sk_samples > 0)
        for (size_t t = 0; t < n; ++t) out[t] /= (double)c->sk_samples;
    if (n_samples) *n_samples = c->sk_samples;
    return FMLB_OK;
}

fmlb_status fmlb_reset_accumulators(fmlb_ctx *c)
{
    if (!c) return FMLB_E_NULL;
    const size_t n = c->g.nsites;
    hipLaunchKernelGGL(fill_kernel, dim3(stride_blocks(kSkQuantities * n)), dim3(256), 0, c->stream,
                       scr<double>(c, c->lay.skacc), (size_t)kSkQuantities * n, 0.0);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, c->stream, scr<double>(c, c->lay.modeacc),
                       (size_t)4 * c->Q, 0.0);
    LAUNCH_CHECK();
    c->sk_samples = 0;
    c->mode_samples = 0;
    return FMLB_OK;
}

fmlb_status fmlb_get_populations(fmlb_ctx *c, double *host, size_t bytes)
{
    if (!c || !host) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    const size_t n = c->g.nsites;
    if (bytes < 2 * (size_t)c->Q * n * sizeof(double)) return FMLB_E_SIZE;
    double *stage = scr<double>(c, c->lay.stage);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < c->Q; ++i) {
            fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
                using L = decltype(l);
                using S = std::remove_pointer_t<decltype(sp)>;
                const SiteGrid sg = site_grid(c->g);
                hipLaunchKernelGGL((gather_pop_kernel<L, S>), sg.grid, sg.block, 0, c->stream,
                                   reinterpret_cast<const S *>(c->pops[c->cur]), stage, c->g, s, i, ref_of<S>(c, s));
                LAUNCH_CHECK();
                return FMLB_OK;
            });
            if (st) return st;
            HIP_TRY(hipMemcpyAsync(host + ((size_t)s * c->Q + i) * n, stage, n * sizeof(double),
                                   hipMemcpyDeviceToHost, c->stream));
            if (fmlb_status s2 = sync(c)) return s2;
        }
    return FMLB_OK;
}

fmlb_status fmlb_set_populations(fmlb_ctx *c, const double *host, size_t bytes, int64_t step)
{
    if (!c || !host) return FMLB_E_NULL;
    if (step < 0) return FMLB_E_INVALID;
    const size_t n = c->g.nsites;
    if (bytes < 2 * (size_t)c->Q * n * sizeof(double)) return FMLB_E_SIZE;
    double *stage = scr<double>(c, c->lay.stage);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < c->Q; ++i) {
            HIP_TRY(hipMemcpyAsync(stage, host + ((size_t)s * c->Q + i) * n, n * sizeof(double),
                                   hipMemcpyHostToDevice, c->stream));
            fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
                using L = decltype(l);
                using S = std::remove_pointer_t<decltype(sp)>;
                const SiteGrid sg = site_grid(c->g);
                hipLaunchKernelGGL((scatter_pop_kernel<L, S>), sg.grid, sg.block, 0, c->stream,
                                   reinterpret_cast<S *>(c->pops[0]), (const double *)stage, c->g, s, i,
                                   ref_of<S>(c, s));
                LAUNCH_CHECK();
                return FMLB_OK;
            });
            if (st) return st;
            if (fmlb_status s2 = sync(c)) return s2;
        }
    c->cur = 0;
    c->step = step;
    c->ready = true;
    return FMLB_OK;
}

fmlb_status fmlb_save_raw(fmlb_ctx *c, void *host, size_t bytes, int64_t *step)
{
    if (!c || !host) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    const size_t need = 2 * (size_t)c->Q * c->g.nsites * elem_size(c->p.storage);
    if (bytes < need) return FMLB_E_SIZE;
    HIP_TRY(hipMemcpyAsync(host, c->pops[c->cur], need, hipMemcpyDeviceToHost, c->stream));
    if (step) *step = c->step;
    return sync(c);
}

fmlb_status fmlb_load_raw(fmlb_ctx *c, const void *host, size_t bytes, int64_t step)
{
    if (!c || !host) return FMLB_E_NULL;
    if (step < 0) return FMLB_E_INVALID;
    const size_t need = 2 * (size_t)c->Q * c->g.nsites * elem_size(c->p.storage);
    if (bytes < need) return FMLB_E_SIZE;
    HIP_TRY(hipMemcpyAsync(c->pops[0], host, need, hipMemcpyHostToDevice, c->stream));
    c->cur = 0;
    c->step = step;
    c->ready = true;
    return sync(c);
}

fmlb_status fmlb_health(fmlb_ctx *c, int64_t counts[2])
{
    if (!c || !counts) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    const size_t n = c->g.nsites;
    const int nb = stride_blocks(n);
    double *partial = scr<double>(c, c->lay.partial);
    double *misc = scr<double>(c, c->lay.misc);
    fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        hipLaunchKernelGGL((health_kernel<L, S>), dim3(nb), dim3(kRedBlock), 0, c->stream,
                           reinterpret_cast<const S *>(c->pops[c->cur]), partial, c->g, ref_of<S>(c, 0),
                           ref_of<S>(c, 1));
        LAUNCH_CHECK();
        return FMLB_OK;
    });
    if (st) return st;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedBlock), 0, c->stream, (const double *)partial, nb, 2,
                       misc, (double *)nullptr);
    LAUNCH_CHECK();
    double h[2];
    HIP_TRY(hipMemcpyAsync(h, misc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    if (fmlb_status s2 = sync(c)) return s2;
    counts[0] = (int64_t)h[0];
    counts[1] = (int64_t)h[1];
    return FMLB_OK;
}

fmlb_status fmlb_set_counter_offset(fmlb_ctx *c, int64_t site_offset)
{
    if (!c) return FMLB_E_NULL;
    if (site_offset < 0 || site_offset > (int64_t)UINT32_MAX) return FMLB_E_INVALID;
    c->site_off = (uint32_t)site_offset;
    return FMLB_OK;
}

fmlb_status fmlb_set_tile(fmlb_ctx *c, int tile_x, int tile_y, int march)
{
    if (!c) return FMLB_E_NULL;
    if (tile_x < 0 || tile_y < 0 || march < 0) return FMLB_E_INVALID;
    fmlb_status st = dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        if (tile_x == 1) return FMLB_OK;  // two-pass form
        if (march > 4096) return FMLB_E_INVALID;
        if (tile_x == 0 && tile_y == 0) return FMLB_OK;  // default tile, given or default march
        if (!fused_shape_valid<L, S>(tile_x, tile_y, march)) return FMLB_E_INVALID;
        if (!fused_supported<L, S>(c->g, tile_x, tile_y, march)) return FMLB_E_INVALID;
        return FMLB_OK;
    });
    if (st) return st;
    c->tile_x = tile_x;
    c->tile_y = tile_y;
    c->march = march;
    return FMLB_OK;
}

const char *fmlb_status_string(fmlb_status s)
{
    switch (s) {
    case FMLB_OK: return "ok";
    case FMLB_E_INVALID: return "invalid parameter";
    case FMLB_E_SIZE: return "buffer too small";
    case FMLB_E_HIP: return "HIP error";
    case FMLB_E_STATE: return "populations not initialised";
    case FMLB_E_NULL: return "null pointer";
    case FMLB_E_UNSUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}

fmlb_status fmlb_copy_reference(fmlb_ctx *c)
{
    if (!c) return FMLB_E_NULL;
    if (!c->ready) return FMLB_E_STATE;
    return dispatch(c, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        const SiteGrid sg = site_grid(c->g);
        hipLaunchKernelGGL((pull_copy_kernel<L, S>), sg.grid, sg.block, 0, c->stream,
                           reinterpret_cast<const S *>(c->pops[c->cur]), reinterpret_cast<S *>(c->pops[1 - c->cur]),
                           c->g);
        LAUNCH_CHECK();
        return FMLB_OK;
    });
}

fmlb_status fmlb_bandwidth_reference(fmlb_ctx *c, int kind, double *bytes)
{
    if (!c) return FMLB_E_NULL;
    if (kind < 0 || kind > FMLB_BW_COPY16) return FMLB_E_INVALID;
    if (!c->ready) return FMLB_E_STATE;
    const size_t buf = 2 * (size_t)c->Q * c->g.nsites * elem_size(c->p.storage);
    const size_t words = buf / 16;  // the last buf % 16 bytes are left out
    const void *src = c->pops[c->cur];
    void *dst = c->pops[1 - c->cur];
    switch (kind) {
    case FMLB_BW_PULL_COPY:
        if (bytes) *bytes = 2.0 * (double)buf;
        return fmlb_copy_reference(c);
    case FMLB_BW_READ:
        hipLaunchKernelGGL(stream_read_kernel, dim3(2048), dim3(256), 0, c->stream, (const float4_v *)src, words,
                           scr<float>(c, c->lay.misc));
        if (bytes) *bytes = 16.0 * (double)words;
        break;
    case FMLB_BW_WRITE:
        hipLaunchKernelGGL(stream_write_kernel, dim3(256), dim3(256), 0, c->stream, (float4_v *)dst, words);
        if (bytes) *bytes = 16.0 * (double)words;
        break;
    case FMLB_BW_COPY16:
        hipLaunchKernelGGL((stream_copy_kernel<4>), dim3(256), dim3(256), 0, c->stream, (const float4_v *)src,
                           (float4_v *)dst, words);
        if (bytes) *bytes = 32.0 * (double)words;
        break;
    }
    LAUNCH_CHECK();
    return FMLB_OK;
}

int32_t fmlb_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
