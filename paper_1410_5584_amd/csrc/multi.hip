// Host runtime of the N-species entry points (fmlb_multi_*, include/fmlb.h):
// validation, buffer carving, dispatch over (lattice, storage, N), host
// transfers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/fmlb.h"
#include "multi.h"

using namespace fmlb;

namespace fmlb {
extern thread_local int32_t g_last_hip;
}

namespace {

#define MULTI_TRY(...)                                 \
    do {                                               \
        hipError_t e_ = (__VA_ARGS__);                 \
        if (e_ != hipSuccess) {                        \
            g_last_hip = (int32_t)e_;                  \
            return FMLB_E_HIP;                         \
        }                                              \
    } while (0)

constexpr int kMultiBlocks = 512;  // reduction blocks (partial sums)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_multi(const fmlb_multi_params *p)
{
    if (!p) return false;
    if (p->lattice != FMLB_D2Q9 && p->lattice != FMLB_D3Q19) return false;
    if (p->storage != FMLB_F64 && p->storage != FMLB_F32) return false;
    if (p->flags & ~(uint32_t)(FMLB_NOISE_OFF | FMLB_NOISE_NO_SDF)) return false;
    if (p->nspecies < 2 || p->nspecies > FMLB_MAX_SPECIES) return false;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
    if (p->lattice == FMLB_D2Q9 && p->nz != 1) return false;
    if ((double)p->nx * (double)p->ny * (double)p->nz >= 2147483648.0) return false;
    if (!(p->tau_d > 0.5) || !std::isfinite(p->tau_d)) return false;
    if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return false;
    for (int s = 0; s < p->nspecies; ++s) {
        if (!(p->tau[s] > 0.5) || !std::isfinite(p->tau[s])) return false;
        if (!std::isfinite(p->rho_ref[s])) return false;
        for (int t = 0; t < p->nspecies; ++t)
            if (!std::isfinite(p->G[s][t]) || p->G[s][t] != p->G[t][s]) return false;
    }
    return true;
}

struct MultiLayout {
    size_t phi, stage, partial, total;
};

MultiLayout multi_layout(const fmlb_multi_params *p)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const size_t real = p->storage == FMLB_F64 ? 8 : 4;
    MultiLayout l{};
    size_t o = 0;
    l.phi = o;
    o += align_up((size_t)p->nspecies * n * real);
    l.stage = o;
    o += align_up(4 * n * sizeof(double));  // rho and up to 3 momentum components
    l.partial = o;
    o += align_up((size_t)kMultiBlocks * 4 * sizeof(double));
    l.total = o;
    return l;
}

}  // namespace

struct fmlb_multi {
    fmlb_multi_params p;
    hipStream_t stream;
    void *pops[2];
    unsigned char *scratch;
    MultiLayout lay;
    Geom g;
    int Q, D, N;
    int cur;
    int64_t step;
    bool ready;
    int form;                   // FMLB_MULTI_*
    int tile_x, tile_y, march;  // 0: defaults
};

namespace {

template <class F>
fmlb_status multi_dispatch(const fmlb_multi *m, F &&f)
{
    const bool d3 = m->p.lattice == FMLB_D3Q19, f64 = m->p.storage == FMLB_F64;
    if (d3 && f64) return f(D3Q19{}, (double *)nullptr);
    if (d3) return f(D3Q19{}, (float *)nullptr);
    if (f64) return f(D2Q9{}, (double *)nullptr);
    return f(D2Q9{}, (float *)nullptr);
}

struct Grid {
    dim3 grid, block;
};

Grid multi_grid(const Geom &g)
{
    const int bx = g.nx >= 256 ? 256 : ((g.nx + 63) / 64) * 64;
    return Grid{dim3((g.nx + bx - 1) / bx, g.ny, g.nz), dim3(bx)};
}

template <class Real>
MultiPhys<Real> multi_phys(const fmlb_multi_params &p)
{
    MultiPhys<Real> ph{};
    const bool noisy = p.kT > 0.0 && !(p.flags & FMLB_NOISE_OFF);
    const bool sdf = noisy && !(p.flags & FMLB_NOISE_NO_SDF);
    const double mu = 3.0 * p.kT;  // mu = k_B T / c_s^2
    const double lam_d = 1.0 / p.tau_d;
    ph.lam_d = (Real)lam_d;
    ph.sd2 = sdf ? (Real)((2.0 * lam_d - lam_d * lam_d) * p.kT) : (Real)0;
    for (int s = 0; s < kMaxSpecies; ++s) {
        const bool in = s < p.nspecies;
        const double lam = in ? 1.0 / p.tau[s] : 1.0;
        ph.lam[s] = (Real)lam;
        ph.gain[s] = (in && noisy) ? (Real)std::sqrt((2.0 * lam - lam * lam) * mu) : (Real)0;
        ph.ref[s] = (in && p.storage != FMLB_F64) ? (Real)p.rho_ref[s] : (Real)0;
        for (int t = 0; t < kMaxSpecies; ++t) ph.G[s][t] = (in && t < p.nspecies) ? (Real)p.G[s][t] : (Real)0;
    }
    ph.key0 = (uint32_t)p.seed;
    ph.key1 = (uint32_t)(p.seed >> 32);
    return ph;
}

double ref_of(const fmlb_multi *m, int s) { return m->p.storage == FMLB_F64 ? 0.0 : m->p.rho_ref[s]; }

// Fused tiles: D3Q19 64x4, 64x8, 32x8; D2Q9 64x1, 128x1, 256x1.
bool multi_tile_valid(int D, int tx, int ty)
{
    if (D == 3) return (tx == 64 && (ty == 4 || ty == 8)) || (tx == 32 && ty == 8);
    return ty == 1 && (tx == 64 || tx == 128 || tx == 256);
}

// Asynchronous tiles: D3Q19 64x4, 64x8, 32x8, 32x4; D2Q9 64x1, 128x1, 256x1;
// each where its LDS fits.
bool multi_async_tile_valid(int D, int N, int tx, int ty)
{
    const bool shape = D == 3 ? (tx == 64 && (ty == 4 || ty == 8)) || (tx == 32 && (ty == 8 || ty == 4))
                              : ty == 1 && (tx == 64 || tx == 128 || tx == 256);
    return shape && multi_async_lds_bytes(D, D == 3 ? 19 : 9, N, tx, ty) <= kMaxLdsBytes;
}

// The asynchronous form runs FP32 storage whose species arrays are
// addressable by 32-bit buffer offsets.
bool multi_async_supported(const fmlb_multi *m)
{
    return m->p.storage == FMLB_F32 && (double)m->Q * (double)m->g.nsites * 4.0 < 4294967295.0;
}

// Default march of a fused tile: the longest that still gives about two
// workgroups per CU.
void multi_default_tile(const fmlb_multi *m, int &tx, int &ty, int &march)
{
    const Geom &g = m->g;
    if (m->tile_x > 1) {
        tx = m->tile_x;
        ty = m->tile_y;
    } else if (m->D == 3) {
        tx = 64;
        ty = 8;
    } else {
        tx = g.nx >= 256 ? 256 : (g.nx >= 128 ? 128 : 64);
        ty = 1;
    }
    const long cols = (long)((g.nx + tx - 1) / tx) * (m->D == 3 ? (long)((g.ny + ty - 1) / ty) : 1L);
    const int nm = m->D == 3 ? g.nz : g.ny;
    march = 1;
    while (march < 64 && cols * ((nm + 2L * march - 1) / (2L * march)) >= 512) march *= 2;
}

template <class L, class S, int N, int T0, int T1>
hipError_t multi_fused_launch(const MultiArgs<S> &a, int march, hipStream_t stream)
{
    const Geom &g = a.g;
    const int n1 = L::D == 3 ? g.ny : 1, nm = L::D == 3 ? g.nz : g.ny;
    const unsigned blocks = (unsigned)((g.nx + T0 - 1) / T0) * (unsigned)((n1 + T1 - 1) / T1) *
                            (unsigned)((nm + march - 1) / march);
    hipLaunchKernelGGL((multi_fused_kernel<L, S, N, T0, T1>), dim3(blocks), dim3(T0 * T1), 0, stream, a, march);
    return hipGetLastError();
}

template <class L, class S, int N>
hipError_t multi_fused_dispatch(const MultiArgs<S> &a, int tx, int ty, int march, hipStream_t stream)
{
    if constexpr (L::D == 3) {
        if (tx == 64 && ty == 4) return multi_fused_launch<L, S, N, 64, 4>(a, march, stream);
        if (tx == 64 && ty == 8) return multi_fused_launch<L, S, N, 64, 8>(a, march, stream);
        return multi_fused_launch<L, S, N, 32, 8>(a, march, stream);
    } else {
        if (tx == 64) return multi_fused_launch<L, S, N, 64, 1>(a, march, stream);
        if (tx == 128) return multi_fused_launch<L, S, N, 128, 1>(a, march, stream);
        return multi_fused_launch<L, S, N, 256, 1>(a, march, stream);
    }
}

// Default tile of the asynchronous form.
void multi_async_default(const fmlb_multi *m, int &tx, int &ty)
{
    const Geom &g = m->g;
    if (m->tile_x > 1) {
        tx = m->tile_x;
        ty = m->tile_y;
    } else if (m->D == 3) {
        // measured at 256^3: two species 1.20 ms with 64x8 against 1.30 with
        // 64x4 (two workgroups per CU); three and four species only fit 64x4
        tx = 64;
        ty = multi_async_tile_valid(3, m->N, 64, 8) ? 8 : 4;
    } else {
        tx = g.nx >= 256 ? 256 : (g.nx >= 128 ? 128 : 64);
        ty = 1;
    }
}

constexpr int kComputeUnits = 256;  // MI355X

// march 0: the longest march (a power of two) that still gives every CU as
// many workgroups as fit on it at once (LDS and registers decide how many);
// longer marches re-read fewer halo planes.
template <class L, int N, int T0, int T1>
hipError_t multi_async_launch(const MultiArgs<float> &a, int march, hipStream_t stream)
{
    const Geom &g = a.g;
    const int n1 = L::D == 3 ? g.ny : 1, nm = L::D == 3 ? g.nz : g.ny;
    const long cols = (long)((g.nx + T0 - 1) / T0) * (long)((n1 + T1 - 1) / T1);
    if (march == 0) {
        static std::atomic<int> cached{0};  // the same for every device of this kind
        int per_cu = cached.load(std::memory_order_relaxed);
        if (per_cu == 0) {
            const hipError_t e =
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, multi_async_kernel<L, N, T0, T1>, T0 * T1, 0);
            if (e != hipSuccess) return e;
            cached.store(per_cu, std::memory_order_relaxed);
        }
        const long target = (long)kComputeUnits * (per_cu > 0 ? per_cu : 1);
        march = 1;
        while (march < 4096 && cols * ((nm + 2L * march - 1) / (2L * march)) >= target) march *= 2;
    }
    const unsigned blocks = (unsigned)cols * (unsigned)((nm + march - 1) / march);
    hipLaunchKernelGGL((multi_async_kernel<L, N, T0, T1>), dim3(blocks), dim3(T0 * T1), 0, stream, a, march);
    return hipGetLastError();
}

template <class L, int N>
hipError_t multi_async_dispatch(const MultiArgs<float> &a, int tx, int ty, int march, hipStream_t stream)
{
    if constexpr (L::D == 3) {
        constexpr bool fits8 = multi_async_lds_bytes(3, 19, N, 64, 8) <= kMaxLdsBytes;
        if (tx == 64 && ty == 4) return multi_async_launch<L, N, 64, 4>(a, march, stream);
        if constexpr (fits8)
            if (tx == 64 && ty == 8) return multi_async_launch<L, N, 64, 8>(a, march, stream);
        if (ty == 8) return multi_async_launch<L, N, 32, 8>(a, march, stream);
        return multi_async_launch<L, N, 32, 4>(a, march, stream);
    } else {
        if (tx == 64) return multi_async_launch<L, N, 64, 1>(a, march, stream);
        if (tx == 128) return multi_async_launch<L, N, 128, 1>(a, march, stream);
        return multi_async_launch<L, N, 256, 1>(a, march, stream);
    }
}

template <class L, class S, int N>
fmlb_status multi_run(fmlb_multi *m, int64_t n)
{
    using Real = typename Storage<S>::Real;
    const Grid gr = multi_grid(m->g);
    // Default: the asynchronous single pass where it applies, else the
    // two-pass form (the register single pass is slower than both).
    int form = m->form;
    if (form == FMLB_MULTI_AUTO) form = multi_async_supported(m) ? FMLB_MULTI_ASYNC : FMLB_MULTI_TWO_PASS;
    int tx = 0, ty = 0, march = 0;
    if (form == FMLB_MULTI_FUSED) multi_default_tile(m, tx, ty, march);
    if (form == FMLB_MULTI_ASYNC) {
        multi_async_default(m, tx, ty);
        march = m->march;
    }

    if (form == FMLB_MULTI_FUSED && m->march != 0) march = m->march;
    for (int64_t t = 0; t < n; ++t) {
        MultiArgs<S> a{};
        a.src = reinterpret_cast<const S *>(m->pops[m->cur]);
        a.dst = reinterpret_cast<S *>(m->pops[1 - m->cur]);
        a.phi = reinterpret_cast<Real *>(m->scratch + m->lay.phi);
        a.g = m->g;
        a.ph = multi_phys<Real>(m->p);
        a.step_lo = (uint32_t)(uint64_t)m->step;
        a.step_hi = (uint32_t)((uint64_t)m->step >> 32);
        if (form == FMLB_MULTI_ASYNC) {
            if constexpr (std::is_same<S, float>::value)
                MULTI_TRY(multi_async_dispatch<L, N>(a, tx, ty, march, m->stream));
            else
                return FMLB_E_INVALID;
        } else if (form == FMLB_MULTI_FUSED) {
            MULTI_TRY(multi_fused_dispatch<L, S, N>(a, tx, ty, march, m->stream));
        } else {
            hipLaunchKernelGGL((multi_potential_kernel<L, S, N>), gr.grid, gr.block, 0, m->stream, a);
            MULTI_TRY(hipGetLastError());
            hipLaunchKernelGGL((multi_step_kernel<L, S, N>), gr.grid, gr.block, 0, m->stream, a);
            MULTI_TRY(hipGetLastError());
        }
        m->cur = 1 - m->cur;
        m->step += 1;
    }
    return FMLB_OK;
}

}  // namespace

extern "C" {

size_t fmlb_multi_required_bytes(const fmlb_multi_params *p, int which)
{
    if (!valid_multi(p)) return 0;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const int Q = p->lattice == FMLB_D2Q9 ? 9 : 19;
    const size_t elem = p->storage == FMLB_F64 ? 8 : 4;
    switch (which) {
    case FMLB_BUF_POPS_A:
    case FMLB_BUF_POPS_B: return align_up((size_t)p->nspecies * Q * n * elem);
    case FMLB_BUF_SCRATCH: return multi_layout(p).total;
    }
    return 0;
}

fmlb_status fmlb_multi_create(const fmlb_multi_params *p, void *hip_stream, void *const dev_buf[3], fmlb_multi **out)
{
    if (!p || !dev_buf || !out) return FMLB_E_NULL;
    if (!dev_buf[0] || !dev_buf[1] || !dev_buf[2]) return FMLB_E_NULL;
    *out = nullptr;
    if (!valid_multi(p)) return FMLB_E_INVALID;
    for (int b = 0; b < 3; ++b)
        if (((uintptr_t)dev_buf[b] & 255) != 0) return FMLB_E_INVALID;
    fmlb_multi *m = new (std::nothrow) fmlb_multi{};
    if (!m) return FMLB_E_HIP;
    m->p = *p;
    m->stream = (hipStream_t)hip_stream;
    m->pops[0] = dev_buf[0];
    m->pops[1] = dev_buf[1];
    m->scratch = (unsigned char *)dev_buf[2];
    m->lay = multi_layout(p);
    m->g = Geom{p->nx, p->ny, p->nz, (size_t)p->nx * p->ny * p->nz, (size_t)p->nx * p->ny * p->nz};
    m->Q = p->lattice == FMLB_D2Q9 ? 9 : 19;
    m->D = p->lattice == FMLB_D2Q9 ? 2 : 3;
    m->N = p->nspecies;
    *out = m;
    return FMLB_OK;
}

void fmlb_multi_destroy(fmlb_multi *m) { delete m; }

int64_t fmlb_multi_current_step(const fmlb_multi *m) { return m ? m->step : -1; }

fmlb_status fmlb_multi_set_form(fmlb_multi *m, int form, int tile_x, int tile_y, int march)
{
    if (!m) return FMLB_E_NULL;
    if (tile_x < 0 || tile_y < 0 || march < 0 || march > 4096) return FMLB_E_INVALID;
    switch (form) {
    case FMLB_MULTI_AUTO:
    case FMLB_MULTI_TWO_PASS:
        if (tile_x != 0 || tile_y != 0 || march != 0) return FMLB_E_INVALID;
        break;
    case FMLB_MULTI_FUSED:
        if (tile_x != 0 && !multi_tile_valid(m->D, tile_x, tile_y)) return FMLB_E_INVALID;
        break;
    case FMLB_MULTI_ASYNC:
        if (!multi_async_supported(m)) return FMLB_E_UNSUPPORTED;
        if (tile_x != 0 && !multi_async_tile_valid(m->D, m->N, tile_x, tile_y)) return FMLB_E_INVALID;
        break;

    default: return FMLB_E_INVALID;
    }
    if (tile_x == 0 && tile_y != 0) return FMLB_E_INVALID;
    m->form = form;
    m->tile_x = tile_x;
    m->tile_y = tile_y;
    m->march = march;
    return FMLB_OK;
}

fmlb_status fmlb_multi_set_tile(fmlb_multi *m, int tile_x, int tile_y, int march)
{
    if (!m) return FMLB_E_NULL;
    if (tile_x == 0 && tile_y == 0 && march == 0) return fmlb_multi_set_form(m, FMLB_MULTI_AUTO, 0, 0, 0);
    if (tile_x == 1 && tile_y == 0 && march == 0) return fmlb_multi_set_form(m, FMLB_MULTI_TWO_PASS, 0, 0, 0);
    if (tile_x <= 1) return FMLB_E_INVALID;
    return fmlb_multi_set_form(m, FMLB_MULTI_FUSED, tile_x, tile_y, march);
}

fmlb_status fmlb_multi_init_density(fmlb_multi *m, const double *rho)
{
    if (!m || !rho) return FMLB_E_NULL;
    const size_t n = m->g.nsites;
    double *stage = reinterpret_cast<double *>(m->scratch + m->lay.stage);
    const Grid gr = multi_grid(m->g);
    const fmlb_status st = multi_dispatch(m, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        for (int s = 0; s < m->N; ++s) {
            MULTI_TRY(hipMemcpyAsync(stage, rho + (size_t)s * n, n * sizeof(double), hipMemcpyHostToDevice, m->stream));
            hipLaunchKernelGGL((multi_init_kernel<L, S>), gr.grid, gr.block, 0, m->stream,
                               reinterpret_cast<S *>(m->pops[0]), (const double *)stage, m->g, s, ref_of(m, s));
            MULTI_TRY(hipGetLastError());
            MULTI_TRY(hipStreamSynchronize(m->stream));  // the stage is reused
        }
        return FMLB_OK;
    });
    if (st != FMLB_OK) return st;
    m->cur = 0;
    m->step = 0;
    m->ready = true;
    return FMLB_OK;
}

fmlb_status fmlb_multi_step(fmlb_multi *m, int64_t n)
{
    if (!m) return FMLB_E_NULL;
    if (n < 0) return FMLB_E_INVALID;
    if (!m->ready) return FMLB_E_STATE;
    return multi_dispatch(m, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        switch (m->N) {
        case 2: return multi_run<L, S, 2>(m, n);
        case 3: return multi_run<L, S, 3>(m, n);
        case 4: return multi_run<L, S, 4>(m, n);
        }
        return FMLB_E_INVALID;
    });
}

fmlb_status fmlb_multi_get_populations(fmlb_multi *m, double *host, size_t bytes)
{
    if (!m || !host) return FMLB_E_NULL;
    if (!m->ready) return FMLB_E_STATE;
    const size_t n = m->g.nsites;
    if (bytes < (size_t)m->N * m->Q * n * sizeof(double)) return FMLB_E_SIZE;
    double *stage = reinterpret_cast<double *>(m->scratch + m->lay.stage);
    const Grid gr = multi_grid(m->g);
    return multi_dispatch(m, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        using Real = typename Storage<S>::Real;
        for (int s = 0; s < m->N; ++s)
            for (int i = 0; i < m->Q; ++i) {
                hipLaunchKernelGGL((gather_pop_kernel<L, S>), gr.grid, gr.block, 0, m->stream,
                                   reinterpret_cast<const S *>(m->pops[m->cur]), stage, m->g, s, i, (Real)ref_of(m, s));
                MULTI_TRY(hipGetLastError());
                MULTI_TRY(hipMemcpyAsync(host + ((size_t)s * m->Q + i) * n, stage, n * sizeof(double),
                                         hipMemcpyDeviceToHost, m->stream));
                MULTI_TRY(hipStreamSynchronize(m->stream));
            }
        return FMLB_OK;
    });
}

fmlb_status fmlb_multi_set_populations(fmlb_multi *m, const double *host, size_t bytes, int64_t step)
{
    if (!m || !host) return FMLB_E_NULL;
    if (step < 0) return FMLB_E_INVALID;
    const size_t n = m->g.nsites;
    if (bytes < (size_t)m->N * m->Q * n * sizeof(double)) return FMLB_E_SIZE;
    double *stage = reinterpret_cast<double *>(m->scratch + m->lay.stage);
    const Grid gr = multi_grid(m->g);
    const fmlb_status st = multi_dispatch(m, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        using Real = typename Storage<S>::Real;
        for (int s = 0; s < m->N; ++s)
            for (int i = 0; i < m->Q; ++i) {
                MULTI_TRY(hipMemcpyAsync(stage, host + ((size_t)s * m->Q + i) * n, n * sizeof(double),
                                         hipMemcpyHostToDevice, m->stream));
                hipLaunchKernelGGL((scatter_pop_kernel<L, S>), gr.grid, gr.block, 0, m->stream,
                                   reinterpret_cast<S *>(m->pops[0]), (const double *)stage, m->g, s, i,
                                   (Real)ref_of(m, s));
                MULTI_TRY(hipGetLastError());
                MULTI_TRY(hipStreamSynchronize(m->stream));
            }
        return FMLB_OK;
    });
    if (st != FMLB_OK) return st;
    m->cur = 0;
    m->step = step;
    m->ready = true;
    return FMLB_OK;
}

fmlb_status fmlb_multi_moments(fmlb_multi *m, double *rho, double *j)
{
    if (!m) return FMLB_E_NULL;
    if (!m->ready) return FMLB_E_STATE;
    const size_t n = m->g.nsites;
    double *stage = reinterpret_cast<double *>(m->scratch + m->lay.stage);
    const Grid gr = multi_grid(m->g);
    return multi_dispatch(m, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        for (int s = 0; s < m->N; ++s) {
            hipLaunchKernelGGL((multi_moment_kernel<L, S>), gr.grid, gr.block, 0, m->stream,
                               reinterpret_cast<const S *>(m->pops[m->cur]), stage, m->g, s, ref_of(m, s));
            MULTI_TRY(hipGetLastError());
            if (rho)
                MULTI_TRY(hipMemcpyAsync(rho + (size_t)s * n, stage, n * sizeof(double), hipMemcpyDeviceToHost,
                                         m->stream));
            if (j)
                MULTI_TRY(hipMemcpyAsync(j + (size_t)s * m->D * n, stage + n, (size_t)m->D * n * sizeof(double),
                                         hipMemcpyDeviceToHost, m->stream));
            MULTI_TRY(hipStreamSynchronize(m->stream));
        }
        return FMLB_OK;
    });
}

fmlb_status fmlb_multi_global_sums(fmlb_multi *m, double *out)
{
    if (!m || !out) return FMLB_E_NULL;
    if (!m->ready) return FMLB_E_STATE;
    double *partial = reinterpret_cast<double *>(m->scratch + m->lay.partial);
    const size_t blocks = std::min<size_t>(kMultiBlocks, (m->g.nsites + 255) / 256);
    std::vector<double> host(blocks * 4);
    for (int a = 0; a < m->N + m->D; ++a) out[a] = 0.0;
    return multi_dispatch(m, [&](auto l, auto sp) -> fmlb_status {
        using L = decltype(l);
        using S = std::remove_pointer_t<decltype(sp)>;
        for (int s = 0; s < m->N; ++s) {
            hipLaunchKernelGGL((multi_sums_kernel<L, S>), dim3((unsigned)blocks), dim3(256), 0, m->stream,
                               reinterpret_cast<const S *>(m->pops[m->cur]), partial, m->g, s, ref_of(m, s));
            MULTI_TRY(hipGetLastError());
            MULTI_TRY(hipMemcpyAsync(host.data(), partial, blocks * 4 * sizeof(double), hipMemcpyDeviceToHost,
                                     m->stream));
            MULTI_TRY(hipStreamSynchronize(m->stream));
            for (size_t b = 0; b < blocks; ++b) {
                out[s] += host[b * 4];
                for (int al = 0; al < m->D; ++al) out[m->N + al] += host[b * 4 + 1 + al];
            }
        }
        return FMLB_OK;
    });
}

}  // extern "C"
