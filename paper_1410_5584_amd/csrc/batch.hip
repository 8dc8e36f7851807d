// Batched replicas: many independent D2Q9 FP32 lattices advanced by one
// launch per step (two when some replicas are too wide to pack).  The
// launch covers a work list of items: packed runs of a replica's sites
// (batch_pack_walk) or one-row tiles (the single-lattice fused_tile_async),
// each with the replica's own geometry, parameters, seed and site
// numbering and the single lattice's per-site helpers, so every replica
// evolves bit for bit as it would alone.  Each replica's population arrays
// are padded to a multiple of 64 floats (Geom::pitch).
//
// The step number lives in device memory and every launch reads it, so a
// captured HIP graph of several steps can be replayed any number of times:
// its last node advances the counter.  Buffer parity follows the step number
// (step n's pre-collision state sits in population buffer n mod 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/fmlb.h"
#include "fused.h"
#include "observables.h"

using namespace fmlb;

namespace fmlb {
extern thread_local int32_t g_last_hip;  // defined with the single-lattice entry points
}  // namespace fmlb

namespace {

#define BATCH_TRY(...)                                 \
    do {                                               \
        hipError_t e_ = (__VA_ARGS__);                 \
        if (e_ != hipSuccess) {                        \
            g_last_hip = (int32_t)e_;                   \
            return FMLB_E_HIP;                         \
        }                                              \
    } while (0)

constexpr int kQ = 9;
constexpr int kBatchReduceBlocks = 256;
constexpr int kGraphSteps = 32;  // steps per captured graph
constexpr int kMinTile = 64;     // narrowest supported tile (sizes the work list)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchRep {
    uint64_t off;     // element offset of the replica's [2][Q][sites] block in each buffer
    Geom g;
    Phys<float> ph;
    float ref[2];
};

struct SiteGrid2 {
    dim3 grid, block;
};

struct BatchItem {
    uint32_t rep;
    uint32_t tile_chunk;  // tile index << 16 | chunk index
};

// Elements per population array of a replica: the site count rounded up to
// 64 (256 bytes), so that every array starts on a cache-line boundary (an
// odd site count otherwise shifts every array but the first: 231 replicas
// of 181^2 ran at 0.281 ms per step against 0.214-0.224 for power-of-two
// widths of the same total size).
size_t replica_pitch(const fmlb_params &p) { return ((size_t)p.nx * p.ny + 63) & ~(size_t)63; }

bool valid_replica(const fmlb_params &p)
{
    if (p.lattice != FMLB_D2Q9 || p.storage != FMLB_F32) return false;
    if (p.flags & ~(uint32_t)(FMLB_NOISE_OFF | FMLB_NOISE_NO_SDF)) return false;
    if (p.nx < 1 || p.ny < 1 || p.nz != 1) return false;
    if (p.nx > 65535 * kMinTile || p.ny > 65535) return false;
    if ((double)replica_pitch(p) * kQ * 2 * 4 >= 4294967295.0) return false;
    if (!(p.tau[0] > 0.5) || !(p.tau[1] > 0.5) || !(p.tau_d > 0.5)) return false;
    if (!std::isfinite(p.tau[0]) || !std::isfinite(p.tau[1]) || !std::isfinite(p.tau_d)) return false;
    if (!(p.kT >= 0.0) || !std::isfinite(p.kT) || !std::isfinite(p.G)) return false;
    if (!std::isfinite(p.rho_ref[0]) || !std::isfinite(p.rho_ref[1])) return false;
    return true;
}

struct BatchLayout {
    size_t reps, items, step, stage, partial, modeacc, misc, total;
    size_t max_items, max_sites;
};

BatchLayout batch_layout(const fmlb_params *p, int n)
{
    BatchLayout l{};
    size_t items = 0, max_sites = 0;
    for (int r = 0; r < n; ++r) {
        items += (size_t)((p[r].nx + kMinTile - 1) / kMinTile) * (size_t)p[r].ny;  // chunk 1 is the worst case
        max_sites = std::max(max_sites, (size_t)p[r].nx * p[r].ny);
    }
    size_t o = 0;
    l.reps = o;
    o += align256((size_t)n * sizeof(BatchRep));
    l.items = o;
    o += align256(items * sizeof(BatchItem));
    l.step = o;
    o += 256;
    l.stage = o;
    o += align256(2 * max_sites * sizeof(double));
    l.partial = o;
    o += align256((size_t)kBatchReduceBlocks * 4 * kQ * sizeof(double));
    l.modeacc = o;
    o += align256((size_t)n * 4 * kQ * sizeof(double));
    l.misc = o;
    o += align256(64 * sizeof(double));
    l.total = o;
    l.max_items = items;
    l.max_sites = max_sites;
    return l;
}

Phys<float> replica_phys(const fmlb_params &p)
{
    Phys<float> ph{};
    const double lam0 = 1.0 / p.tau[0], lam1 = 1.0 / p.tau[1], lam_d = 1.0 / p.tau_d;
    const double mu = 3.0 * p.kT;
    const bool noisy = (p.kT > 0.0) && !(p.flags & FMLB_NOISE_OFF);
    const bool sdf = noisy && !(p.flags & FMLB_NOISE_NO_SDF);
    ph.lam[0] = (float)lam0;
    ph.lam[1] = (float)lam1;
    ph.lam_d = (float)lam_d;
    ph.negG = (float)(-p.G);
    ph.gain[0] = noisy ? (float)std::sqrt((2.0 * lam0 - lam0 * lam0) * mu) : 0.f;
    ph.gain[1] = noisy ? (float)std::sqrt((2.0 * lam1 - lam1 * lam1) * mu) : 0.f;
    ph.sd_gain = sdf ? (float)std::sqrt((2.0 * lam_d - lam_d * lam_d) * p.kT) : 0.f;
    ph.key0 = (uint32_t)p.seed;
    ph.key1 = (uint32_t)(p.seed >> 32);
    return ph;
}

template <int T0>
__global__ __launch_bounds__(T0) void batch_step_kernel(float *bufA, float *bufB, const BatchRep *reps,
                                                        const BatchItem *items, unsigned nitems,
                                                        const int64_t *step_dev, int offset, int chunk)
{
    const BatchItem it = items[xcd_contiguous(blockIdx.x, nitems)];
    const BatchRep &R = reps[it.rep];
    const int64_t step = *step_dev + offset;
    const bool odd = (step & 1) != 0;
    StepArgs<D2Q9, float> a{};
    a.src = (odd ? bufB : bufA) + R.off;
    a.dst = (odd ? bufA : bufB) + R.off;
    a.rho = nullptr;
    a.g = R.g;
    a.ph = R.ph;
    a.ref[0] = R.ref[0];
    a.ref[1] = R.ref[1];
    a.step_lo = (uint32_t)(uint64_t)step;
    a.step_hi = (uint32_t)((uint64_t)step >> 32);
    const int t0 = (int)(it.tile_chunk >> 16), ck = (int)(it.tile_chunk & 0xffffu);
    const int mbeg = ck * chunk;
    const int mend = min(mbeg + chunk, R.g.ny);
    if constexpr (FMLB_FUSED_ASYNC)
        fused_tile_async<D2Q9, float, T0, 1>(a, t0, 0, mbeg, mend);
    else
        fused_tile<D2Q9, float, T0, 1>(a, t0, 0, mbeg, mend);
}

// Packed sites: one workgroup of T threads walks a contiguous run of a
// replica's sites in row-major order, T sites per block (thread t: logical
// site l0 + k T + t of block k), so replicas of any width below T fill the
// lanes that one-row tiles leave idle (a 256-wide tile on a width-40
// replica runs 40 of its 256 lanes; here only a replica's last block is
// partly idle).  Logical sites count on past the lattice's end: site l is
// (l mod L, (l div L) mod ny), which is the periodic image in y, and a
// neighbour's logical index is l + c_y L + c_x (+-L where x wraps), at most
// 2L - 1 sites away (a row end's neighbour across the wrap in the next or
// previous row).  The asynchronous tile walk of the single lattice
// otherwise: block k+1's populations go straight from memory into LDS
// while block k collides; the densities enter a ring of four blocks
// indexed by (l - l0 + T) mod 4T, so with 2L - 1 <= T every neighbour of
// block k is in blocks k-1, k or k+1.  A thread stores only sites of its
// item.  Same
// helpers as the single lattice (moments, lattice_acceleration,
// collide_site): every replica evolves bit for bit as it would alone.
template <int T>
__device__ __forceinline__ void batch_pack_walk(const StepArgs<D2Q9, float> &a, long l0, long l1)
{
    using Lt = D2Q9;
    using Real = float;
    using Raw = uint32_t;
    constexpr int Q = Lt::Q;
    constexpr int RING = 4 * T;
    __shared__ Real ring[2][RING];
    __shared__ Raw own[2 * Q][T];

    const int L = a.g.nx, ny = a.g.ny;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const long nblk = (l1 - l0 + T - 1) / T;
    const uint32_t pop_bytes = (uint32_t)a.g.pitch * 4u;
    __amdgpu_buffer_rsrc_t rsrc[2], rdst[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rsrc[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.src + (size_t)s * Q * a.g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
        rdst[s] = __builtin_amdgcn_make_buffer_rsrc((void *)(a.dst + (size_t)s * Q * a.g.pitch), 0,
                                                    (int)(Q * pop_bytes), kBufferWord3);
    }
    const Real ref[2] = {a.ref[0], a.ref[1]};
    // (x, y) of logical site l, and the same T sites further on
    const long span = (long)L * ny;
    auto coords = [&](long l, int &x, int &y) {
        const long m = ((l % span) + span) % span;
        y = (int)(m / L);
        x = (int)(m - (long)y * L);
    };
    const int dxb = T % L, dyb = T / L;
    auto advance = [&](int x, int y, int &x2, int &y2) {
        x2 = x + dxb;
        y2 = y + dyb;
        if (x2 >= L) {
            x2 -= L;
            y2 += 1;
        }
        y2 = (int)((unsigned)y2 % (unsigned)ny);
    };
    auto pull_off = [&](int x, int y, int i) __attribute__((always_inline)) -> uint32_t {
        const int xs = wrap(x, -Lt::cx[i], L);
        const int ys = wrap(y, -Lt::cy[i], ny);
        return ((uint32_t)xs + (uint32_t)L * (uint32_t)ys) * 4u;
    };
    auto pull = [&](int x, int y, Real (&f)[2][Q]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const uint32_t voff = pull_off(x, y, i);
#pragma unroll
            for (int s = 0; s < 2; ++s) f[s][i] = BufIO<float>::load(rsrc[s], voff, (uint32_t)i * pop_bytes);
        }
    };
    auto dma = [&](int s, int x, int y) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            lds_void_t *dst = (lds_void_t *)(&own[s * Q + i][0] + wave * 64);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc[s], dst, 4, pull_off(x, y, i), (uint32_t)i * pop_bytes, 0, 0);
        }
    };
    // ring position of block k's thread-t site
    auto rpos = [&](long k) { return (int)(((k + 1) * T + tid) & (RING - 1)); };

    Real cur[2][Q], rc[2], jc[2][3];
    // Prologue: densities of blocks -1 and 0, populations and moments of
    // block 0 (register pulls), then the asynchronous pull of block 1.
#pragma unroll 1
    for (int k = -1; k <= 0; ++k) {
        int x, y;
        coords(l0 + (long)k * T + tid, x, y);
        Real f[2][Q];
        pull(x, y, f);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Real r, j[3];
            moments<Lt, Real>(f[s], r, j);
            ring[s][rpos(k)] = r;
            if (k == 0) {
                rc[s] = r;
#pragma unroll
                for (int al = 0; al < 3; ++al) jc[s][al] = j[al];
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[s][i] = f[s][i];
            }
        }
    }
    int xc, yc, xn, yn;  // this thread's site in block k and block k+1
    coords(l0 + tid, xc, yc);
    advance(xc, yc, xn, yn);
    dma(0, xn, yn);
    dma(1, xn, yn);

#pragma unroll 1
    for (long k = 0; k < nblk; ++k) {
        // Block k+1 has landed.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        Real nxt[2][Q], rn[2], jn[2][3];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) nxt[s][i] = __builtin_bit_cast(float, own[s * Q + i][tid]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            moments<Lt, Real>(nxt[s], rn[s], jn[s]);
            ring[s][rpos(k + 1)] = rn[s];
        }
        // Workgroup barrier for the density ring only.
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);

        // Ring positions of the neighbours: logical offset c_y L + c_x, with
        // +-L where x wraps.
        const int me = rpos(k);
        auto nb = [&](int i, int s) -> Real {
            const int cx = Lt::cx[i], cy = Lt::cy[i];
            const int dx = cx == 0 ? 0 : (cx > 0 ? (xc == L - 1 ? 1 - L : 1) : (xc == 0 ? L - 1 : -1));
            return ring[s][(me + cy * L + dx) & (RING - 1)];
        };
        Real acc[2][3];
        lattice_acceleration<Lt, Real>(nb, a.ph.negG, acc);
        // Every LDS read of this iteration is done: the loads of block k+2.
        const bool more = k + 1 < nblk;
        int x2, y2;
        advance(xn, yn, x2, y2);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_sched_barrier(0);
        if (more) dma(0, x2, y2);
        __builtin_amdgcn_sched_barrier(0);
        const bool store = l0 + k * T + tid < l1;
        const uint32_t site = (uint32_t)xc + (uint32_t)L * (uint32_t)yc;
        const uint32_t voff = site * 4u;
        collide_site<Lt, Real>(cur, rc, jc, acc, a.ph, ref, Counter{site, a.step_lo, a.step_hi}, [&](int s, auto &fs) {
            if (s == 0) {
                __builtin_amdgcn_sched_barrier(0);
                if (more) dma(1, x2, y2);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (store) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    store_stepped<float>(fs[i], rdst[s], voff, (uint32_t)i * pop_bytes, site, (uint32_t)(s * Q + i),
                                         a.step_lo, a.ph.key0, a.ph.key1);
            }
        });
        xc = xn;
        yc = yn;
        xn = x2;
        yn = y2;
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

// Packed-site items: tile_chunk holds the item's index among its replica's
// items, each `chunk` blocks of T sites.
template <int T>
__global__ __launch_bounds__(T) void batch_pack_kernel(float *bufA, float *bufB, const BatchRep *reps,
                                                       const BatchItem *items, unsigned nitems,
                                                       const int64_t *step_dev, int offset, int chunk)
{
    const BatchItem it = items[xcd_contiguous(blockIdx.x, nitems)];
    const BatchRep &R = reps[it.rep];
    const int64_t step = *step_dev + offset;
    const bool odd = (step & 1) != 0;
    StepArgs<D2Q9, float> a{};
    a.src = (odd ? bufB : bufA) + R.off;
    a.dst = (odd ? bufA : bufB) + R.off;
    a.rho = nullptr;
    a.g = R.g;
    a.ph = R.ph;
    a.ref[0] = R.ref[0];
    a.ref[1] = R.ref[1];
    a.step_lo = (uint32_t)(uint64_t)step;
    a.step_hi = (uint32_t)((uint64_t)step >> 32);
    const long len = (long)T * chunk;
    const long l0 = (long)it.tile_chunk * len;
    batch_pack_walk<T>(a, l0, min(l0 + len, (long)R.g.nsites));
}

// Advances the device step counter (one lane, vector store).
__global__ void batch_advance_kernel(int64_t *step_dev, int n)
{
    if (threadIdx.x == 0) step_dev[threadIdx.x] += n;
}

// Sets the device step counter.
__global__ void batch_set_step_kernel(int64_t *step_dev, int64_t v)
{
    if (threadIdx.x == 0) step_dev[threadIdx.x] = v;
}

}  // namespace

struct fmlb_batch {
    std::vector<fmlb_params> p;
    std::vector<BatchRep> reps;
    std::vector<char> ready;
    int n;
    hipStream_t stream;
    float *buf[2];
    unsigned char *scratch;
    BatchLayout lay;
    int64_t step;
    int tile_x, chunk;  // tile_x FMLB_BATCH_PACKED(_512): packed sites, else one-row tiles
    unsigned nitems;
    unsigned npack;     // packed-site items, at the front of the work list
    hipGraphExec_t gexec;
    hipStream_t cap_stream;
    int64_t mode_samples;
};

namespace {

template <class T>
T *bscr(fmlb_batch *b, size_t off)
{
    return reinterpret_cast<T *>(b->scratch + off);
}

constexpr int kPackedTile = FMLB_BATCH_PACKED;         // packed sites, 256 threads
constexpr int kPackedTile512 = FMLB_BATCH_PACKED_512;  // packed sites, 512 threads

bool batch_tile_valid(int tx)
{
    return tx == kPackedTile || tx == kPackedTile512 || tx == 64 || tx == 128 || tx == 256;
}

int pack_threads(int tx) { return tx == kPackedTile512 ? 512 : 256; }

// Widest replica packed in blocks of T sites (a neighbour within one block).
constexpr int pack_max_width(int T) { return (T + 1) / 2; }

// Packed-site items of replica p for `chunk` blocks of T sites per item (0:
// too wide to pack).
long pack_items(const fmlb_params &p, int T, int chunk)
{
    if (p.nx > pack_max_width(T)) return 0;
    const long len = (long)T * chunk;
    return ((long)p.nx * p.ny + len - 1) / len;
}

// Default: packed sites in blocks of 512, with the longest march (blocks per
// item, up to 16) that still leaves about 2048 items (eight per CU).
void batch_default_shape(const fmlb_batch *b, int &tx, int &chunk)
{
    tx = kPackedTile512;
    chunk = 1;
    for (;;) {
        long items = 0;
        for (const auto &p : b->p)
            items += p.nx > pack_max_width(512) ? (long)((p.nx + 255) / 256) * ((p.ny + 2L * chunk - 1) / (2L * chunk))
                                                 : pack_items(p, 512, 2 * chunk);
        if (chunk >= 16 || items < 2048) break;
        chunk *= 2;
    }
}

// The work list: packed tx puts the packed-site items of every replica up to
// pack_max_width(T) wide first (the item's index among its replica's items),
// then one-row 256-wide tiles of `chunk` rows for wider replicas; other tx:
// one-row tiles of tx sites and `chunk` rows for every replica.
fmlb_status build_items(fmlb_batch *b, int tx, int chunk)
{
    std::vector<BatchItem> items;
    unsigned npack = 0;
    const bool packed = tx == kPackedTile || tx == kPackedTile512;
    const int T = pack_threads(tx);
    if (packed) {
        for (int r = 0; r < b->n; ++r)
            for (long i = 0; i < pack_items(b->p[r], T, chunk); ++i) items.push_back(BatchItem{(uint32_t)r, (uint32_t)i});
        npack = (unsigned)items.size();
    }
    const int wt = packed ? 256 : tx;
    for (int r = 0; r < b->n; ++r) {
        if (packed && b->p[r].nx <= pack_max_width(T)) continue;
        const int tiles = (b->p[r].nx + wt - 1) / wt, chunks = (b->p[r].ny + chunk - 1) / chunk;
        for (int ck = 0; ck < chunks; ++ck)
            for (int t = 0; t < tiles; ++t) items.push_back(BatchItem{(uint32_t)r, ((uint32_t)t << 16) | (uint32_t)ck});
    }
    if (items.size() > b->lay.max_items || items.empty()) return FMLB_E_INVALID;
    b->npack = npack;
    BATCH_TRY(hipMemcpyAsync(bscr<BatchItem>(b, b->lay.items), items.data(), items.size() * sizeof(BatchItem),
                             hipMemcpyHostToDevice, b->stream));
    BATCH_TRY(hipStreamSynchronize(b->stream));
    b->nitems = (unsigned)items.size();
    b->tile_x = tx;
    b->chunk = chunk;
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return FMLB_OK;
}

fmlb_status launch_batch_step(fmlb_batch *b, int offset, hipStream_t stream)
{
    const int64_t *sd = bscr<int64_t>(b, b->lay.step);
    const BatchRep *reps = bscr<BatchRep>(b, b->lay.reps);
    const BatchItem *items = bscr<BatchItem>(b, b->lay.items);
    switch (b->tile_x) {
    case kPackedTile:
    case kPackedTile512:
        if (b->npack > 0 && b->tile_x == kPackedTile)
            hipLaunchKernelGGL(batch_pack_kernel<256>, dim3(b->npack), dim3(256), 0, stream, b->buf[0], b->buf[1], reps,
                               items, b->npack, sd, offset, b->chunk);
        if (b->npack > 0 && b->tile_x == kPackedTile512)
            hipLaunchKernelGGL(batch_pack_kernel<512>, dim3(b->npack), dim3(512), 0, stream, b->buf[0], b->buf[1], reps,
                               items, b->npack, sd, offset, b->chunk);
        if (b->nitems > b->npack)
            hipLaunchKernelGGL(batch_step_kernel<256>, dim3(b->nitems - b->npack), dim3(256), 0, stream, b->buf[0],
                               b->buf[1], reps, items + b->npack, b->nitems - b->npack, sd, offset, b->chunk);
        break;
    case 64:
        hipLaunchKernelGGL(batch_step_kernel<64>, dim3(b->nitems), dim3(64), 0, stream, b->buf[0], b->buf[1],
                           reps, items, b->nitems, sd, offset, b->chunk);
        break;
    case 128:
        hipLaunchKernelGGL(batch_step_kernel<128>, dim3(b->nitems), dim3(128), 0, stream, b->buf[0], b->buf[1],
                           reps, items, b->nitems, sd, offset, b->chunk);
        break;
    case 256:
        hipLaunchKernelGGL(batch_step_kernel<256>, dim3(b->nitems), dim3(256), 0, stream, b->buf[0], b->buf[1],
                           reps, items, b->nitems, sd, offset, b->chunk);
        break;
    default: return FMLB_E_INVALID;
    }
    BATCH_TRY(hipGetLastError());
    return FMLB_OK;
}

fmlb_status launch_steps(fmlb_batch *b, int n, hipStream_t stream)
{
    for (int t = 0; t < n; ++t)
        if (fmlb_status st = launch_batch_step(b, t, stream)) return st;
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, stream, bscr<int64_t>(b, b->lay.step), n);
    BATCH_TRY(hipGetLastError());
    return FMLB_OK;
}

// The graph is recorded on a private stream (capture is not allowed on the
// legacy default stream) and replayed on the batch's stream.
fmlb_status capture_graph(fmlb_batch *b)
{
    if (!b->cap_stream) BATCH_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    BATCH_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const fmlb_status st = launch_steps(b, kGraphSteps, b->cap_stream);
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    BATCH_TRY(e);
    const hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BATCH_TRY(ei);
    return FMLB_OK;
}

float *replica_src(fmlb_batch *b, int r) { return b->buf[b->step & 1] + b->reps[r].off; }

SiteGrid2 replica_grid(const Geom &g)
{
    return SiteGrid2{dim3((g.nx + 63) / 64, g.ny, 1), dim3(64)};
}

}  // namespace

extern "C" {

size_t fmlb_batch_required_bytes(const fmlb_params *p, int n, int which)
{
    if (!p || n < 1 || n > 65535) return 0;
    size_t pops = 0;
    for (int r = 0; r < n; ++r) {
        if (!valid_replica(p[r])) return 0;
        pops += align256(2 * (size_t)kQ * replica_pitch(p[r]) * sizeof(float));
    }
    switch (which) {
    case FMLB_BUF_POPS_A:
    case FMLB_BUF_POPS_B: return pops;
    case FMLB_BUF_SCRATCH: return batch_layout(p, n).total;
    }
    return 0;
}

fmlb_status fmlb_batch_create(const fmlb_params *p, int n, void *hip_stream, void *const dev_buf[3],
                              fmlb_batch **out)
{
    if (!p || !dev_buf || !out) return FMLB_E_NULL;
    *out = nullptr;
    if (!dev_buf[0] || !dev_buf[1] || !dev_buf[2]) return FMLB_E_NULL;
    if (n < 1 || n > 65535) return FMLB_E_INVALID;
    for (int r = 0; r < n; ++r)
        if (!valid_replica(p[r])) return FMLB_E_INVALID;
    for (int k = 0; k < 3; ++k)
        if (reinterpret_cast<uintptr_t>(dev_buf[k]) % 256 != 0) return FMLB_E_INVALID;
    fmlb_batch *b = new (std::nothrow) fmlb_batch();
    if (!b) return FMLB_E_INVALID;
    b->p.assign(p, p + n);
    b->n = n;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->buf[0] = reinterpret_cast<float *>(dev_buf[0]);
    b->buf[1] = reinterpret_cast<float *>(dev_buf[1]);
    b->scratch = reinterpret_cast<unsigned char *>(dev_buf[2]);
    b->lay = batch_layout(p, n);
    b->step = 0;
    b->gexec = nullptr;
    b->cap_stream = nullptr;
    b->mode_samples = 0;
    b->ready.assign(n, 0);
    uint64_t off = 0;
    for (int r = 0; r < n; ++r) {
        BatchRep R{};
        R.off = off;
        R.g = Geom{p[r].nx, p[r].ny, 1, (size_t)p[r].nx * p[r].ny, replica_pitch(p[r])};
        R.ph = replica_phys(p[r]);
        R.ref[0] = (float)p[r].rho_ref[0];
        R.ref[1] = (float)p[r].rho_ref[1];
        b->reps.push_back(R);
        off += align256(2 * (size_t)kQ * R.g.pitch * sizeof(float)) / sizeof(float);
    }
    fmlb_status st = FMLB_OK;
    auto fail = [&](fmlb_status s) {
        delete b;
        return s;
    };
    if (hipMemcpyAsync(bscr<BatchRep>(b, b->lay.reps), b->reps.data(), n * sizeof(BatchRep), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return fail(FMLB_E_HIP);
    hipLaunchKernelGGL(batch_set_step_kernel, dim3(1), dim3(64), 0, b->stream, bscr<int64_t>(b, b->lay.step),
                       (int64_t)0);
    if (hipGetLastError() != hipSuccess) return fail(FMLB_E_HIP);
    int tx, chunk;
    batch_default_shape(b, tx, chunk);
    if ((st = build_items(b, tx, chunk))) return fail(st);
    if ((st = fmlb_batch_reset_modes(b))) return fail(st);
    *out = b;
    return FMLB_OK;
}

void fmlb_batch_destroy(fmlb_batch *b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

int fmlb_batch_size(const fmlb_batch *b) { return b ? b->n : -1; }

int64_t fmlb_batch_total_sites(const fmlb_batch *b)
{
    if (!b) return -1;
    int64_t t = 0;
    for (const auto &R : b->reps) t += (int64_t)R.g.nsites;
    return t;
}

int64_t fmlb_batch_current_step(const fmlb_batch *b) { return b ? b->step : -1; }

fmlb_status fmlb_batch_init_density(fmlb_batch *b, int r, const double *rho1, const double *rho2)
{
    if (!b || !rho1 || !rho2) return FMLB_E_NULL;
    if (r < 0 || r >= b->n) return FMLB_E_INVALID;
    const Geom g = b->reps[r].g;
    double *stage = bscr<double>(b, b->lay.stage);
    BATCH_TRY(hipMemcpyAsync(stage, rho1, g.nsites * sizeof(double), hipMemcpyHostToDevice, b->stream));
    BATCH_TRY(hipMemcpyAsync(stage + g.nsites, rho2, g.nsites * sizeof(double), hipMemcpyHostToDevice, b->stream));
    const SiteGrid2 sg = replica_grid(g);
    hipLaunchKernelGGL((init_kernel<D2Q9, float>), sg.grid, sg.block, 0, b->stream, replica_src(b, r),
                       (const double *)stage, g, b->reps[r].ref[0], b->reps[r].ref[1]);
    BATCH_TRY(hipGetLastError());
    BATCH_TRY(hipStreamSynchronize(b->stream));  // the stage is reused by the next call
    b->ready[r] = 1;
    return FMLB_OK;
}

fmlb_status fmlb_batch_step(fmlb_batch *b, int64_t n, int use_graph)
{
    if (!b) return FMLB_E_NULL;
    if (n < 0) return FMLB_E_INVALID;
    for (char rd : b->ready)
        if (!rd) return FMLB_E_STATE;
    int64_t left = n;
    if (use_graph && n >= kGraphSteps) {
        if (!b->gexec)
            if (fmlb_status st = capture_graph(b)) return st;
        for (; left >= kGraphSteps; left -= kGraphSteps) BATCH_TRY(hipGraphLaunch(b->gexec, b->stream));
    }
    while (left > 0) {
        const int k = (int)std::min<int64_t>(left, 1 << 20);
        if (fmlb_status st = launch_steps(b, k, b->stream)) return st;
        left -= k;
    }
    b->step += n;
    return FMLB_OK;
}

fmlb_status fmlb_batch_set_tile(fmlb_batch *b, int tile_x, int chunk)
{
    if (!b) return FMLB_E_NULL;
    int dtx, dch;
    batch_default_shape(b, dtx, dch);
    const int tx = tile_x == 0 ? dtx : tile_x, ch = chunk == 0 ? dch : chunk;
    if (!batch_tile_valid(tx) || ch < 1 || ch > 4096) return FMLB_E_INVALID;
    return build_items(b, tx, ch);
}

fmlb_status fmlb_batch_autotune(fmlb_batch *b, int reps, int *tile_x, int *march)
{
    if (!b) return FMLB_E_NULL;
    if (reps < 1 || reps > 1000) return FMLB_E_INVALID;
    for (char rd : b->ready)
        if (!rd) return FMLB_E_STATE;
    static const int kTiles[] = {kPackedTile, kPackedTile512, 64, 128, 256};
    static const int kMarch[] = {1, 2, 4, 8, 16, 32, 64};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BATCH_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FMLB_E_HIP;
    }
    float best = 1e30f;
    int btx = b->tile_x, bch = b->chunk;
    fmlb_status st = FMLB_OK;
    for (int tx : kTiles) {
        for (int ch : kMarch) {
            if ((st = build_items(b, tx, ch))) break;
            // Step n -> n+1 recomputed `reps` times: the state of step n is
            // only read, the counter is not advanced, so the run is invisible.
            for (int w = 0; w < 2 && !st; ++w) st = launch_batch_step(b, 0, b->stream);
            if (!st && hipEventRecord(e0, b->stream) != hipSuccess) st = FMLB_E_HIP;
            for (int k = 0; k < reps && !st; ++k) st = launch_batch_step(b, 0, b->stream);
            if (!st && hipEventRecord(e1, b->stream) != hipSuccess) st = FMLB_E_HIP;
            if (!st && hipEventSynchronize(e1) != hipSuccess) st = FMLB_E_HIP;
            float ms = 0;
            if (!st && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = FMLB_E_HIP;
            if (st) break;
            if (ms < best) {
                best = ms;
                btx = tx;
                bch = ch;
            }
        }
        if (st) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if ((st = build_items(b, btx, bch))) return st;
    if (tile_x) *tile_x = btx;
    if (march) *march = bch;
    return FMLB_OK;
}

fmlb_status fmlb_batch_get_populations(fmlb_batch *b, int r, double *host, size_t bytes)
{
    if (!b || !host) return FMLB_E_NULL;
    if (r < 0 || r >= b->n) return FMLB_E_INVALID;
    if (!b->ready[r]) return FMLB_E_STATE;
    const Geom g = b->reps[r].g;
    if (bytes < 2 * (size_t)kQ * g.nsites * sizeof(double)) return FMLB_E_SIZE;
    double *stage = bscr<double>(b, b->lay.stage);
    const SiteGrid2 sg = replica_grid(g);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < kQ; ++i) {
            hipLaunchKernelGGL((gather_pop_kernel<D2Q9, float>), sg.grid, sg.block, 0, b->stream,
                               (const float *)replica_src(b, r), stage, g, s, i, b->reps[r].ref[s]);
            BATCH_TRY(hipGetLastError());
            BATCH_TRY(hipMemcpyAsync(host + ((size_t)s * kQ + i) * g.nsites, stage, g.nsites * sizeof(double),
                                     hipMemcpyDeviceToHost, b->stream));
            BATCH_TRY(hipStreamSynchronize(b->stream));
        }
    return FMLB_OK;
}

fmlb_status fmlb_batch_global_sums(fmlb_batch *b, int r, double *out)
{
    if (!b || !out) return FMLB_E_NULL;
    if (r < 0 || r >= b->n) return FMLB_E_INVALID;
    if (!b->ready[r]) return FMLB_E_STATE;
    const Geom g = b->reps[r].g;
    double *partial = bscr<double>(b, b->lay.partial);
    double *misc = bscr<double>(b, b->lay.misc);
    const int nb = (int)std::min<size_t>((g.nsites + kRedBlock - 1) / kRedBlock, kBatchReduceBlocks);
    hipLaunchKernelGGL((sums_kernel<D2Q9, float>), dim3(nb), dim3(kRedBlock), 0, b->stream,
                       (const float *)replica_src(b, r), partial, g, b->reps[r].ref[0], b->reps[r].ref[1]);
    BATCH_TRY(hipGetLastError());
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedBlock), 0, b->stream, (const double *)partial, nb, 4, misc,
                       (double *)nullptr);
    BATCH_TRY(hipGetLastError());
    BATCH_TRY(hipMemcpyAsync(out, misc, 4 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    BATCH_TRY(hipStreamSynchronize(b->stream));
    return FMLB_OK;
}

fmlb_status fmlb_batch_reset_modes(fmlb_batch *b)
{
    if (!b) return FMLB_E_NULL;
    const size_t nv = (size_t)b->n * 4 * kQ;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, b->stream,
                       bscr<double>(b, b->lay.modeacc), nv, 0.0);
    BATCH_TRY(hipGetLastError());
    b->mode_samples = 0;
    return FMLB_OK;
}

fmlb_status fmlb_batch_mode_accumulate(fmlb_batch *b)
{
    if (!b) return FMLB_E_NULL;
    for (char rd : b->ready)
        if (!rd) return FMLB_E_STATE;
    double *partial = bscr<double>(b, b->lay.partial);
    for (int r = 0; r < b->n; ++r) {
        const Geom g = b->reps[r].g;
        const int nb = (int)std::min<size_t>((g.nsites + kRedBlock - 1) / kRedBlock, kBatchReduceBlocks);
        hipLaunchKernelGGL((mode_stats_kernel<D2Q9, float>), dim3(nb), dim3(kRedBlock), 0, b->stream,
                           (const float *)replica_src(b, r), partial, g, b->reps[r].ref[0], b->reps[r].ref[1]);
        BATCH_TRY(hipGetLastError());
        hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedBlock), 0, b->stream, (const double *)partial, nb,
                           4 * kQ, (double *)nullptr, bscr<double>(b, b->lay.modeacc) + (size_t)r * 4 * kQ);
        BATCH_TRY(hipGetLastError());
    }
    b->mode_samples += 1;
    return FMLB_OK;
}

fmlb_status fmlb_batch_mode_variances(fmlb_batch *b, int r, double *out, int64_t *n_samples)
{
    if (!b || !out) return FMLB_E_NULL;
    if (r < 0 || r >= b->n) return FMLB_E_INVALID;
    if (!(b->p[r].kT > 0.0)) return FMLB_E_INVALID;  // the ratio is defined for k_B T > 0
    if (b->mode_samples == 0) return FMLB_E_STATE;
    double acc[4 * kQ];
    BATCH_TRY(hipMemcpyAsync(acc, bscr<double>(b, b->lay.modeacc) + (size_t)r * 4 * kQ, sizeof(acc),
                             hipMemcpyDeviceToHost, b->stream));
    BATCH_TRY(hipStreamSynchronize(b->stream));
    const fmlb_params &p = b->p[r];
    const double cnt = (double)b->mode_samples * (double)b->reps[r].g.nsites;
    const double mu = 3.0 * p.kT;
    for (int s = 0; s < 2; ++s) {
        const double rho_mean = acc[(s * kQ) * 2] / cnt;  // mean of mode 0 (m_0 = rho)
        for (int a = 0; a < kQ; ++a) {
            const double m1 = acc[(s * kQ + a) * 2] / cnt;
            const double m2 = acc[(s * kQ + a) * 2 + 1] / cnt;
            const double N = (double)D2Q9::Nnum[a] / D2Q9::Nden[a];
            out[s * kQ + a] = rho_mean > 0.0 ? (m2 - m1 * m1) / (N * mu * rho_mean) : NAN;
        }
    }
    if (n_samples) *n_samples = b->mode_samples;
    return FMLB_OK;
}

}  // extern "C"
