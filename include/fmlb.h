/*
 * fmlb — fluctuating multicomponent lattice Boltzmann on MI355X (gfx950).
 *
 * C ABI of the hot path of the two-species fluctuating lattice Boltzmann
 * equation (FLBE) of Belardinelli, Sbragaglia, Biferale, Gross and Varnik,
 * "Fluctuating multicomponent lattice Boltzmann model" (arXiv:1410.5584):
 * one fused stream + collide + noise + mean-field-force step per call site,
 * on D2Q9 or D3Q19, plus the observables the paper checks it with.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns fmlb_status: 0 on success, a negative code on
 *    error.  No function aborts or throws; on error nothing is launched and
 *    the context is unchanged unless stated.  fmlb_status_string() names a code.
 *  - Device memory is owned by the caller (e.g. PyTorch).  The library
 *    borrows the buffers passed to fmlb_create(), never frees them, and
 *    allocates no device memory itself, on the step path or elsewhere.
 *  - Host pointers are owned by the caller and only read / written during the
 *    call.
 *  - One context drives one HIP stream (passed as a hipStream_t cast to
 *    void*; NULL = the legacy default stream).  Launches are asynchronous on
 *    that stream unless a function is documented as synchronising.  A context
 *    is not thread-safe.
 *  - Lattice sites are indexed s = x + nx * (y + ny * z), x fastest; D2Q9
 *    lattices have nz = 1.  Periodic boundaries in every direction.
 *  - Velocity order.  D2Q9: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *    (-1,-1) (1,-1).  D3Q19: (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0)
 *    (0,0,1) (0,0,-1) (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *    (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
 *  - Mode order (used by fmlb_mode_variances).  D2Q9: Table I of the paper
 *    (rho, j_x, j_y, e, P_ww, P_xy, q_x, q_y, epsilon).  D3Q19: the Hermite
 *    modes of Eq. (26) (1, c_x, c_y, c_z, c_x^2-1/3, c_y^2-1/3, c_z^2-1/3,
 *    c_x c_y, c_y c_z, c_x c_z) followed by the ghosts (3|c|^2-5) c_alpha,
 *    (c_y^2-c_z^2) c_x, (c_z^2-c_x^2) c_y, (c_x^2-c_y^2) c_z,
 *    (2|c|^2-3)(3c_x^2-|c|^2), (2|c|^2-3)(c_y^2-c_z^2), 3|c|^4-6|c|^2+1.
 *  - Every observable refers to the pre-collision populations f_bar(r, n)
 *    after n completed steps (Sec. V A, Eq. (63): the stored variables of
 *    the scheme); the barycentric velocity is the physical one,
 *    v_b_bar + a_b / 2 (Eq. (70)).
 *  - Thermal noise uses the counter-based generator Philox4x32-10 (Salmon et
 *    al., SC'11) keyed by the 64-bit seed, with counter (site, step mod 2^32,
 *    block, step / 2^32); the four words of block j are words 4j..4j+3 of
 *    the site's stream, and word w gives the normals 2w, 2w+1 by
 *    trigonometric Box-Muller from the uniforms u = (2U + 1) / 2^17 of its
 *    high (radius) and low (angle) 16 bits.  Normal k of a site feeds: k < D
 *    the momentum noise (+ for species 1, - for species 2, Eq. (74)); then
 *    the non-momentum modes a = D+1..Q-1 of species 1, then of species 2.
 *    Results therefore depend only on (seed, site, step), never on launch
 *    shape or on how many steps one call advances.
 */
#ifndef FMLB_H
#define FMLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fmlb_status;

enum {
    FMLB_OK = 0,
    FMLB_E_INVALID = -1, /* a parameter is out of range (see fmlb_params)          */
    FMLB_E_SIZE = -2,    /* a buffer is too small                                   */
    FMLB_E_HIP = -3,     /* a HIP call failed; fmlb_last_hip_error() has the code   */
    FMLB_E_STATE = -4,   /* populations not initialised yet                         */
    FMLB_E_NULL = -5,    /* a required pointer is NULL                              */
    FMLB_E_UNSUPPORTED = -6 /* the combination is not built (e.g. S(k) on a huge lattice) */
};

typedef enum { FMLB_D2Q9 = 0, FMLB_D3Q19 = 1 } fmlb_lattice;

/* Storage of the populations in device memory.  The arithmetic is FP64 for
 * FMLB_F64 and FP32 for every other storage.  FP32 and the 16-bit forms
 * store the deviation f_i - w_i rho_ref (16-bit: rounded to nearest even),
 * and the FP32 step updates the deviations directly, so its rounding is
 * relative to the fluctuations rather than to w_i rho.  FP64 stores
 * absolute values. */
typedef enum {
    FMLB_F64 = 0,
    FMLB_F32 = 1,
    FMLB_BF16_DEV = 2,
    FMLB_F16_DEV = 3
} fmlb_storage;

enum {
    FMLB_NOISE_OFF = 1u,    /* deterministic lattice Boltzmann (no thermal noise)            */
    FMLB_NOISE_NO_SDF = 2u, /* no noise on the momentum modes ("no-sdf", Sec. VI A)          */
    /* 16-bit storage only (FMLB_E_INVALID otherwise): the steps round the stored
     * deviations stochastically instead of to nearest even.  The bits below the
     * kept ones get a uniform offset from an integer hash of (site, species x Q +
     * population, step), so each rounding is unbiased and the errors of
     * neighbouring sites are independent.  Round-to-nearest errs alike at all
     * sites of a domain of nearly equal deviations, which drifts the species
     * masses of a demixed lattice (D3Q19 256^3 at G = 1.2: 2.3e-4 of the total
     * over 5000 steps with BF16); stochastic rounding keeps the drift at the
     * level of independent errors.  Costs some ALU time in the 16-bit step.
     * Initial states and host writes still round to nearest. */
    FMLB_ROUND_STOCHASTIC = 4u
};

/* Parameters of one lattice (all in lattice units, k_B = 1). */
typedef struct fmlb_params {
    int32_t lattice;    /* fmlb_lattice                                                    */
    int32_t storage;    /* fmlb_storage                                                    */
    int32_t nx, ny, nz; /* >= 1 each; nz == 1 for D2Q9                                     */
    double tau[2];      /* lambda_bar_sigma = 1/tau_sigma for the transport and ghost modes
                           of species sigma (Table I, one value per species); tau > 1/2     */
    double tau_d;       /* lambda_bar_d = 1/tau_d for the momentum modes of both species
                           (Eq. (37): common, so total momentum is conserved); > 1/2       */
    double G;           /* coupling of the lattice force, Eq. (87) (G = G')               */
    double kT;          /* k_B T >= 0; mu = k_B T / c_s^2 with c_s^2 = 1/3 (Eq. (18))      */
    double rho_ref[2];  /* reference density per species for the FP32 / 16-bit deviation storage */
    uint64_t seed;      /* Philox key                                                      */
    uint32_t flags;     /* FMLB_NOISE_* and FMLB_ROUND_STOCHASTIC bits; others: FMLB_E_INVALID */
} fmlb_params;

typedef struct fmlb_ctx fmlb_ctx;

/* Buffer indices for fmlb_required_bytes / fmlb_create. */
enum { FMLB_BUF_POPS_A = 0, FMLB_BUF_POPS_B = 1, FMLB_BUF_SCRATCH = 2 };

/* Bytes the caller must provide for buffer `which` (FMLB_BUF_*), 0 if the
 * parameters are invalid.  POPS_A / POPS_B: 2 * Q * sites * element size
 * (the two population arrays of the pull scheme).  SCRATCH: densities,
 * FP64 staging for host transfers, FP64 structure-factor accumulators and
 * DFT workspace, reduction partials.  Each buffer must be 256-byte aligned. */
size_t fmlb_required_bytes(const fmlb_params *p, int which);

/* Validate `p` and bind the three caller-owned device buffers (FMLB_BUF_*
 * order) and the HIP stream.  Errors: FMLB_E_NULL, FMLB_E_INVALID (tau or
 * tau_d <= 1/2, kT < 0, a size < 1, D2Q9 with nz != 1, unknown lattice or
 * storage, more than 2^31 sites), FMLB_E_HIP.  The populations are
 * uninitialised until fmlb_init_density or fmlb_set_populations. */
fmlb_status fmlb_create(const fmlb_params *p, void *hip_stream, void *const dev_buf[3],
                        fmlb_ctx **out);

/* Free the context (not the caller's buffers).  NULL is a no-op. */
void fmlb_destroy(fmlb_ctx *ctx);

/* Rest state f_bar_i(r, 0) = w_i rho_sigma(r) from host densities
 * rho1[sites], rho2[sites] (FP64); sets the step counter to 0.  The uniform
 * rest state is the paper's initial condition (Sec. VI A).  Synchronises. */
fmlb_status fmlb_init_density(fmlb_ctx *ctx, const double *rho1, const double *rho2);

/* Advance n >= 0 steps of the FLBE update, Eq. (84): per site, pull the
 * populations streamed from r - c_i, compute rho, j_bar (Eq. (86)), the
 * lattice force of Eq. (87) from the neighbours' densities of the same step,
 * the collision R_a of Eq. (85) with the renormalised forcing of Eq. (72)
 * and the noise of Eq. (74) with the local densities (Sec. IV B), and write
 * the post-collision populations.  Asynchronous. */
fmlb_status fmlb_step(fmlb_ctx *ctx, int64_t n);

/* Number of completed steps. */
int64_t fmlb_current_step(const fmlb_ctx *ctx);

/* rho[2][sites] and j_bar[2][D][sites] (Eq. (86)) of the current state,
 * FP64, into host memory.  Either pointer may be NULL.  Synchronises. */
fmlb_status fmlb_moments(fmlb_ctx *ctx, double *rho, double *j);

/* FP64 global sums of the current state: out[0] = sum rho_1,
 * out[1] = sum rho_2, out[2 + alpha] = sum (j_bar_1 + j_bar_2)_alpha,
 * alpha < D (mass and total momentum, conserved by the update: R_0 = 0 and
 * opposite momentum noise, Sec. V A / Eq. (74)).  out has 2 + D entries.
 * Synchronises. */
fmlb_status fmlb_global_sums(fmlb_ctx *ctx, double *out);

/* Add the current state's mode statistics to the running sums: for every
 * species and mode a, sum over sites of m_a and m_a^2 (m_a = sum_i T_ai
 * f_bar_i, Eq. (80)), in FP64.  Asynchronous. */
fmlb_status fmlb_mode_accumulate(fmlb_ctx *ctx);

/* out[2][Q] = (<m_a^2> - <m_a>^2) / (N_a mu <rho_sigma>), the
 * equipartition ratio of Eq. (50) (1 in equilibrium), from the running sums;
 * <rho_sigma> is the sampled mean density (the mean of mode 0 over sites and
 * snapshots; NaN for a species whose mean density is not positive) and
 * n_samples the number of accumulated snapshots.  FMLB_E_INVALID when
 * k_B T = 0 (the ratio is undefined), FMLB_E_STATE before any accumulate.
 * Synchronises. */
fmlb_status fmlb_mode_variances(fmlb_ctx *ctx, double *out, int64_t *n_samples);

/* Structure factors (Sec. VI A): add |X_hat(k)|^2 / sites-type products of
 * the current state to FP64 accumulators, X_hat(k) = sum_r dX(r) e^{-i k.r},
 * dX = X - spatial mean, k = 2 pi n / L.  Accumulated quantities (index
 * `which` of fmlb_sk_get): 0 S_rho1rho1, 1 S_rho2rho2, 2 Re S_rho1rho2,
 * 3 S_j1j1, 4 S_j2j2, 5 Re S_j1j2 (j_bar, averaged over the D components),
 * 6 S_vbvb (physical barycentric velocity, averaged over components).
 * Asynchronous. */
fmlb_status fmlb_sk_accumulate(fmlb_ctx *ctx);

/* out[sites] (same k layout as the lattice, k_x fastest, FFT order) = the
 * mean of quantity `which` over the accumulated snapshots; n_samples may be
 * NULL.  FMLB_E_INVALID for an unknown `which`.  Synchronises. */
fmlb_status fmlb_sk_get(fmlb_ctx *ctx, int which, double *out, int64_t *n_samples);

/* For callers that cannot allocate device memory or call an allocator (code
 * under HIP graph capture, allocation-free serving loops): the accumulation
 * of fmlb_sk_accumulate without a context.  The work arrays (the FP64
 * moments of both species and one complex FP64 field: 80 bytes per site)
 * live in a static device array of the library, one per GPU, of
 * FMLB_SK_STATIC_MAX_SITES * 80 bytes (80 MiB), held until the process ends.
 *   p:    the lattice, storage and rho_ref of the state (validated as by
 *         fmlb_create).
 *   pops: device, the stored state as a context keeps it (pull layout,
 *         [2][Q][sites] values of p->storage; the bytes fmlb_save_raw returns).
 *   acc:  device, [7][sites] doubles owned and cleared by the caller; the
 *         seven quantities of fmlb_sk_accumulate (same order and k layout)
 *         are added to it, so acc / n_snapshots is what fmlb_sk_get returns.
 * Asynchronous on hip_stream.  FMLB_E_SIZE above FMLB_SK_STATIC_MAX_SITES
 * sites, FMLB_E_UNSUPPORTED for an axis longer than 2048.  Nothing is
 * allocated.  Calls that overlap on one GPU share the static array and race;
 * a call may start once the previous call on that GPU has completed (stream
 * order suffices). */
#define FMLB_SK_STATIC_MAX_SITES (1 << 20)
fmlb_status fmlb_sk_accumulate_static(const fmlb_params *p, const void *pops, double *acc, void *hip_stream);

/* Clear the structure-factor and mode accumulators.  Asynchronous. */
fmlb_status fmlb_reset_accumulators(fmlb_ctx *ctx);

/* Pre-collision populations f_bar[2][Q][sites] (FP64, absolute values) to /
 * from host memory: checkpoint and test I/O.  `bytes` must be at least
 * 16 * Q * sites.  set_populations also sets the step counter (the noise
 * of the next step uses counter `step`).  Synchronise. */
fmlb_status fmlb_get_populations(fmlb_ctx *ctx, double *host, size_t bytes);
fmlb_status fmlb_set_populations(fmlb_ctx *ctx, const double *host, size_t bytes, int64_t step);

/* Bit-exact checkpoint of the stored state in its device representation
 * (fmlb_required_bytes(p, FMLB_BUF_POPS_A) bytes: deviations from w_i rho_ref
 * for FP32 and 16-bit storage, so restore into a lattice with the same
 * rho_ref) plus the step counter.
 * Restoring and stepping reproduces an uninterrupted run bit for bit.
 * Synchronise. */
fmlb_status fmlb_save_raw(fmlb_ctx *ctx, void *host, size_t bytes, int64_t *step);
fmlb_status fmlb_load_raw(fmlb_ctx *ctx, const void *host, size_t bytes, int64_t step);

/* counts[0] = sites where not (rho_1 > 0 and rho_2 > 0) (the noise amplitude
 * of such a site is taken as 0, Sec. VII: local densities), counts[1] =
 * sites with a non-finite population, for the current state.  Synchronises. */
fmlb_status fmlb_health(fmlb_ctx *ctx, int64_t counts[2]);

/* Launch shape of the fused step: tile of tile_x x tile_y sites per
 * workgroup in the plane orthogonal to the march axis (z for D3Q19, y for
 * D2Q9, where tile_y must be 1) and `march` planes walked per workgroup.
 * Supported tiles: D3Q19 256x2 (full-width rows: only for nx = 256), 128x4,
 * 64x4, 64x8, 32x8, 32x16; D2Q9 64x1, 128x1, 256x1; march 1..4096.
 * 0 = default for each argument: the tile from the lattice width and the
 * storage, the march the longest that still gives about one workgroup per
 * CU (D3Q19) or per two tile rows (small D2Q9 lattices, which are bound by
 * latency).  tile_x = 1 selects the two-pass form (a density pass, then the
 * step).  Results do not depend on the choice (same bits).  FMLB_E_INVALID
 * for an unsupported shape. */
fmlb_status fmlb_set_tile(fmlb_ctx *ctx, int tile_x, int tile_y, int march);

/* Offset added (mod 2^32) to the site word of the noise counter: the step at
 * local site s draws the normals the convention above assigns to site
 * (s + site_offset) mod 2^32, so the noise stays independent per mode and
 * site (Sec. VI A) across lattices that share a seed.  A lattice that holds
 * one slab of a larger lattice (its edge planes copied in from the
 * neighbouring slabs after every step, as a decomposition across GPUs
 * would) sets it to the larger lattice's index of its first site minus its
 * own, mod 2^32, and then draws exactly the noise of the undivided run.
 * Default 0.  A lattice with a nonzero offset steps in the two-pass form
 * (density pass, then step; same bits as the fused form), which keeps the
 * fused kernels free of the extra argument.  Applies to the following steps.
 * FMLB_E_INVALID outside [0, 2^32). */
fmlb_status fmlb_set_counter_offset(fmlb_ctx *ctx, int64_t site_offset);

/* Memory reference for the roofline (not part of the method): one launch of
 * a plain copy kernel that reads every population of the current state with
 * the pull offsets of a step (one site per thread, workgroups in row order)
 * and writes it unchanged to the other buffer: the same bytes and addresses
 * as one step, with no halo, no ring, no arithmetic.  Its time is the
 * practical floor of the step's traffic on the device.  The state is not
 * changed (the other buffer is scratch between steps; the step counter does
 * not advance).  Asynchronous. */
fmlb_status fmlb_copy_reference(fmlb_ctx *ctx);

/* Further memory references for the roofline (not part of the method), one
 * launch each over the current population buffer viewed as 16-byte words
 * (a tail of fewer than 16 bytes is left out):
 *   FMLB_BW_PULL_COPY  fmlb_copy_reference;
 *   FMLB_BW_READ       read every word of the state (2048 workgroups);
 *   FMLB_BW_WRITE      write zeros over the other buffer (256 workgroups);
 *   FMLB_BW_COPY16     copy the state to the other buffer, unshifted,
 *                      16-byte words, 4 in flight per thread (256 workgroups).
 * *bytes (may be NULL) receives the bytes the launch reads plus writes.  The
 * state is unchanged (the other buffer is scratch between steps).
 * FMLB_E_INVALID for an unknown kind.  Asynchronous. */
enum { FMLB_BW_PULL_COPY = 0, FMLB_BW_READ = 1, FMLB_BW_WRITE = 2, FMLB_BW_COPY16 = 3 };
fmlb_status fmlb_bandwidth_reference(fmlb_ctx *ctx, int kind, double *bytes);

/* Human-readable name of a status code; the last HIP error code of any call. */
const char *fmlb_status_string(fmlb_status s);
int32_t fmlb_last_hip_error(void);

/* ------------------------------------------------------------------------ */
/* Batched replicas (many independent small lattices, e.g. a parameter scan   */
/* of the Sec. VI A equipartition and structure-factor checks): D2Q9          */
/* lattices of any nx x ny with FP32 storage, each with its own seed, k_B T,  */
/* G and relaxation times, advanced together by ONE launch per step over a    */
/* work list of (replica, tile, chunk) items.  Each item runs the same        */
/* per-tile code as the single-lattice fused step with the replica's own      */
/* geometry, parameters, seed and site numbering, so replica r evolves bit    */
/* for bit as an fmlb_ctx created from p[r] would (same step numbers).        */
/*                                                                            */
/* Layout: buffers A and B each hold every replica's [2][9][sites_r] block,   */
/* in replica order, each block starting on a 256-byte boundary.  The         */
/* pre-collision state of step n is in buffer (n mod 2).  The step number     */
/* also lives in the scratch buffer, read by every step launch, so the steps  */
/* can be replayed from a captured HIP graph.                                 */
/* ------------------------------------------------------------------------ */
typedef struct fmlb_batch fmlb_batch;

/* Bytes of buffer `which` (FMLB_BUF_*) for n replicas p[0..n-1]; 0 if any
 * p[r] is not a valid D2Q9 / FMLB_F32 lattice (flags: FMLB_NOISE_* bits only)
 * or n is outside [1, 65535].  POPS_A / POPS_B: per replica 2 x 9 population
 * arrays of nx ny floats each padded to a multiple of 64 (so that every array
 * starts on a 256-byte boundary). */
size_t fmlb_batch_required_bytes(const fmlb_params *p, int n, int which);

/* Borrow three 256-byte-aligned device buffers of at least the required
 * sizes; the replica parameters are copied.  The batch starts at step 0 with
 * no replica initialised.  Synchronises.  FMLB_E_INVALID as for
 * fmlb_batch_required_bytes or a misaligned buffer. */
fmlb_status fmlb_batch_create(const fmlb_params *p, int n, void *hip_stream,
                              void *const dev_buf[3], fmlb_batch **out);
void fmlb_batch_destroy(fmlb_batch *b);
int fmlb_batch_size(const fmlb_batch *b);
int64_t fmlb_batch_total_sites(const fmlb_batch *b);
int64_t fmlb_batch_current_step(const fmlb_batch *b);

/* Rest state f_bar_i = w_i rho_sigma of replica r from host FP64 densities
 * rho1[sites_r], rho2[sites_r], placed at the batch's current step (the step
 * counter is not reset).  Synchronises. */
fmlb_status fmlb_batch_init_density(fmlb_batch *b, int r, const double *rho1, const double *rho2);

/* Advance every replica n steps (asynchronous).  use_graph != 0 replays a
 * HIP graph of 32 steps on the batch's stream for each whole group of 32
 * (recorded at first use on a private stream the batch owns) and launches
 * the rest directly; the results are identical.  FMLB_E_STATE until every
 * replica has been initialised. */
fmlb_status fmlb_batch_step(fmlb_batch *b, int64_t n, int use_graph);

/* Work-list shape (results do not depend on it; discards a captured graph):
 *   tile_x = FMLB_BATCH_PACKED (T = 256) or FMLB_BATCH_PACKED_512 (T = 512):
 *     packed sites.  A workgroup of T threads walks a contiguous run of a
 *     replica's sites in row-major order, T sites per block and `march`
 *     blocks per item, for replicas up to (T + 1) / 2 wide (128 or 256);
 *     wider replicas get 256-site one-row tiles of `march` rows in a second
 *     launch.
 *   tile_x = 64, 128 or 256: one-row tiles of tile_x sites, `march` rows
 *     per item, for every replica.
 * march 1..4096.  0 = default for each: FMLB_BATCH_PACKED_512, with the
 * longest march up to 16 that leaves about 2048 items. */
#define FMLB_BATCH_PACKED 1
#define FMLB_BATCH_PACKED_512 2
fmlb_status fmlb_batch_set_tile(fmlb_batch *b, int tile_x, int march);

/* Tile autotuner: times every supported work-list shape (tile_x packed 256
 * and 512, 64, 128, 256 x march 1, 2, 4, 8, 16, 32, 64) over `reps` recomputations of the next step
 * (the state and the step counter are left unchanged: each trial re-reads
 * the current state and overwrites the other buffer), keeps the fastest and
 * reports it.  Synchronises.  FMLB_E_STATE until every replica is
 * initialised; FMLB_E_INVALID for reps outside [1, 1000]. */
fmlb_status fmlb_batch_autotune(fmlb_batch *b, int reps, int *tile_x, int *march);

/* As fmlb_get_populations, for replica r.  Synchronises. */
fmlb_status fmlb_batch_get_populations(fmlb_batch *b, int r, double *host, size_t bytes);

/* As fmlb_global_sums, for replica r: out[4] = sum rho_1, sum rho_2,
 * sum (j_bar_1 + j_bar_2)_x, _y.  Synchronises. */
fmlb_status fmlb_batch_global_sums(fmlb_batch *b, int r, double *out);

/* Equipartition statistics of every replica: accumulate adds the current
 * state's per-replica mode sums (as fmlb_mode_accumulate); variances gives
 * replica r's out[2][9] normalised with its own k_B T and sampled mean
 * densities (as fmlb_mode_variances, with the same errors); reset clears
 * every replica's sums. */
fmlb_status fmlb_batch_mode_accumulate(fmlb_batch *b);
fmlb_status fmlb_batch_mode_variances(fmlb_batch *b, int r, double *out, int64_t *n_samples);
fmlb_status fmlb_batch_reset_modes(fmlb_batch *b);

/* ------------------------------------------------------------------------
 * N species (2..FMLB_MAX_SPECIES): the multicomponent form of the model
 * (Apps. C and D).  Per site and species sigma:
 *   a_sigma = -sum_s' G[sigma][s'] sum_i w_i rho_s'(r + c_i) c_i   (Eq. (87)
 *             with one coupling per pair; G symmetric),
 *   u = sum_sigma (j_bar_sigma + rho_sigma a_sigma / 2) / rho_t,
 *   momentum modes relaxed with lambda_d towards rho_sigma u, with the
 *   forcing of Eq. (72) and a noise of covariance (2 lambda_d - lambda_d^2)
 *   k_B T (rho_sigma delta - rho_sigma rho_s' / rho_t) per component (App. D;
 *   zero total), sampled as L z with L the Cholesky factor of the block of
 *   species 1..N-1 (normals k D + alpha) and the last species taking minus
 *   the sum; every other mode of species sigma as in the binary model, with
 *   its own tau and the normals D (N - 1) + sigma (Q - D - 1) + ....  For
 *   N = 2 this is the binary model on the same normals (same sample path up
 *   to rounding).  One kernel per step (the potentials of the next plane in
 *   an LDS ring, its populations pulled into LDS ahead of use) or two (a
 *   potential pass, then the step); fmlb_multi_set_form.  Storage FMLB_F64
 *   or FMLB_F32 (deviations from w_i rho_ref).
 * ------------------------------------------------------------------------ */
#define FMLB_MAX_SPECIES 4

typedef struct fmlb_multi_params {
    int32_t lattice;    /* fmlb_lattice                                             */
    int32_t storage;    /* FMLB_F64 or FMLB_F32                                     */
    int32_t nspecies;   /* 2 .. FMLB_MAX_SPECIES                                    */
    int32_t nx, ny, nz; /* as fmlb_params                                           */
    double tau[FMLB_MAX_SPECIES];  /* per species (transport and ghost modes), > 1/2 */
    double tau_d;                  /* momentum modes of every species, > 1/2        */
    double G[FMLB_MAX_SPECIES][FMLB_MAX_SPECIES]; /* symmetric pair couplings        */
    double kT;                     /* >= 0                                           */
    double rho_ref[FMLB_MAX_SPECIES]; /* reference densities of the FP32 deviations  */
    uint64_t seed;
    uint32_t flags;                /* FMLB_NOISE_* bits; others: FMLB_E_INVALID       */
} fmlb_multi_params;

typedef struct fmlb_multi fmlb_multi;

/* Bytes of buffer `which` (FMLB_BUF_*), 0 for invalid parameters: POPS_A /
 * POPS_B: N * Q * sites * element size; SCRATCH: the potentials, FP64
 * staging and reduction partials.  256-byte aligned buffers. */
size_t fmlb_multi_required_bytes(const fmlb_multi_params *p, int which);

/* Validate and bind three caller-owned device buffers and a HIP stream.
 * FMLB_E_INVALID: nspecies outside 2..4, G not symmetric, storage other than
 * F64/F32, or the conditions of fmlb_create.  The library allocates no
 * device memory. */
fmlb_status fmlb_multi_create(const fmlb_multi_params *p, void *hip_stream, void *const dev_buf[3],
                              fmlb_multi **out);
void fmlb_multi_destroy(fmlb_multi *m);

/* Rest state f_bar_i = w_i rho[sigma][site] from host FP64 densities
 * rho[N][sites]; step counter 0.  Synchronises. */
fmlb_status fmlb_multi_init_density(fmlb_multi *m, const double *rho);

/* Advance n >= 0 steps (asynchronous).  FMLB_E_STATE before an initial state. */
fmlb_status fmlb_multi_step(fmlb_multi *m, int64_t n);

/* Launch forms of the N-species step; all give the same bits.
 *   FMLB_MULTI_AUTO (default): ASYNC where it applies (FP32 storage, one
 *     species' array under 4 GiB), else TWO_PASS.
 *   FMLB_MULTI_TWO_PASS: a potential pass, then the step (any storage).
 *   FMLB_MULTI_FUSED: one pass with register pulls: a tile_x x tile_y tile of
 *     the plane orthogonal to the march axis (D3Q19: 64x4, 64x8 or 32x8;
 *     D2Q9: 64x1, 128x1 or 256x1) walking `march` planes.
 *   FMLB_MULTI_ASYNC: one pass, the next plane's populations pulled straight
 *     into LDS while the current plane collides (D3Q19 tiles 64x4, 64x8, 32x8
 *     or 32x4 where their LDS fits: 64x8 two species only; D2Q9 64x1, 128x1
 *     or 256x1); FP32 storage only.
 * tile_x = tile_y = 0 and march = 0 select the defaults (march: 1..4096).
 * FMLB_E_INVALID for an unknown form or shape, or a tile or march given to
 * AUTO / TWO_PASS; FMLB_E_UNSUPPORTED for ASYNC on a lattice it does not
 * run. */
enum { FMLB_MULTI_AUTO = 0, FMLB_MULTI_TWO_PASS = 1, FMLB_MULTI_FUSED = 2, FMLB_MULTI_ASYNC = 3 };
fmlb_status fmlb_multi_set_form(fmlb_multi *m, int form, int tile_x, int tile_y, int march);

/* Shorthand kept for the register single pass: (0, 0, 0) = AUTO,
 * (1, 0, 0) = TWO_PASS, tile_x > 1 = FUSED with that tile and march;
 * anything else FMLB_E_INVALID. */
fmlb_status fmlb_multi_set_tile(fmlb_multi *m, int tile_x, int tile_y, int march);
int64_t fmlb_multi_current_step(const fmlb_multi *m);

/* Pre-collision populations f_bar[N][Q][sites] (FP64, absolute) to / from
 * host memory (bytes >= 8 N Q sites); set also sets the step counter.
 * Synchronise. */
fmlb_status fmlb_multi_get_populations(fmlb_multi *m, double *host, size_t bytes);
fmlb_status fmlb_multi_set_populations(fmlb_multi *m, const double *host, size_t bytes, int64_t step);

/* rho[N][sites] and j_bar[N][D][sites] (FP64) of the current state; either
 * may be NULL.  Synchronises. */
fmlb_status fmlb_multi_moments(fmlb_multi *m, double *rho, double *j);

/* out[sigma] = sum rho_sigma (sigma < N), out[N + alpha] = total momentum
 * sum_sigma j_bar_sigma,alpha (alpha < D); FP64.  Synchronises. */
fmlb_status fmlb_multi_global_sums(fmlb_multi *m, double *out);

#ifdef __cplusplus
}
#endif
#endif /* FMLB_H */
