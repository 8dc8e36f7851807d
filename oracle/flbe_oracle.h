/*
 * FP64 CPU oracle of the two-species fluctuating lattice Boltzmann equation
 * (Belardinelli, Sbragaglia, Biferale, Gross, Varnik, "Fluctuating
 * multicomponent lattice Boltzmann model", arXiv:1410.5584).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this code; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no code, header, table or constant with the GPU implementation.
 *
 * It follows the paper's algorithm step by step (Sec. V, Eqs. (84)-(86);
 * Table I; Eq. (87) for the lattice force; Eq. (74) for the noise), in plain
 * double precision, one site at a time, with no fusion or reordering beyond
 * what the equations state.  Layout of every field array: species-major, then
 * velocity / mode / component, then site index s = x + nx*(y + ny*z).
 */
#ifndef FLBE_ORACLE_H
#define FLBE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_D2Q9 0
#define ORC_D3Q19 1

#define ORC_NOISE_OFF 1u   /* no thermal noise at all (deterministic LBE)            */
#define ORC_NOISE_NO_SDF 2u /* no noise on the momentum modes (Sec. VI A, "no-sdf") */

typedef struct orc_params {
    int32_t lattice;  /* ORC_D2Q9 or ORC_D3Q19 */
    int32_t nx, ny, nz;
    double tau[2];    /* lambda_bar = 1/tau for the transport and ghost modes of species 1, 2 */
    double tau_d;     /* lambda_bar_d = 1/tau_d, momentum modes of both species (Eq. (37)) */
    double G;         /* coupling of the lattice force, Eq. (87) */
    double kT;        /* k_B T; mu = k_B T / c_s^2 (Eq. (18)) */
    uint64_t seed;    /* Philox key */
    uint32_t flags;
} orc_params;

typedef struct orc_sim orc_sim;

/* Lattice and mode basis.  c: [Q][3] ints, w: [Q], T: [Q][Q] row a = mode,
 * column i = velocity, N: [Q].  Returns Q, or -1 for an unknown lattice. */
int orc_basis(int lattice, int *D, int *c, double *w, double *T, double *N);

/* Philox4x32-10 bijection (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The K Gaussian normals of one site and step (project convention: counter
 * (site, step_lo, block, step_hi), key (seed_lo, seed_hi), each 32-bit word
 * split into two 16-bit uniforms, trigonometric Box-Muller on consecutive
 * pairs, i.e. one word per pair of normals). */
#define ORC_MAX_NORMALS 128 /* normals per site and step (D3Q19 with 4 species: 69) */
void orc_uniforms(uint64_t seed, uint32_t site, int64_t step, int n, double *u);
/* Returns 0, or -1 (z untouched) unless 0 <= K <= ORC_MAX_NORMALS. */
int orc_normals(uint64_t seed, uint32_t site, int64_t step, int K, double *z);

orc_sim *orc_create(const orc_params *p);
void orc_destroy(orc_sim *s);
int64_t orc_num_sites(const orc_sim *s);
int64_t orc_current_step(const orc_sim *s);

/* Pre-collision populations f_bar[2][Q][sites] = w_i rho_sigma(r): the
 * uniform-velocity rest state of Sec. VI A.  Step counter reset to 0. */
int orc_init_density(orc_sim *s, const double *rho1, const double *rho2);
int orc_set_populations(orc_sim *s, const double *f, int64_t step);
int orc_get_populations(const orc_sim *s, double *f);

/* Advance n steps of Eq. (84). */
int orc_step(orc_sim *s, int64_t n);

/* Observables of the stored pre-collision state: rho[2][sites],
 * j_bar[2][D][sites] (Eq. (86)), force F[2][D][sites] = rho_sigma a_sigma
 * (Eq. (87)).  Any pointer may be NULL. */
int orc_moments(const orc_sim *s, double *rho, double *j, double *F);

/* Post-collision populations f*[2][Q] at one site of the stored state (the
 * right-hand side of Eq. (84) before streaming). */
int orc_collide_site(const orc_sim *s, int64_t site, double *fstar);

/* Sites with rho_sigma <= 0 (either species), sites with a non-finite population. */
int orc_health(const orc_sim *s, int64_t counts[2]);

/* Threads the OpenMP loops use. */
int orc_num_threads(void);

/* ------------------------------------------------------------------------- */
/* N species (flbe_multi.c): the multicomponent model of Apps. C and D.       */
/* ------------------------------------------------------------------------- */
#define ORC_MAX_SPECIES 4

typedef struct orc_multi_params {
    int32_t lattice;   /* ORC_D2Q9 or ORC_D3Q19 */
    int32_t nspecies;  /* 2 .. ORC_MAX_SPECIES */
    int32_t nx, ny, nz;
    double tau[ORC_MAX_SPECIES];  /* transport and ghost modes of each species */
    double tau_d;                 /* momentum modes of every species */
    double G[ORC_MAX_SPECIES][ORC_MAX_SPECIES]; /* pair couplings, symmetric */
    double kT;
    uint64_t seed;
    uint32_t flags;
} orc_multi_params;

typedef struct orc_multi orc_multi;

orc_multi *orc_multi_create(const orc_multi_params *p);
void orc_multi_destroy(orc_multi *s);
int64_t orc_multi_current_step(const orc_multi *s);
/* f_bar[N][Q][sites] = w_i rho[sigma][site]; step counter reset to 0. */
int orc_multi_init_density(orc_multi *s, const double *rho);
int orc_multi_set_populations(orc_multi *s, const double *f, int64_t step);
int orc_multi_get_populations(const orc_multi *s, double *f);
int orc_multi_step(orc_multi *s, int64_t n);
/* rho[N][sites], j_bar[N][D][sites], F[N][D][sites] of the stored state (any may be NULL). */
int orc_multi_moments(orc_multi *s, double *rho, double *j, double *F);
/* Post-collision populations f*[N][Q] at one site of the stored state. */
int orc_multi_collide_site(orc_multi *s, int64_t site, double *fstar);

#ifdef __cplusplus
}
#endif
#endif
