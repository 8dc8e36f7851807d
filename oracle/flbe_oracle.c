/*
 * FP64 CPU oracle of the two-species fluctuating lattice Boltzmann equation
 * of arXiv:1410.5584.  TEST INFRASTRUCTURE ONLY: see flbe_oracle.h.
 *
 * One time step, written in the paper's order and notation (Sec. V):
 *
 *   pass 1  rho_sigma = sum_i f_bar_i,  j_bar_sigma = sum_i c_i f_bar_i   (Eq. (86))
 *   pass 2  for every site r and species sigma:
 *           a_sigma(r) = -G sum_i w_i rho_sigma'(r + c_i) c_i              (Eq. (87))
 *           v_b_bar = (j_bar + j_bar')/rho_t, a_b = (rho a + rho' a')/rho_t  (after Eq. (85))
 *           m_a = sum_i T_ai f_bar_i                                         (Eq. (80))
 *           R_a = lambda_a (m_eq_a(rho, v_b_bar + a_b/2) - m_a)
 *                 + (1 - lambda_a/2) Phi_a + xi_bar_a                        (Eqs. (85), (72), (74))
 *           f*_i = f_bar_i + w_i sum_a T_ai R_a / N_a                        (Eq. (84), right side)
 *   pass 3  f_bar_i(r + c_i, n + 1) = f*_i(r)                                 (Eq. (84), left side)
 *
 * Everything is double precision; no step is fused with another.
 */
#include "flbe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19
#define SPECIES 2

struct orc_sim {
    orc_params p;
    int Q, D, K;          /* velocities, dimensions, normals per site */
    int c[QMAX][3];
    double w[QMAX];
    double T[QMAX][QMAX]; /* T[a][i] */
    double N[QMAX];
    int64_t nsites;
    int64_t step;
    double *f;     /* [2][Q][nsites]  pre-collision f_bar(r, n) */
    double *fnew;  /* [2][Q][nsites]  next state (written by streaming) */
    double *rho;   /* [2][nsites]     pass-1 densities of f */
    double *j;     /* [2][3][nsites]  pass-1 momenta of f */
    int moments_valid;
};

/* ------------------------------------------------------------------------- */
/* Lattices and the mode basis                                               */
/* ------------------------------------------------------------------------- */

/* D2Q9 velocities.  With c_s^2 = 1/3 (Sec. V B) the isotropy relations of
 * Eq. (77) fix the weights: sum w = 1, sum w c_x^2 = 1/3 and sum w c_x^2 c_y^2
 * = 1/9 give 4/9 (rest), 1/9 (axis), 1/36 (diagonal). */
static const int D2Q9_C[9][2] = {
    {0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};

/* D3Q19 velocities.  The same three relations of Eq. (77) give 1/3 (rest),
 * 1/18 (6 axis links) and 1/36 (12 edge links); the fourth-order relation
 * sum w c_x^4 = 3 c_s^4 then holds as well. */
static const int D3Q19_C[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Table I: the D2Q9 modes T_a(c_i), a = 0..8, verbatim. */
static double table1_mode(int a, int cx, int cy)
{
    const double c2 = (double)(cx * cx + cy * cy);
    switch (a) {
    case 0: return 1.0;                               /* rho          */
    case 1: return cx;                                /* j_x          */
    case 2: return cy;                                /* j_y          */
    case 3: return 3.0 * c2 - 2.0;                    /* e            */
    case 4: return 2.0 * cx * cx - c2;                /* P_ww         */
    case 5: return (double)(cx * cy);                 /* P_xy         */
    case 6: return (3.0 * c2 - 4.0) * cx;             /* q_x          */
    case 7: return (3.0 * c2 - 4.0) * cy;             /* q_y          */
    case 8: return 9.0 * c2 * c2 - 15.0 * c2 + 2.0;   /* epsilon      */
    }
    return 0.0;
}

/* D3Q19 modes.  Modes 0..9 are the Hermite modes of Eq. (26), T_0 = 1,
 * T_alpha = c_alpha, T_theta(alpha beta) = c_alpha c_beta - c_s^2 delta,
 * ordered by the index theta_(alpha beta) given after Eq. (25) (xx, yy, zz,
 * xy, yz, xz).  The paper does not treat D3Q19; for the nine ghost modes it
 * only asks (Sec. V B) that the discrete orthogonality and completeness of
 * Eq. (79) hold.  This oracle uses the weighted-orthogonal set
 *   q_alpha = (3|c|^2 - 5) c_alpha,
 *   (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z,
 *   (2|c|^2 - 3)(3 c_x^2 - |c|^2), (2|c|^2 - 3)(c_y^2 - c_z^2),
 *   3|c|^4 - 6|c|^2 + 1,
 * the same construction as Table I's ghosts (odd cubic currents, even
 * quartic modes) carried to three dimensions. */
static double d3q19_mode(int a, int cx, int cy, int cz)
{
    const double x = cx, y = cy, z = cz;
    const double c2 = x * x + y * y + z * z;
    const double third = 1.0 / 3.0;
    switch (a) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x - third;
    case 5: return y * y - third;
    case 6: return z * z - third;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    case 17: return (2.0 * c2 - 3.0) * (y * y - z * z);
    case 18: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    }
    return 0.0;
}

int orc_basis(int lattice, int *D, int *c, double *w, double *T, double *N)
{
    int Q, dim;
    if (lattice == ORC_D2Q9) {
        Q = 9;
        dim = 2;
    } else if (lattice == ORC_D3Q19) {
        Q = 19;
        dim = 3;
    } else {
        return -1;
    }
    for (int i = 0; i < Q; ++i) {
        int ci[3] = {0, 0, 0};
        if (lattice == ORC_D2Q9) {
            ci[0] = D2Q9_C[i][0];
            ci[1] = D2Q9_C[i][1];
        } else {
            ci[0] = D3Q19_C[i][0];
            ci[1] = D3Q19_C[i][1];
            ci[2] = D3Q19_C[i][2];
        }
        const int c2 = ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2];
        double wi;
        if (lattice == ORC_D2Q9)
            wi = (c2 == 0) ? 4.0 / 9.0 : (c2 == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
        else
            wi = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        if (c)
            for (int k = 0; k < 3; ++k) c[3 * i + k] = ci[k];
        if (w) w[i] = wi;
        if (T)
            for (int a = 0; a < Q; ++a)
                T[a * Q + i] = (lattice == ORC_D2Q9) ? table1_mode(a, ci[0], ci[1])
                                                      : d3q19_mode(a, ci[0], ci[1], ci[2]);
    }
    if (N) {
        /* Squared norms, N_a = sum_i w_i T_ai^2 (Eq. (79)). */
        for (int a = 0; a < Q; ++a) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) {
                int ci[3] = {0, 0, 0};
                if (lattice == ORC_D2Q9) {
                    ci[0] = D2Q9_C[i][0];
                    ci[1] = D2Q9_C[i][1];
                } else {
                    ci[0] = D3Q19_C[i][0];
                    ci[1] = D3Q19_C[i][1];
                    ci[2] = D3Q19_C[i][2];
                }
                const int c2 = ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2];
                double wi;
                if (lattice == ORC_D2Q9)
                    wi = (c2 == 0) ? 4.0 / 9.0 : (c2 == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
                else
                    wi = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
                const double t = (lattice == ORC_D2Q9) ? table1_mode(a, ci[0], ci[1])
                                                       : d3q19_mode(a, ci[0], ci[1], ci[2]);
                s += wi * t * t;
            }
            N[a] = s;
        }
    }
    if (D) *D = dim;
    return Q;
}

/* ------------------------------------------------------------------------- */
/* Random numbers                                                            */
/* ------------------------------------------------------------------------- */

/* Philox4x32-10 as published by Salmon et al. (SC'11): ten rounds of two
 * 32x32->64-bit multiplications; the key is bumped by the Weyl constants
 * between rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        const uint32_t y3 = (uint32_t)p0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Uniform number k of a site and step.  Word w = k / 2 of the site's stream
 * is word w % 4 of block j = w / 4, Philox4x32-10(counter = (site,
 * step mod 2^32, j, step / 2^32), key = (seed mod 2^32, seed / 2^32)).
 * Each word gives two 16-bit integers, U = word >> 16 (even k) and
 * U = word & 0xffff (odd k); the uniform is u = (2U + 1) / 2^17, in (0, 1). */
void orc_uniforms(uint64_t seed, uint32_t site, int64_t step, int n, double *u)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4] = {0, 0, 0, 0};
    int have = -1;
    for (int k = 0; k < n; ++k) {
        const int w = k / 2, j = w / 4;
        if (j != have) {
            const uint32_t ctr[4] = {site, (uint32_t)(uint64_t)step, (uint32_t)j,
                                     (uint32_t)((uint64_t)step >> 32)};
            orc_philox4x32_10(ctr, key, x);
            have = j;
        }
        const uint32_t word = x[w % 4];
        const uint32_t U = (k % 2 == 0) ? (word >> 16) : (word & 0xffffu);
        u[k] = ldexp(2.0 * (double)U + 1.0, -17);
    }
}

/* Gaussian normals by the trigonometric Box-Muller transform on consecutive
 * pairs of uniforms (Sec. VI A: independent Gaussian noise per mode and site,
 * Box-Muller):  z_2p = sqrt(-2 ln u_2p) cos(2 pi u_2p+1),
 *               z_2p+1 = sqrt(-2 ln u_2p) sin(2 pi u_2p+1). */
int orc_normals(uint64_t seed, uint32_t site, int64_t step, int K, double *z)
{
    double u[ORC_MAX_NORMALS]; /* 2 ceil(K / 2) <= ORC_MAX_NORMALS uniforms (the bound is even) */
    if (K < 0 || K > ORC_MAX_NORMALS || !z) return -1;
    const int pairs = (K + 1) / 2;
    orc_uniforms(seed, site, step, 2 * pairs, u);
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < pairs; ++p) {
        const double r = sqrt(-2.0 * log(u[2 * p]));
        const double th = two_pi * u[2 * p + 1];
        z[2 * p] = r * cos(th);
        if (2 * p + 1 < K) z[2 * p + 1] = r * sin(th);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Simulation state                                                          */
/* ------------------------------------------------------------------------- */

orc_sim *orc_create(const orc_params *p)
{
    if (!p) return NULL;
    if (p->lattice != ORC_D2Q9 && p->lattice != ORC_D3Q19) return NULL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    if (p->lattice == ORC_D2Q9 && p->nz != 1) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->p = *p;
    int c[QMAX * 3];
    double T[QMAX * QMAX];
    s->Q = orc_basis(p->lattice, &s->D, c, s->w, T, s->N);
    s->K = s->D + SPECIES * (s->Q - s->D - 1);
    if (s->K > ORC_MAX_NORMALS) {
        free(s);
        return NULL;
    }
    for (int i = 0; i < s->Q; ++i)
        for (int k = 0; k < 3; ++k) s->c[i][k] = c[3 * i + k];
    for (int a = 0; a < s->Q; ++a)
        for (int i = 0; i < s->Q; ++i) s->T[a][i] = T[a * s->Q + i];
    s->nsites = (int64_t)p->nx * p->ny * p->nz;
    const size_t npop = (size_t)SPECIES * s->Q * s->nsites;
    s->f = (double *)calloc(npop, sizeof(double));
    s->fnew = (double *)calloc(npop, sizeof(double));
    s->rho = (double *)calloc((size_t)SPECIES * s->nsites, sizeof(double));
    s->j = (double *)calloc((size_t)SPECIES * 3 * s->nsites, sizeof(double));
    if (!s->f || !s->fnew || !s->rho || !s->j) {
        orc_destroy(s);
        return NULL;
    }
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->f);
    free(s->fnew);
    free(s->rho);
    free(s->j);
    free(s);
}

int64_t orc_num_sites(const orc_sim *s) { return s ? s->nsites : -1; }
int64_t orc_current_step(const orc_sim *s) { return s ? s->step : -1; }

static inline double *pop(const orc_sim *s, double *base, int sp, int i)
{
    return base + ((size_t)sp * s->Q + i) * (size_t)s->nsites;
}

/* Site index of r + c_i with periodic wrap. */
static inline int64_t neighbour(const orc_sim *s, int64_t site, const int ci[3])
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const int x = (int)(site % nx);
    const int y = (int)((site / nx) % ny);
    const int z = (int)(site / ((int64_t)nx * ny));
    const int xn = ((x + ci[0]) % nx + nx) % nx;
    const int yn = ((y + ci[1]) % ny + ny) % ny;
    const int zn = ((z + ci[2]) % nz + nz) % nz;
    return (int64_t)xn + (int64_t)nx * (yn + (int64_t)ny * zn);
}

int orc_init_density(orc_sim *s, const double *rho1, const double *rho2)
{
    if (!s || !rho1 || !rho2) return -1;
    const double *rho[2] = {rho1, rho2};
    for (int sp = 0; sp < SPECIES; ++sp)
        for (int i = 0; i < s->Q; ++i) {
            double *fi = pop(s, s->f, sp, i);
            for (int64_t r = 0; r < s->nsites; ++r) fi[r] = s->w[i] * rho[sp][r];
        }
    s->step = 0;
    s->moments_valid = 0;
    return 0;
}

int orc_set_populations(orc_sim *s, const double *f, int64_t step)
{
    if (!s || !f || step < 0) return -1;
    memcpy(s->f, f, sizeof(double) * (size_t)SPECIES * s->Q * s->nsites);
    s->step = step;
    s->moments_valid = 0;
    return 0;
}

int orc_get_populations(const orc_sim *s, double *f)
{
    if (!s || !f) return -1;
    memcpy(f, s->f, sizeof(double) * (size_t)SPECIES * s->Q * s->nsites);
    return 0;
}

/* Pass 1: rho_sigma = sum_i f_bar_i and j_bar_sigma = sum_i c_i f_bar_i at every
 * site (Eq. (86)). */
static void pass1_moments(orc_sim *s)
{
    const int64_t ns = s->nsites;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < ns; ++r) {
        for (int sp = 0; sp < SPECIES; ++sp) {
            double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < s->Q; ++i) {
                const double fi = pop(s, s->f, sp, i)[r];
                rho += fi;
                for (int al = 0; al < s->D; ++al) j[al] += s->c[i][al] * fi;
            }
            s->rho[(size_t)sp * ns + r] = rho;
            for (int al = 0; al < 3; ++al) s->j[((size_t)sp * 3 + al) * ns + r] = j[al];
        }
    }
    s->moments_valid = 1;
}

/* Lattice force of Eq. (87): a_sigma(r) = -G sum_i w_i rho_sigma'(r + c_i) c_i,
 * from the pass-1 densities of the same time level. */
static void lattice_acceleration(const orc_sim *s, int64_t r, double a[2][3])
{
    const int64_t ns = s->nsites;
    for (int sp = 0; sp < SPECIES; ++sp) {
        const int other = 1 - sp;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < s->Q; ++i) {
            const int64_t nb = neighbour(s, r, s->c[i]);
            const double rho_o = s->rho[(size_t)other * ns + nb];
            for (int al = 0; al < s->D; ++al) acc[al] += s->w[i] * rho_o * s->c[i][al];
        }
        for (int al = 0; al < 3; ++al) a[sp][al] = (al < s->D) ? -s->p.G * acc[al] : 0.0;
    }
}

/* Collision at one site (right-hand side of Eq. (84)); needs pass 1. */
static void collide_site(const orc_sim *s, int64_t r, double fstar[2][QMAX])
{
    const int Q = s->Q, D = s->D;
    const int64_t ns = s->nsites;
    const orc_params *p = &s->p;

    double rho[2], jb[2][3], a[2][3], F[2][3];
    for (int sp = 0; sp < SPECIES; ++sp) {
        rho[sp] = s->rho[(size_t)sp * ns + r];
        for (int al = 0; al < 3; ++al) jb[sp][al] = s->j[((size_t)sp * 3 + al) * ns + r];
    }
    lattice_acceleration(s, r, a);
    for (int sp = 0; sp < SPECIES; ++sp)
        for (int al = 0; al < 3; ++al) F[sp][al] = rho[sp] * a[sp][al];

    /* Equilibrium velocity v_b_bar + a_b / 2 (Eq. (85) and the definitions
     * that follow it). */
    const double rt = rho[0] + rho[1];
    double u[3] = {0.0, 0.0, 0.0};
    if (rt > 0.0)
        for (int al = 0; al < D; ++al) {
            const double vb_bar = (jb[0][al] + jb[1][al]) / rt;
            const double ab = (F[0][al] + F[1][al]) / rt;
            u[al] = vb_bar + 0.5 * ab;
        }

    /* Thermal noise (Eq. (74)); mu = k_B T / c_s^2 with c_s^2 = 1/3 (Eq. (18)). */
    const int noisy = (p->kT > 0.0) && !(p->flags & ORC_NOISE_OFF);
    double z[ORC_MAX_NORMALS];
    if (!noisy || orc_normals(p->seed, (uint32_t)r, s->step, s->K, z) != 0)
        for (int k = 0; k < s->K; ++k) z[k] = 0.0; /* K <= ORC_MAX_NORMALS: checked by orc_create */
    const double mu = 3.0 * p->kT;
    const double lam_d = 1.0 / p->tau_d;
    double sig_d = 0.0;
    if (noisy && !(p->flags & ORC_NOISE_NO_SDF) && rho[0] > 0.0 && rho[1] > 0.0)
        sig_d = sqrt((2.0 * lam_d - lam_d * lam_d) * p->kT * rho[0] * rho[1] / rt);

    for (int sp = 0; sp < SPECIES; ++sp) {
        const double *fb[QMAX];
        for (int i = 0; i < Q; ++i) fb[i] = pop(s, s->f, sp, i) + r;
        const double lam = 1.0 / p->tau[sp];

        /* Moments m_a = sum_i T_ai f_bar_i (Eq. (80)). */
        double m[QMAX];
        for (int a_ = 0; a_ < Q; ++a_) {
            double acc = 0.0;
            for (int i = 0; i < Q; ++i) acc += s->T[a_][i] * (*fb[i]);
            m[a_] = acc;
        }

        double R[QMAX];
        R[0] = 0.0; /* mass is conserved: R_0 = 0 (Sec. V A) */

        /* Momentum modes (a = 1..D): relaxation lambda_d (Eq. (37)), m_eq =
         * rho u_alpha (Table I), Phi_alpha = rho a_alpha (first-order term of
         * Eq. (31)), noise +xi for species 1 and -xi for species 2 (Eq. (74)). */
        const double sign = (sp == 0) ? 1.0 : -1.0;
        for (int al = 0; al < D; ++al) {
            const double xi = sign * sig_d * z[al];
            R[1 + al] = lam_d * (rho[sp] * u[al] - m[1 + al]) + (1.0 - 0.5 * lam_d) * F[sp][al] + xi;
        }

        /* Physical species velocity rho v = rho v_bar + R_alpha / 2 (Eq. (65)
         * for the momentum modes; the same as Eq. (71)). */
        double v[3] = {0.0, 0.0, 0.0};
        if (rho[sp] > 0.0)
            for (int al = 0; al < D; ++al) v[al] = (m[1 + al] + 0.5 * R[1 + al]) / rho[sp];

        /* Discrete truncated Maxwellian (Eq. (29)) and second-order forcing
         * (Eq. (31)), with omega -> w_i and c_s^2 = 1/3. */
        double feq[QMAX], phi[QMAX];
        double uu = 0.0, av = 0.0;
        for (int al = 0; al < D; ++al) {
            uu += u[al] * u[al];
            av += a[sp][al] * v[al];
        }
        for (int i = 0; i < Q; ++i) {
            double cu = 0.0, ca = 0.0, cv = 0.0;
            for (int al = 0; al < D; ++al) {
                cu += s->c[i][al] * u[al];
                ca += s->c[i][al] * a[sp][al];
                cv += s->c[i][al] * v[al];
            }
            feq[i] = s->w[i] * rho[sp] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            phi[i] = s->w[i] * rho[sp] * (3.0 * ca + 9.0 * (ca * cv - av / 3.0));
        }

        /* Transport and ghost modes (a = D+1..Q-1): relaxation lambda_sigma,
         * m_eq_a and Phi_a as projections (Table I caption: m_eq_a =
         * sum_i T_ai f_eq_i), renormalised forcing (Eq. (72)), diagonal
         * noise of variance (2 lambda - lambda^2) N_a mu rho (Eq. (74)). */
        for (int a_ = D + 1; a_ < Q; ++a_) {
            double meq = 0.0, Phi = 0.0;
            for (int i = 0; i < Q; ++i) {
                meq += s->T[a_][i] * feq[i];
                Phi += s->T[a_][i] * phi[i];
            }
            double sig = 0.0;
            if (noisy && rho[sp] > 0.0) sig = sqrt((2.0 * lam - lam * lam) * s->N[a_] * mu * rho[sp]);
            const double zz = z[D + sp * (Q - D - 1) + (a_ - D - 1)];
            R[a_] = lam * (meq - m[a_]) + (1.0 - 0.5 * lam) * Phi + sig * zz;
        }

        /* f*_i = f_bar_i + w_i sum_a T_ai R_a / N_a (Eq. (84)). */
        for (int i = 0; i < Q; ++i) {
            double acc = 0.0;
            for (int a_ = 0; a_ < Q; ++a_) acc += s->T[a_][i] * R[a_] / s->N[a_];
            fstar[sp][i] = *fb[i] + s->w[i] * acc;
        }
    }
}

int orc_step(orc_sim *s, int64_t n)
{
    if (!s || n < 0) return -1;
    const int64_t ns = s->nsites;
    for (int64_t t = 0; t < n; ++t) {
        pass1_moments(s);
        /* Pass 2 and 3: collide every site, then stream f*_i to r + c_i. */
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < ns; ++r) {
            double fstar[2][QMAX];
            collide_site(s, r, fstar);
            for (int sp = 0; sp < SPECIES; ++sp)
                for (int i = 0; i < s->Q; ++i) {
                    const int64_t dst = neighbour(s, r, s->c[i]);
                    pop(s, s->fnew, sp, i)[dst] = fstar[sp][i];
                }
        }
        double *tmp = s->f;
        s->f = s->fnew;
        s->fnew = tmp;
        s->step += 1;
        s->moments_valid = 0;
    }
    return 0;
}

int orc_moments(const orc_sim *cs, double *rho, double *j, double *F)
{
    orc_sim *s = (orc_sim *)cs;
    if (!s) return -1;
    if (!s->moments_valid) pass1_moments(s);
    const int64_t ns = s->nsites;
    const int D = s->D;
    if (rho) memcpy(rho, s->rho, sizeof(double) * SPECIES * (size_t)ns);
    if (j)
        for (int sp = 0; sp < SPECIES; ++sp)
            for (int al = 0; al < D; ++al)
                memcpy(j + ((size_t)sp * D + al) * ns, s->j + ((size_t)sp * 3 + al) * ns,
                       sizeof(double) * (size_t)ns);
    if (F) {
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < ns; ++r) {
            double a[2][3];
            lattice_acceleration(s, r, a);
            for (int sp = 0; sp < SPECIES; ++sp)
                for (int al = 0; al < D; ++al)
                    F[((size_t)sp * D + al) * ns + r] = s->rho[(size_t)sp * ns + r] * a[sp][al];
        }
    }
    return 0;
}

int orc_collide_site(const orc_sim *cs, int64_t site, double *fstar)
{
    orc_sim *s = (orc_sim *)cs;
    if (!s || !fstar || site < 0 || site >= s->nsites) return -1;
    if (!s->moments_valid) pass1_moments(s);
    double out[2][QMAX];
    collide_site(s, site, out);
    for (int sp = 0; sp < SPECIES; ++sp)
        for (int i = 0; i < s->Q; ++i) fstar[sp * s->Q + i] = out[sp][i];
    return 0;
}

int orc_health(const orc_sim *cs, int64_t counts[2])
{
    orc_sim *s = (orc_sim *)cs;
    if (!s || !counts) return -1;
    if (!s->moments_valid) pass1_moments(s);
    int64_t nonpos = 0, nonfinite = 0;
    for (int64_t r = 0; r < s->nsites; ++r) {
        if (!(s->rho[r] > 0.0) || !(s->rho[s->nsites + r] > 0.0)) nonpos++;
        int bad = 0;
        for (int sp = 0; sp < SPECIES; ++sp)
            for (int i = 0; i < s->Q; ++i)
                if (!isfinite(pop(s, s->f, sp, i)[r])) bad = 1;
        nonfinite += bad;
    }
    counts[0] = nonpos;
    counts[1] = nonfinite;
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
