/*
 * FP64 CPU oracle of the N-species fluctuating lattice Boltzmann equation
 * (arXiv:1410.5584, the multicomponent form of Apps. C and D).  TEST
 * INFRASTRUCTURE ONLY: see flbe_oracle.h.
 *
 * The binary step of flbe_oracle.c with species sigma = 1..N:
 *
 *   pass 1  rho_sigma = sum_i f_bar_i,  j_bar_sigma = sum_i c_i f_bar_i       (Eq. (86))
 *   pass 2  a_sigma(r) = -sum_s' G_sigma,s' sum_i w_i rho_s'(r + c_i) c_i
 *             (Eq. (87) with one coupling per pair of species; G symmetric)
 *           u = sum_sigma (j_bar_sigma + rho_sigma a_sigma / 2) / rho_t         (after Eq. (85))
 *           momentum modes: R = lambda_d (rho_sigma u - j_bar_sigma)
 *                               + (1 - lambda_d/2) rho_sigma a_sigma + xi_sigma
 *             with <xi_sigma,alpha xi_s',beta> = (2 lambda_d - lambda_d^2) k_B T
 *             (rho_sigma delta_sigma,s' - rho_sigma rho_s' / rho_t) delta_alpha,beta:
 *             the covariance of App. D (momentum part of the noise of the
 *             multicomponent model, lambda_d (delta - C) with the lattice
 *             factor 2 lambda - lambda^2 of Eq. (74));
 *           transport and ghost modes of each species as in the binary model;
 *           f*_i = f_bar_i + w_i sum_a T_ai R_a / N_a                        (Eq. (84))
 *   pass 3  f_bar_i(r + c_i, n + 1) = f*_i(r)
 *
 * Sampling the momentum noise (a convention of this project; the paper
 * gives only the covariance): the rows and columns of species 1..N-1 of
 * the covariance form a positive-definite matrix when every density is
 * positive; its Cholesky factor L gives xi_sigma,alpha = sum_k L_sigma,k
 * z_(k D + alpha) for sigma < N, and xi_N = -(xi_1 + ... + xi_(N-1)) because
 * every row of the covariance sums to zero (the total momentum receives no
 * noise).  For N = 2 this is xi_1 = sqrt(...) z_alpha = -xi_2, the binary
 * model's noise on the same normals.  The normals of the non-momentum modes
 * of species sigma follow at D (N - 1) + sigma (Q - D - 1) + (a - D - 1).
 */
#include "flbe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19
#define KMAX ORC_MAX_NORMALS

struct orc_multi {
    orc_multi_params p;
    int N, Q, D, K;
    int c[QMAX][3];
    double w[QMAX];
    double T[QMAX][QMAX];
    double Nn[QMAX];
    int64_t nsites;
    int64_t step;
    double *f;    /* [N][Q][nsites] */
    double *fnew;
    double *rho;  /* [N][nsites] */
    double *j;    /* [N][3][nsites] */
    int moments_valid; /* rho / j hold pass 1 of the current state */
};

orc_multi *orc_multi_create(const orc_multi_params *p)
{
    if (!p) return NULL;
    if (p->nspecies < 2 || p->nspecies > ORC_MAX_SPECIES) return NULL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    if (p->lattice == ORC_D2Q9 && p->nz != 1) return NULL;
    if (!(p->tau_d > 0.5) || !(p->kT >= 0.0)) return NULL;
    for (int s = 0; s < p->nspecies; ++s) {
        if (!(p->tau[s] > 0.5)) return NULL;
        for (int t = 0; t < p->nspecies; ++t)
            if (p->G[s][t] != p->G[t][s]) return NULL; /* pair forces need G symmetric */
    }
    orc_multi *s = (orc_multi *)calloc(1, sizeof(orc_multi));
    if (!s) return NULL;
    s->p = *p;
    s->N = p->nspecies;
    int cc[QMAX * 3];
    double T[QMAX * QMAX];
    s->Q = orc_basis(p->lattice, &s->D, cc, s->w, T, s->Nn);
    if (s->Q < 0) {
        free(s);
        return NULL;
    }
    for (int i = 0; i < s->Q; ++i)
        for (int al = 0; al < 3; ++al) s->c[i][al] = cc[3 * i + al];
    for (int a = 0; a < s->Q; ++a)
        for (int i = 0; i < s->Q; ++i) s->T[a][i] = T[a * s->Q + i];
    s->K = s->D * (s->N - 1) + s->N * (s->Q - s->D - 1);
    if (s->K > KMAX) {
        free(s);
        return NULL;
    }
    s->nsites = (int64_t)p->nx * p->ny * p->nz;
    const size_t nf = (size_t)s->N * s->Q * s->nsites;
    s->f = (double *)calloc(nf, sizeof(double));
    s->fnew = (double *)calloc(nf, sizeof(double));
    s->rho = (double *)calloc((size_t)s->N * s->nsites, sizeof(double));
    s->j = (double *)calloc((size_t)s->N * 3 * s->nsites, sizeof(double));
    if (!s->f || !s->fnew || !s->rho || !s->j) {
        orc_multi_destroy(s);
        return NULL;
    }
    return s;
}

void orc_multi_destroy(orc_multi *s)
{
    if (!s) return;
    free(s->f);
    free(s->fnew);
    free(s->rho);
    free(s->j);
    free(s);
}

int64_t orc_multi_current_step(const orc_multi *s) { return s ? s->step : -1; }

static inline double *mpop(const orc_multi *s, double *base, int sp, int i)
{
    return base + ((size_t)sp * s->Q + i) * s->nsites;
}

static inline int64_t mneighbour(const orc_multi *s, int64_t site, const int ci[3])
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const int x = (int)(site % nx);
    const int y = (int)((site / nx) % ny);
    const int z = (int)(site / ((int64_t)nx * ny));
    const int xn = (x + ci[0] + nx) % nx;
    const int yn = (y + ci[1] + ny) % ny;
    const int zn = (z + ci[2] + nz) % nz;
    return (int64_t)xn + (int64_t)nx * ((int64_t)yn + (int64_t)ny * zn);
}

int orc_multi_init_density(orc_multi *s, const double *rho)
{
    if (!s || !rho) return -1;
    for (int sp = 0; sp < s->N; ++sp)
        for (int i = 0; i < s->Q; ++i)
            for (int64_t r = 0; r < s->nsites; ++r)
                mpop(s, s->f, sp, i)[r] = s->w[i] * rho[(size_t)sp * s->nsites + r];
    s->step = 0;
    s->moments_valid = 0;
    return 0;
}

int orc_multi_set_populations(orc_multi *s, const double *f, int64_t step)
{
    if (!s || !f || step < 0) return -1;
    memcpy(s->f, f, (size_t)s->N * s->Q * s->nsites * sizeof(double));
    s->step = step;
    s->moments_valid = 0;
    return 0;
}

int orc_multi_get_populations(const orc_multi *s, double *f)
{
    if (!s || !f) return -1;
    memcpy(f, s->f, (size_t)s->N * s->Q * s->nsites * sizeof(double));
    return 0;
}

/* Pass 1 (Eq. (86)). */
static void multi_pass1(orc_multi *s)
{
    const int64_t ns = s->nsites;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < ns; ++r)
        for (int sp = 0; sp < s->N; ++sp) {
            double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < s->Q; ++i) {
                const double fi = mpop(s, s->f, sp, i)[r];
                rho += fi;
                for (int al = 0; al < s->D; ++al) j[al] += s->c[i][al] * fi;
            }
            s->rho[(size_t)sp * ns + r] = rho;
            for (int al = 0; al < 3; ++al) s->j[((size_t)sp * 3 + al) * ns + r] = j[al];
        }
    s->moments_valid = 1;
}

/* a_sigma(r) = -sum_s' G_sigma,s' sum_i w_i rho_s'(r + c_i) c_i (Eq. (87)
 * with a coupling per pair of species). */
static void multi_acceleration(const orc_multi *s, int64_t r, double a[ORC_MAX_SPECIES][3])
{
    const int64_t ns = s->nsites;
    for (int sp = 0; sp < s->N; ++sp) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < s->N; ++o) {
            const double G = s->p.G[sp][o];
            if (G == 0.0) continue;
            for (int i = 0; i < s->Q; ++i) {
                const double rho_o = s->rho[(size_t)o * ns + mneighbour(s, r, s->c[i])];
                for (int al = 0; al < s->D; ++al) acc[al] += G * s->w[i] * rho_o * s->c[i][al];
            }
        }
        for (int al = 0; al < 3; ++al) a[sp][al] = (al < s->D) ? -acc[al] : 0.0;
    }
}

/* Lower Cholesky factor of the n x n symmetric positive-definite A (row
 * major, leading dimension ORC_MAX_SPECIES).  A pivot that rounds to <= 0
 * (a density far below the others) gives a zero column instead of a NaN. */
static void cholesky(int n, const double A[ORC_MAX_SPECIES][ORC_MAX_SPECIES],
                     double L[ORC_MAX_SPECIES][ORC_MAX_SPECIES])
{
    for (int i = 0; i < ORC_MAX_SPECIES; ++i)
        for (int k = 0; k < ORC_MAX_SPECIES; ++k) L[i][k] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k <= i; ++k) {
            double sum = A[i][k];
            for (int m = 0; m < k; ++m) sum -= L[i][m] * L[k][m];
            if (i == k)
                L[i][k] = sum > 0.0 ? sqrt(sum) : 0.0;
            else
                L[i][k] = L[k][k] > 0.0 ? sum / L[k][k] : 0.0;
        }
}

static void multi_collide_site(const orc_multi *s, int64_t r, double fstar[ORC_MAX_SPECIES][QMAX])
{
    const int Q = s->Q, D = s->D, NS = s->N;
    const int64_t ns = s->nsites;
    const orc_multi_params *p = &s->p;

    double rho[ORC_MAX_SPECIES], jb[ORC_MAX_SPECIES][3], a[ORC_MAX_SPECIES][3], F[ORC_MAX_SPECIES][3];
    for (int sp = 0; sp < NS; ++sp) {
        rho[sp] = s->rho[(size_t)sp * ns + r];
        for (int al = 0; al < 3; ++al) jb[sp][al] = s->j[((size_t)sp * 3 + al) * ns + r];
    }
    multi_acceleration(s, r, a);
    for (int sp = 0; sp < NS; ++sp)
        for (int al = 0; al < 3; ++al) F[sp][al] = rho[sp] * a[sp][al];

    double rt = 0.0;
    for (int sp = 0; sp < NS; ++sp) rt += rho[sp];
    double u[3] = {0.0, 0.0, 0.0};
    if (rt > 0.0)
        for (int al = 0; al < D; ++al) {
            double jt = 0.0, Ft = 0.0;
            for (int sp = 0; sp < NS; ++sp) {
                jt += jb[sp][al];
                Ft += F[sp][al];
            }
            u[al] = jt / rt + 0.5 * (Ft / rt);
        }

    const int noisy = (p->kT > 0.0) && !(p->flags & ORC_NOISE_OFF);
    double z[KMAX];
    if (!noisy || orc_normals(p->seed, (uint32_t)r, s->step, s->K, z) != 0)
        for (int k = 0; k < s->K; ++k) z[k] = 0.0; /* K <= KMAX: checked by orc_multi_create */
    const double mu = 3.0 * p->kT;
    const double lam_d = 1.0 / p->tau_d;

    /* Momentum noise xi[sigma][alpha] with the covariance of App. D. */
    double xi[ORC_MAX_SPECIES][3];
    for (int sp = 0; sp < ORC_MAX_SPECIES; ++sp)
        for (int al = 0; al < 3; ++al) xi[sp][al] = 0.0;
    int all_positive = rt > 0.0;
    for (int sp = 0; sp < NS; ++sp) all_positive = all_positive && rho[sp] > 0.0;
    if (noisy && !(p->flags & ORC_NOISE_NO_SDF) && all_positive) {
        const double amp = (2.0 * lam_d - lam_d * lam_d) * p->kT;
        double Cv[ORC_MAX_SPECIES][ORC_MAX_SPECIES], L[ORC_MAX_SPECIES][ORC_MAX_SPECIES];
        for (int s1 = 0; s1 < NS - 1; ++s1)
            for (int s2 = 0; s2 < NS - 1; ++s2)
                Cv[s1][s2] = amp * ((s1 == s2 ? rho[s1] : 0.0) - rho[s1] * rho[s2] / rt);
        cholesky(NS - 1, Cv, L);
        for (int al = 0; al < D; ++al) {
            double total = 0.0;
            for (int sp = 0; sp < NS - 1; ++sp) {
                double v = 0.0;
                for (int k = 0; k <= sp; ++k) v += L[sp][k] * z[k * D + al];
                xi[sp][al] = v;
                total += v;
            }
            xi[NS - 1][al] = -total;
        }
    }

    for (int sp = 0; sp < NS; ++sp) {
        const double *fb[QMAX];
        for (int i = 0; i < Q; ++i) fb[i] = mpop(s, s->f, sp, i) + r;
        const double lam = 1.0 / p->tau[sp];

        double m[QMAX];
        for (int a_ = 0; a_ < Q; ++a_) {
            double acc = 0.0;
            for (int i = 0; i < Q; ++i) acc += s->T[a_][i] * (*fb[i]);
            m[a_] = acc;
        }
        double R[QMAX];
        R[0] = 0.0;
        for (int al = 0; al < D; ++al)
            R[1 + al] = lam_d * (rho[sp] * u[al] - m[1 + al]) + (1.0 - 0.5 * lam_d) * F[sp][al] + xi[sp][al];

        double v[3] = {0.0, 0.0, 0.0};
        if (rho[sp] > 0.0)
            for (int al = 0; al < D; ++al) v[al] = (m[1 + al] + 0.5 * R[1 + al]) / rho[sp];

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
        const int zbase = D * (NS - 1) + sp * (Q - D - 1);
        for (int a_ = D + 1; a_ < Q; ++a_) {
            double meq = 0.0, Phi = 0.0;
            for (int i = 0; i < Q; ++i) {
                meq += s->T[a_][i] * feq[i];
                Phi += s->T[a_][i] * phi[i];
            }
            double sig = 0.0;
            if (noisy && rho[sp] > 0.0) sig = sqrt((2.0 * lam - lam * lam) * s->Nn[a_] * mu * rho[sp]);
            R[a_] = lam * (meq - m[a_]) + (1.0 - 0.5 * lam) * Phi + sig * z[zbase + (a_ - D - 1)];
        }
        for (int i = 0; i < Q; ++i) {
            double acc = 0.0;
            for (int a_ = 0; a_ < Q; ++a_) acc += s->T[a_][i] * R[a_] / s->Nn[a_];
            fstar[sp][i] = *fb[i] + s->w[i] * acc;
        }
    }
}

int orc_multi_step(orc_multi *s, int64_t n)
{
    if (!s || n < 0) return -1;
    const int64_t ns = s->nsites;
    for (int64_t t = 0; t < n; ++t) {
        multi_pass1(s);
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < ns; ++r) {
            double fstar[ORC_MAX_SPECIES][QMAX];
            multi_collide_site(s, r, fstar);
            for (int sp = 0; sp < s->N; ++sp)
                for (int i = 0; i < s->Q; ++i) mpop(s, s->fnew, sp, i)[mneighbour(s, r, s->c[i])] = fstar[sp][i];
        }
        double *tmp = s->f;
        s->f = s->fnew;
        s->fnew = tmp;
        s->step += 1;
        s->moments_valid = 0;
    }
    return 0;
}

int orc_multi_collide_site(orc_multi *s, int64_t site, double *fstar)
{
    if (!s || !fstar || site < 0 || site >= s->nsites) return -1;
    if (!s->moments_valid) multi_pass1(s);
    double out[ORC_MAX_SPECIES][QMAX];
    multi_collide_site(s, site, out);
    for (int sp = 0; sp < s->N; ++sp)
        for (int i = 0; i < s->Q; ++i) fstar[(size_t)sp * s->Q + i] = out[sp][i];
    return 0;
}

int orc_multi_moments(orc_multi *s, double *rho, double *j, double *F)
{
    if (!s) return -1;
    multi_pass1(s);
    const int64_t ns = s->nsites;
    const int D = s->D;
    for (int64_t r = 0; r < ns; ++r) {
        double a[ORC_MAX_SPECIES][3];
        if (F) multi_acceleration(s, r, a);
        for (int sp = 0; sp < s->N; ++sp) {
            const double rs = s->rho[(size_t)sp * ns + r];
            if (rho) rho[(size_t)sp * ns + r] = rs;
            for (int al = 0; al < D; ++al) {
                if (j) j[((size_t)sp * D + al) * ns + r] = s->j[((size_t)sp * 3 + al) * ns + r];
                if (F) F[((size_t)sp * D + al) * ns + r] = rs * a[sp][al];
            }
        }
    }
    return 0;
}
