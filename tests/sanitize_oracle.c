/*
 * Drives every entry point of the C oracle (oracle/flbe_oracle.c,
 * oracle/flbe_multi.c) over the cases with the most normals per site and the
 * largest per-site arrays, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exit status 0 when
 * every call returned what it should; the sanitizers abort on any invalid
 * access or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/flbe_oracle.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                                    \
        }                                                               \
    } while (0)

static double *perturbed(int64_t n, double base, unsigned seed)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        seed = seed * 1664525u + 1013904223u;
        r[k] = base * (1.0 + 0.05 * ((double)(seed >> 8) / 16777216.0 - 0.5));
    }
    return r;
}

static void binary_case(int lattice, int nx, int ny, int nz)
{
    orc_params p = {lattice, nx, ny, nz, {0.8, 1.3}, 0.9, 0.7, 1e-4, 12345u, 0u};
    orc_sim *s = orc_create(&p);
    CHECK(s);
    const int64_t n = orc_num_sites(s);
    const int Q = lattice == ORC_D2Q9 ? 9 : 19, D = lattice == ORC_D2Q9 ? 2 : 3;
    double *r1 = perturbed(n, 1.0, 1u), *r2 = perturbed(n, 0.9, 2u);
    CHECK(orc_init_density(s, r1, r2) == 0);
    CHECK(orc_step(s, 3) == 0);
    double *f = (double *)malloc(sizeof(double) * 2 * Q * (size_t)n);
    double *rho = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    double *j = (double *)malloc(sizeof(double) * 2 * D * (size_t)n);
    double *F = (double *)malloc(sizeof(double) * 2 * D * (size_t)n);
    CHECK(orc_get_populations(s, f) == 0);
    CHECK(orc_moments(s, rho, j, F) == 0);
    CHECK(orc_moments(s, NULL, NULL, NULL) == 0);
    double fstar[2 * 19];
    for (int64_t r = 0; r < n; ++r) CHECK(orc_collide_site(s, r, fstar) == 0);
    CHECK(orc_collide_site(s, -1, fstar) == -1);
    CHECK(orc_collide_site(s, n, fstar) == -1);
    int64_t counts[2];
    CHECK(orc_health(s, counts) == 0 && counts[0] == 0 && counts[1] == 0);
    f[0] = NAN;
    CHECK(orc_set_populations(s, f, 7) == 0);
    CHECK(orc_health(s, counts) == 0 && counts[1] == 1);
    CHECK(orc_current_step(s) == 7);
    free(f);
    free(rho);
    free(j);
    free(F);
    free(r1);
    free(r2);
    orc_destroy(s);
}

static void multi_case(int lattice, int N, int nx, int ny, int nz)
{
    orc_multi_params p = {lattice, N, nx, ny, nz, {0.8, 1.1, 1.3, 0.95}, 0.9, {{0}}, 1e-4, 99u, 0u};
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) p.G[a][b] = a == b ? 0.0 : 0.1 * (1 + a + b);
    orc_multi *s = orc_multi_create(&p);
    CHECK(s);
    const int64_t n = (int64_t)nx * ny * nz;
    const int Q = lattice == ORC_D2Q9 ? 9 : 19, D = lattice == ORC_D2Q9 ? 2 : 3;
    double *rho0 = (double *)malloc(sizeof(double) * N * (size_t)n);
    for (int sp = 0; sp < N; ++sp) {
        double *r = perturbed(n, 1.0 - 0.1 * sp, 3u + sp);
        for (int64_t k = 0; k < n; ++k) rho0[(size_t)sp * n + k] = r[k];
        free(r);
    }
    CHECK(orc_multi_init_density(s, rho0) == 0);
    CHECK(orc_multi_step(s, 3) == 0);
    double *f = (double *)malloc(sizeof(double) * N * Q * (size_t)n);
    double *rho = (double *)malloc(sizeof(double) * N * (size_t)n);
    double *j = (double *)malloc(sizeof(double) * N * D * (size_t)n);
    double *F = (double *)malloc(sizeof(double) * N * D * (size_t)n);
    CHECK(orc_multi_get_populations(s, f) == 0);
    CHECK(orc_multi_set_populations(s, f, 3) == 0);
    CHECK(orc_multi_moments(s, rho, j, F) == 0);
    double fstar[ORC_MAX_SPECIES * 19];
    for (int64_t r = 0; r < n; ++r) CHECK(orc_multi_collide_site(s, r, fstar) == 0);
    CHECK(orc_multi_collide_site(s, n, fstar) != 0);
    CHECK(orc_multi_current_step(s) == 3);
    free(f);
    free(rho);
    free(j);
    free(F);
    free(rho0);
    orc_multi_destroy(s);
}

int main(void)
{
    /* Normals: every count up to the bound, and the bound itself enforced. */
    double z[ORC_MAX_NORMALS];
    for (int K = 0; K <= ORC_MAX_NORMALS; ++K) CHECK(orc_normals(5u, 3u, 11, K, z) == 0);
    CHECK(orc_normals(5u, 3u, 11, ORC_MAX_NORMALS + 1, z) == -1);
    CHECK(orc_normals(5u, 3u, 11, -1, z) == -1);
    for (int k = 0; k < ORC_MAX_NORMALS; ++k) CHECK(isfinite(z[k]));
    double u[2 * ORC_MAX_NORMALS];
    orc_uniforms(5u, 3u, 11, 2 * ORC_MAX_NORMALS, u);

    /* Basis of both lattices and an unknown one. */
    int D, c[19 * 3];
    double w[19], T[19 * 19], Nn[19];
    CHECK(orc_basis(ORC_D2Q9, &D, c, w, T, Nn) == 9 && D == 2);
    CHECK(orc_basis(ORC_D3Q19, &D, c, w, T, Nn) == 19 && D == 3);
    CHECK(orc_basis(7, &D, c, w, T, Nn) == -1);

    /* Invalid parameters are rejected. */
    orc_params bad = {ORC_D2Q9, 4, 4, 2, {1.0, 1.0}, 1.0, 0.0, 0.0, 1u, 0u};
    CHECK(orc_create(&bad) == NULL);
    orc_multi_params mbad = {ORC_D2Q9, ORC_MAX_SPECIES + 1, 4, 4, 1, {1, 1, 1, 1}, 1.0, {{0}}, 0.0, 1u, 0u};
    CHECK(orc_multi_create(&mbad) == NULL);

    binary_case(ORC_D2Q9, 7, 5, 1);
    binary_case(ORC_D3Q19, 5, 4, 3);
    binary_case(ORC_D3Q19, 1, 1, 1);
    multi_case(ORC_D2Q9, 3, 6, 5, 1);
    multi_case(ORC_D3Q19, ORC_MAX_SPECIES, 4, 3, 3); /* 69 normals per site */
    multi_case(ORC_D3Q19, 2, 1, 1, 1);
    printf("sanitized oracle run: ok\n");
    return 0;
}
