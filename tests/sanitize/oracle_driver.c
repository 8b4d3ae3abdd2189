/* Driver of the FP64 oracle (oracle/oracle.c, included here) for sanitizer
 * builds (AddressSanitizer, UndefinedBehaviorSanitizer): geometry, links,
 * percolation, fixed steps and steady solves of both solvers in 2-D and
 * 3-D, the stop rule, and a short coupled loop.  Prints "ok" and exits 0
 * when every call behaved. */
#include "oracle.c"

#include <stdio.h>

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(1);                                                      \
        }                                                                 \
    } while (0)

static void grid_2d(int nx, int ny, uint64_t seed)
{
    const int64_t N = (int64_t)nx * ny;
    uint8_t *cls = malloc(N), *dom = malloc(N);
    double frac;
    CHECK(orc_geom_discs(nx, ny, 2, 3, 0.2, (int)(seed & 1), seed, cls, &frac) == ORC_OK);
    CHECK(orc_biofilm_layer(nx, ny, 1, cls) == ORC_OK);
    uint32_t *lk = malloc(N * sizeof(uint32_t));
    CHECK(orc_links(nx, ny, 1, cls, 0, lk) == ORC_OK);
    CHECK(orc_links(nx, ny, 1, cls, 1, lk) == ORC_OK);
    CHECK(orc_flow_domain(nx, ny, 1, cls, dom) == ORC_OK);
    if (orc_percolates(nx, ny, 1, cls)) {
        double *f = malloc(9 * N * sizeof(double)), *U = malloc(2 * N * sizeof(double));
        double *g = malloc(5 * N * sizeof(double)), *C = malloc(N * sizeof(double));
        double *rho = malloc(N * sizeof(double));
        int64_t it;
        double res, a, b, s;
        CHECK(orc_fluid_init(ORC_D2Q9, nx, ny, 1, cls, f) == ORC_OK);
        int st = orc_fluid_solve(ORC_D2Q9, nx, ny, 1, cls, 0.8, 0.01, 1e-4, 400, 10, 20, f, U, &it, &res);
        CHECK(st >= 0);
        CHECK(orc_fluid_moments(ORC_D2Q9, nx, ny, 1, cls, NULL, f, U, rho) == ORC_OK);
        CHECK(orc_fluid_fluxes(ORC_D2Q9, nx, ny, 1, cls, 0.01, f, &a, &b) == ORC_OK);
        CHECK(orc_ad_init(ORC_D2Q5, nx, ny, 1, cls, 1.0, U, g) == ORC_OK);
        st = orc_ad_solve(ORC_D2Q5, nx, ny, 1, cls, U, 0.05, 1.0, 1e-3, 0.0, 0, 0.0, 1e-4, 400, 10, 20, g, C,
                          &it, &res);
        CHECK(st >= 0);
        CHECK(orc_ad_fluxes(ORC_D2Q5, nx, ny, 1, cls, 1.0, 1e-3, 0.0, 1, 0.5, U, g, &a, &b, &s) == ORC_OK);
        CHECK(orc_ad_run(ORC_D2Q5, nx, ny, 1, cls, 0.05, 1.0, 1e-3, 0.5, 1, 0.25, NULL, U, 5, g, C) == ORC_OK);
        double *g9 = malloc(9 * N * sizeof(double));
        CHECK(orc_ad_init(ORC_D2Q9, nx, ny, 1, cls, 1.0, U, g9) == ORC_OK);
        CHECK(orc_ad_run(ORC_D2Q9, nx, ny, 1, cls, 0.05, 1.0, 1e-3, 0.0, 0, 0.0, NULL, U, 5, g9, C) == ORC_OK);
        (void)orc_growth_pick(nx, ny, 1, cls, C, 0.5);
        free(g9);
        free(f);
        free(U);
        free(g);
        free(C);
        free(rho);
    }
    free(lk);
    free(cls);
    free(dom);
}

int main(void)
{
    grid_2d(48, 20, 3);
    grid_2d(37, 11, 4);
    /* 3-D */
    {
        const int nx = 24, ny = 12, nz = 10;
        const int64_t N = (int64_t)nx * ny * nz;
        uint8_t *cls = malloc(N);
        double frac;
        CHECK(orc_geom_fibres(nx, ny, nz, 1, 2, 0.2, 5, cls, &frac) == ORC_OK);
        CHECK(orc_biofilm_layer(nx, ny, nz, cls) == ORC_OK);
        double *f = malloc(19 * N * sizeof(double)), *U = malloc(3 * N * sizeof(double));
        double *g = malloc(7 * N * sizeof(double)), *C = malloc(N * sizeof(double));
        CHECK(orc_fluid_init(ORC_D3Q19, nx, ny, nz, cls, f) == ORC_OK);
        CHECK(orc_fluid_run(ORC_D3Q19, nx, ny, nz, cls, 0.7, 0.01, NULL, NULL, 20, f, U, NULL) == ORC_OK);
        CHECK(orc_ad_init(ORC_D3Q7, nx, ny, nz, cls, 1.0, U, g) == ORC_OK);
        CHECK(orc_ad_run(ORC_D3Q7, nx, ny, nz, cls, 0.0375, 1.0, 1e-3, 0.0, 0, 0.0, NULL, U, 20, g, C) == ORC_OK);
        free(f);
        free(U);
        free(g);
        free(C);
        free(cls);
    }
    /* stop rule and a short coupled loop */
    {
        double r[6] = {5, 4, 3, 3, 3, 3};
        int at;
        CHECK(orc_stall_rule(r, NULL, 6, 1e-6, 3, &at) == ORC_STALLED && at == 5);
        const int nx = 48, ny = 20;
        const int64_t N = (int64_t)nx * ny;
        uint8_t *cls = malloc(N);
        double frac;
        CHECK(orc_geom_discs(nx, ny, 2, 3, 0.2, 0, 7, cls, &frac) == ORC_OK);
        CHECK(orc_biofilm_layer(nx, ny, 1, cls) == ORC_OK);
        double xi[3] = {0.1, 0.5, 0.9}, J[4], acc, *U = malloc(2 * N * sizeof(double));
        double *C = malloc(N * sizeof(double));
        int64_t picked[3], itf[4], ita[4];
        int st = orc_coupled_run(nx, ny, 1, cls, 0.8, 0.01, 0.05, 1.0, 1e-3, 0.0, -1, 1e-3, 400, 100, 1000, 3,
                                 xi, picked, J, &acc, itf, ita, U, C);
        CHECK(st == ORC_OK || st == ORC_EINVAL);
        free(U);
        free(C);
        free(cls);
    }
    printf("ok\n");
    return 0;
}
