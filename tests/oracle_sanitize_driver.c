/*
 * Drives every entry point of the FP64 oracle (oracle/mech_oracle.c) on small
 * seeded populations, edge cases and error paths, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only; compiled
 * and run by tests/test_oracle_sanitized.py).  Any out-of-bounds access, leak
 * or undefined operation aborts the run; otherwise it prints "all ok".
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_geometry(int64_t, const double *, const double *, const double *, const double *, double,
                 double *, double *, int64_t *, int64_t *);
int orc_grid(int64_t, const double *, const double *, const double *, const double *, double,
             int32_t *, int32_t *, int32_t *);
int orc_neighbors(int64_t, const double *, const double *, const double *, const double *, double,
                  int32_t *, int64_t *, int32_t *, int64_t);
int orc_brute_neighbors(int64_t, const double *, const double *, const double *, double, int32_t *,
                        int64_t *, int32_t *, int64_t);
int orc_step(int64_t, const double *, const double *, const double *, const double *, double,
             const double *, double *, double *, double *, double *, double *, double *);
int orc_brute_forces(int64_t, const double *, const double *, const double *, const double *, double,
                     double, double *, double *, double *);
int orc_tolerance_scales(int64_t, const double *, const double *, const double *, const double *,
                         double, double, double, double, double *, double *, int32_t *);
int orc_sample(int64_t, const double *, const double *, const double *, const double *, double,
               const double *, double, int64_t, const int64_t *, double *, double *, double *,
               double *, double *, double *, double *, double *, int32_t *);
int orc_step_adjoint(int64_t, const double *, const double *, const double *, const double *, double,
                     const double *, const double *, const double *, const double *, double *,
                     double *, double *, double *, double *);
int orc_adjoint_scales(int64_t, const double *, const double *, const double *, const double *,
                       double, const double *, const double *, const double *, const double *,
                       double, double *, double *, double *, double *, double *);
int orc_integrate(int64_t, double *, double *, double *, const double *, const double *,
                  const double *);
int orc_set_threads(int);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)   /* xorshift64, uniform in [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define EXPECT(c)                                                      \
    do {                                                               \
        if (!(c)) { fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); ++fails; } \
    } while (0)

static void exercise(int64_t n, const double *x, const double *y, const double *z, const double *d)
{
    const double P[5] = {2.0, 1.0, 0.05, 0.02, 0.0};
    double o[3], e;
    int64_t dims[3], nb;
    EXPECT(orc_geometry(n, x, y, z, d, 0.0, o, &e, dims, &nb) == 0);
    int32_t *box = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *start = malloc(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t *perm = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    EXPECT(orc_grid(n, x, y, z, d, 0.0, box, start, perm) == 0);
    int32_t *cnt = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    EXPECT(orc_neighbors(n, x, y, z, d, 0.0, cnt, off, NULL, 0) == 0);
    int64_t tot = off[n];
    int32_t *lst = malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    EXPECT(orc_neighbors(n, x, y, z, d, 0.0, cnt, off, lst, tot) == 0);
    if (tot > 0) EXPECT(orc_neighbors(n, x, y, z, d, 0.0, cnt, off, lst, tot - 1) == 2);
    EXPECT(orc_brute_neighbors(n, x, y, z, e, cnt, off, lst, tot) == 0);
    if (tot > 0) EXPECT(orc_brute_neighbors(n, x, y, z, e, cnt, off, lst, tot - 1) == 2);
    size_t nn = (size_t)(n ? n : 1);
    double *a[12];
    for (int k = 0; k < 12; ++k) a[k] = calloc(nn, sizeof(double));
    EXPECT(orc_step(n, x, y, z, d, 0.0, P, a[0], a[1], a[2], a[3], a[4], a[5]) == 0);
    EXPECT(orc_step(n, x, y, z, d, 0.0, P, NULL, NULL, NULL, a[3], a[4], a[5]) == 0);
    EXPECT(orc_brute_forces(n, x, y, z, d, 2.0, 1.0, a[0], a[1], a[2]) == 0);
    int32_t *c = malloc(sizeof(int32_t) * nn);
    EXPECT(orc_tolerance_scales(n, x, y, z, d, 0.0, 2.0, 1.0, 0x1p-24, a[6], a[7], c) == 0);
    int64_t idx[5] = {0, n - 1, n / 2, 0, n / 3};
    double sm[9][5];
    int32_t sc[5];
    if (n > 0) {
        EXPECT(orc_sample(n, x, y, z, d, 0.0, P, 0x1p-24, 5, idx, sm[0], sm[1], sm[2], sm[3], sm[4],
                          sm[5], sm[6], sm[7], sc) == 0);
        int64_t bad = n;
        EXPECT(orc_sample(n, x, y, z, d, 0.0, P, 0x1p-24, 1, &bad, sm[0], NULL, NULL, NULL, NULL,
                          NULL, NULL, NULL, NULL) == 1);
    }
    for (int64_t i = 0; i < n; ++i) { a[8][i] = urand() - 0.5; a[9][i] = urand() - 0.5; a[10][i] = urand(); }
    double gkg[2], skg[4];
    double *g3[4];
    for (int k = 0; k < 4; ++k) g3[k] = calloc(nn, sizeof(double));
    EXPECT(orc_step_adjoint(n, x, y, z, d, 0.0, P, a[8], a[9], a[10], g3[0], g3[1], g3[2], g3[3],
                            gkg) == 0);
    EXPECT(orc_adjoint_scales(n, x, y, z, d, 0.0, P, a[8], a[9], a[10], 0x1p-53, g3[0], g3[1],
                              g3[2], g3[3], skg) == 0);
    double *px = malloc(sizeof(double) * nn), *py = malloc(sizeof(double) * nn),
           *pz = malloc(sizeof(double) * nn);
    memcpy(px, x, sizeof(double) * (size_t)n);
    memcpy(py, y, sizeof(double) * (size_t)n);
    memcpy(pz, z, sizeof(double) * (size_t)n);
    EXPECT(orc_integrate(n, px, py, pz, a[3], a[4], a[5]) == 0);
    free(px); free(py); free(pz);
    for (int k = 0; k < 4; ++k) free(g3[k]);
    for (int k = 0; k < 12; ++k) free(a[k]);
    free(c); free(lst); free(off); free(cnt); free(perm); free(start); free(box);
}

int main(void)
{
    const int64_t N = 700;
    double *x = malloc(sizeof(double) * N), *y = malloc(sizeof(double) * N),
           *z = malloc(sizeof(double) * N), *d = malloc(sizeof(double) * N);
    for (int t = 1; t <= 2; ++t) {
        orc_set_threads(t == 1 ? 1 : 4);
        /* uniform cube at ~20 neighbours */
        for (int64_t i = 0; i < N; ++i) {
            x[i] = 110.0 * urand(); y[i] = 110.0 * urand(); z[i] = 110.0 * urand();
            d[i] = 8.0 + 4.0 * urand();
        }
        exercise(N, x, y, z, d);
        /* everything in one box, with exact duplicates (coincident centres) */
        for (int64_t i = 0; i < N; ++i) {
            x[i] = 3.0 * urand(); y[i] = (i % 7 == 0) ? 0.0 : 3.0 * urand(); z[i] = 0.5;
            if (i % 11 == 0 && i > 0) { x[i] = x[i - 1]; y[i] = y[i - 1]; }
        }
        exercise(N, x, y, z, d);
        /* collinear, two agents, one agent, none */
        for (int64_t i = 0; i < N; ++i) { x[i] = 9.0 * (double)i; y[i] = z[i] = 0.0; d[i] = 10.0; }
        exercise(N, x, y, z, d);
        exercise(2, x, y, z, d);
        exercise(1, x, y, z, d);
        exercise(0, x, y, z, d);
    }
    /* error paths */
    const double P[5] = {2.0, 1.0, 0.01, 3.0, 0.0};
    const double Pbad[5] = {2.0, 1.0, -0.01, 3.0, 0.0};
    double o[3], e, f[6];
    int64_t dims[3], nb;
    double xs[2] = {0.0, 9.0}, zs[2] = {0.0, 0.0}, ds[2] = {10.0, 10.0};
    EXPECT(orc_geometry(2, xs, zs, zs, ds, 5.0, o, &e, dims, &nb) == 1);
    EXPECT(orc_step(2, xs, zs, zs, ds, 0.0, Pbad, f, f + 1, f + 2, NULL, NULL, NULL) == 1);
    double nan_x[2] = {0.0, 0.0 / 0.0};
    EXPECT(orc_step(2, nan_x, zs, zs, ds, 0.0, P, NULL, NULL, NULL, NULL, NULL, NULL) == 4);
    double far_x[2] = {0.0, 1e300};
    EXPECT(orc_geometry(2, far_x, zs, zs, ds, 0.0, o, &e, dims, &nb) == 2);
    free(x); free(y); free(z); free(d);
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("all ok\n");
    return 0;
}
