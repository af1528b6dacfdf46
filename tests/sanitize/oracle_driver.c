/* Runs the FP64 oracle's entry points on small inputs, edge cases included,
 * under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).  Exit 0
 * when every call returns what it should; a sanitizer report aborts. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_basis(double t, double b[4], double db[4], double d2b[4]);
void oracle_reduce(double r, double cell, int32_t n, int32_t *i, double *t);
int oracle_eval_vgl(const int32_t n[3], const double cell[3], int32_t norb, const double *coefs, int64_t B,
                    const double *pos, double *V, double *G, double *L, int32_t nthreads);
int oracle_eval_v(const int32_t n[3], const double cell[3], int32_t norb, const double *coefs, int64_t B,
                  const double *pos, double *V, int32_t nthreads);
double oracle_round_sig(double x, int32_t p, int32_t emin);
int oracle_dequantize(const double *coefs, int64_t npts, int32_t norb, int32_t fmt, double *out, double *scales);
int oracle_eval_vgh(const int32_t n[3], const double lat[9], int32_t norb, const double *coefs, int64_t B,
                    const double *pos, double *V, double *G, double *H, int32_t nthreads);

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++fails; } } while (0)

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0;
}

int main(void)
{
    uint64_t seed = 12345;
    double b[4], db[4], d2b[4];
    for (int k = 0; k <= 8; ++k) {
        oracle_basis(k / 8.0, b, db, d2b);
        CHECK(fabs(b[0] + b[1] + b[2] + b[3] - 1.0) < 1e-15);
    }
    int32_t i;
    double t;
    const double rs[] = {0.0, -0.0, 1.0, -1e-17, 1e6, 0.999999999999, -3.5, NAN, INFINITY, -INFINITY};
    for (size_t k = 0; k < sizeof(rs) / sizeof(rs[0]); ++k) {
        oracle_reduce(rs[k], 1.0, 7, &i, &t);
        CHECK(i >= 0 && i < 7);
    }
    /* tables of several shapes, orbitals and storage formats */
    const int32_t grids[][3] = {{1, 1, 1}, {2, 3, 1}, {5, 4, 6}, {7, 7, 7}};
    const int32_t norbs[] = {1, 3, 17};
    for (int g = 0; g < 4; ++g)
        for (int o = 0; o < 3; ++o) {
            const int32_t *n = grids[g];
            const int32_t N = norbs[o];
            const int64_t npts = (int64_t)n[0] * n[1] * n[2];
            const int64_t B = 37;
            double *c = malloc(sizeof(double) * npts * N), *dq = malloc(sizeof(double) * npts * N);
            double *sc = malloc(sizeof(double) * N), *pos = malloc(sizeof(double) * B * 3);
            double *V = malloc(sizeof(double) * B * N), *G = malloc(sizeof(double) * B * 3 * N);
            double *L = malloc(sizeof(double) * B * N), *H = malloc(sizeof(double) * B * 6 * N);
            for (int64_t e = 0; e < npts * N; ++e) c[e] = 2 * urand(&seed) - 1;
            for (int64_t e = 0; e < B * 3; ++e) pos[e] = 6 * urand(&seed) - 3;
            pos[4] = NAN;
            pos[9] = INFINITY;
            const double cell[3] = {1.0, 1.3, 0.7};
            const double lat[9] = {1.0, 0.0, 0.0, -0.5, 0.8660254037844386, 0.0, 0.0, 0.0, 1.6};
            CHECK(oracle_eval_vgl(n, cell, N, c, B, pos, V, G, L, 2) == 0);
            CHECK(oracle_eval_v(n, cell, N, c, B, pos, V, 1) == 0);
            CHECK(oracle_eval_vgh(n, lat, N, c, B, pos, V, G, H, 2) == 0);
            for (int fmt = 0; fmt < 4; ++fmt) CHECK(oracle_dequantize(c, npts, N, fmt, dq, sc) == 0);
            CHECK(oracle_eval_vgl(n, cell, N, c, 0, pos, V, G, L, 1) == 0);
            free(c); free(dq); free(sc); free(pos); free(V); free(G); free(L); free(H);
        }
    /* argument errors */
    const int32_t bad[3] = {0, 4, 4};
    double one = 1.0, out = 0.0, cell[3] = {1, 1, 1};
    CHECK(oracle_eval_vgl(bad, cell, 1, &one, 1, cell, &out, &out, &out, 1) == -1);
    const double sing[9] = {1, 0, 0, 2, 0, 0, 0, 0, 1};
    const int32_t n4[3] = {4, 4, 4};
    CHECK(oracle_eval_vgh(n4, sing, 1, &one, 0, cell, &out, &out, &out, 1) == -1);
    CHECK(oracle_dequantize(&one, 1, 1, 7, &out, &out) == -1);
    /* rounding at the edges of both 16-bit formats */
    const double xs[] = {0.0, 1.0, 65504.0, 65520.0, 6e-8, 1e-40, 3.3895e38, -1.0 / 3.0};
    for (size_t k = 0; k < sizeof(xs) / sizeof(xs[0]); ++k) {
        (void)oracle_round_sig(xs[k], 8, -126);
        (void)oracle_round_sig(xs[k], 11, -14);
    }
    printf("oracle driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
