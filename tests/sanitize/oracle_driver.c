/* Runs every entry point of the CPU oracle on small inputs, edge cases and
 * invalid arguments, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exit status 0 when
 * every call returns what it should; the sanitizers abort on any error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fft1d(int n, int sign, const double *in, double *out);
int oracle_fft3d(const int dims[3], int sign, const double *in, double *out);
int oracle_kernel(const double cell[9], const int dims[3], double *K);
int oracle_poisson(const double cell[9], const int dims[3], const double *rho, double *V, double *eh_real,
                   double *eh_recip, double *max_imag);
int oracle_backward(const double cell[9], const int dims[3], const double *grad_v, double grad_e, const double *rho,
                    double *grad_rho);
int oracle_splat(const double cell[9], const int dims[3], int natoms, const double *pos, const double *Z,
                 const double *sigma, double cutoff, int subtract_background, double *rho);
int oracle_splat_points(const double cell[9], const int dims[3], int natoms, const double *pos, const double *Z,
                        const double *sigma, double cutoff, int subtract_background, int npts, const int64_t *idx,
                        double *out);
int oracle_splat_adjoint(const double cell[9], const int dims[3], int natoms, const double *pos, const double *Z,
                         const double *sigma, double cutoff, const double *grad_rho, int nsel, const int *sel,
                         double *grad_pos);

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                            \
        }                                                          \
    } while (0)

static double urand(unsigned *s)
{
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xFFFFFF) / 16777216.0;
}

int main(void)
{
    unsigned seed = 1209;
    /* 1-D transforms: prime, smooth and length-1 */
    const int lens[] = {1, 2, 7, 11, 12, 60, 97};
    for (size_t t = 0; t < sizeof(lens) / sizeof(lens[0]); ++t) {
        const int n = lens[t];
        double *x = malloc(sizeof(double) * 2 * n), *y = malloc(sizeof(double) * 2 * n);
        for (int i = 0; i < 2 * n; ++i) x[i] = urand(&seed) - 0.5;
        CHECK(oracle_fft1d(n, -1, x, y) == 0);
        CHECK(oracle_fft1d(n, +1, y, x) == 0);
        free(x);
        free(y);
    }
    CHECK(oracle_fft1d(0, -1, NULL, NULL) != 0);

    const double cells[2][9] = {{9.0, 0, 0, 0, 8.5, 0, 0, 0, 10.0}, {9.0, 0, 0, 2.5, 8.0, 0, -1.5, 2.0, 10.5}};
    const int dimsets[4][3] = {{1, 1, 1}, {6, 5, 7}, {8, 12, 10}, {1, 9, 4}};
    for (int c = 0; c < 2; ++c)
        for (int ds = 0; ds < 4; ++ds) {
            const int *dims = dimsets[ds];
            const int n = dims[0] * dims[1] * dims[2];
            double *a = malloc(sizeof(double) * 2 * n), *b = malloc(sizeof(double) * 2 * n);
            double *rho = malloc(sizeof(double) * n), *V = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n);
            double *K = malloc(sizeof(double) * n);
            for (int i = 0; i < 2 * n; ++i) a[i] = urand(&seed) - 0.5;
            for (int i = 0; i < n; ++i) rho[i] = urand(&seed) - 0.5;
            CHECK(oracle_fft3d(dims, -1, a, b) == 0);
            CHECK(oracle_kernel(cells[c], dims, K) == 0);
            double er = 0, eg = 0, mi = 0;
            CHECK(oracle_poisson(cells[c], dims, rho, V, &er, &eg, &mi) == 0);
            CHECK(oracle_backward(cells[c], dims, V, 0.7, rho, g) == 0);
            CHECK(oracle_backward(cells[c], dims, NULL, 0.7, rho, g) == 0);
            CHECK(oracle_backward(cells[c], dims, V, 0.0, NULL, g) == 0);
            /* atoms, some outside the cell, one with a wide Gaussian */
            const int na = 5;
            double pos[15], Z[5], sig[5], gp[15];
            for (int i = 0; i < na; ++i) {
                for (int x = 0; x < 3; ++x) pos[3 * i + x] = 30.0 * urand(&seed) - 10.0;
                Z[i] = 1.0 + 3.0 * urand(&seed);
                sig[i] = i == 0 ? 2.5 : 0.6 + 0.4 * urand(&seed);
            }
            CHECK(oracle_splat(cells[c], dims, na, pos, Z, sig, 6.0, 1, rho) == 0);
            CHECK(oracle_splat(cells[c], dims, 0, NULL, NULL, NULL, 6.0, 1, rho) == 0);
            int64_t idx[3] = {0, n / 2, n - 1};
            double pts[3];
            CHECK(oracle_splat_points(cells[c], dims, na, pos, Z, sig, 6.0, 0, 3, idx, pts) == 0);
            CHECK(oracle_splat_adjoint(cells[c], dims, na, pos, Z, sig, 6.0, V, 0, NULL, gp) == 0);
            int sel[2] = {4, 1};
            CHECK(oracle_splat_adjoint(cells[c], dims, na, pos, Z, sig, 6.0, V, 2, sel, gp) == 0);
            free(a);
            free(b);
            free(rho);
            free(V);
            free(g);
            free(K);
        }
    /* rejected arguments: bad dims, a singular cell, bad atoms */
    const int bad_dims[3] = {0, 4, 4}, dims4[3] = {4, 4, 4};
    const double singular[9] = {1, 0, 0, 2, 0, 0, 0, 0, 1};
    double rho[64], V[64], e1, e2, e3;
    for (int i = 0; i < 64; ++i) rho[i] = 0.1 * i;
    CHECK(oracle_poisson(cells[0], bad_dims, rho, V, &e1, &e2, &e3) != 0);
    CHECK(oracle_poisson(singular, dims4, rho, V, &e1, &e2, &e3) != 0);
    double pos[3] = {NAN, 0, 0}, Z[1] = {1.0}, sig[1] = {1.0};
    CHECK(oracle_splat(cells[0], dims4, 1, pos, Z, sig, 6.0, 1, rho) != 0);
    sig[0] = -1.0;
    pos[0] = 0.0;
    CHECK(oracle_splat(cells[0], dims4, 1, pos, Z, sig, 6.0, 1, rho) != 0);
    if (failures) return 1;
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
