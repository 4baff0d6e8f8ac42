/*
 * Driver for the sanitizer run of the oracle (tests/test_oracle_sanitize.py):
 * calls every entry point of oracle/oracle.c on small inputs, built together
 * with it under AddressSanitizer and UndefinedBehaviorSanitizer, and checks
 * the results against each other.  Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_matern_profile(int two_nu, double r);
double oracle_kernel(int d, const double *a, const double *b, int two_nu, int form, double ell, double s2);
int oracle_mvm(int64_t n, int d, const double *x, int64_t ldx, int64_t m, const double *z, int64_t ldz,
               int two_nu, int form, double ell, double s2, const double *v, int64_t ldv, int nrhs,
               double *y, int64_t ldy, double *yabs);
int oracle_mvm_multi(int64_t n, int d, const double *x, int64_t ldx, int64_t m, const double *z, int64_t ldz,
                     int two_nu, int form, double ell, double s2, const double *v, int64_t ldv, int nrhs,
                     double *y, int64_t ldy, double *yabs);
int oracle_kernel_matrix(int64_t n, int d, const double *x, int64_t ldx, int64_t m, const double *z,
                         int64_t ldz, int two_nu, int form, double ell, double s2, double diag, int add_diag,
                         double *kmat, int64_t ldk);
int oracle_cholesky(int64_t n, double *a, int64_t lda);
int oracle_cholesky_solve(int64_t n, const double *l, int64_t ldl, double *b, int64_t ldb, int nrhs);
int oracle_num_threads(void);
int oracle_profile_array(int two_nu, int64_t n, const double *r, double *out);

static uint64_t state = 88172645463325252ull;
static double uniform(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
static void expect(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++fails;
    }
}

int main(void)
{
    enum { N = 37, M = 29, R = 3 };
    for (int d = 1; d <= 3; ++d)
        for (int two_nu = 1; two_nu <= 5; two_nu += 2)
            for (int form = 0; form <= 1; ++form) {
                double *x = malloc(sizeof(double) * N * d), *z = malloc(sizeof(double) * M * d);
                double *v = malloc(sizeof(double) * N * R);
                double *y1 = malloc(sizeof(double) * M * R), *y2 = malloc(sizeof(double) * M * R);
                double *ya = malloc(sizeof(double) * M * R), *yb = malloc(sizeof(double) * M * R);
                for (int i = 0; i < N * d; ++i) x[i] = uniform();
                for (int i = 0; i < M * d; ++i) z[i] = uniform();
                for (int i = 0; i < N * R; ++i) v[i] = 2.0 * uniform() - 1.0;
                expect(oracle_mvm(N, d, x, N, M, z, M, two_nu, form, 0.3, 1.5, v, N, R, y1, M, ya) == 0, "mvm");
                expect(oracle_mvm_multi(N, d, x, N, M, z, M, two_nu, form, 0.3, 1.5, v, N, R, y2, M, yb) == 0,
                       "mvm_multi");
                for (int i = 0; i < M * R; ++i) {
                    expect(fabs(y1[i] - y2[i]) <= 1e-14 * ya[i], "mvm and mvm_multi agree");
                    expect(fabs(y1[i]) <= ya[i] * (1.0 + 1e-15), "|y| <= K|v|");
                }
                /* one row by hand from the scalar kernel */
                double pt[3], ref = 0.0;
                for (int k = 0; k < d; ++k) pt[k] = z[k * M];
                for (int i = 0; i < N; ++i) {
                    double xi[3];
                    for (int k = 0; k < d; ++k) xi[k] = x[k * N + i];
                    ref += oracle_kernel(d, pt, xi, two_nu, form, 0.3, 1.5) * v[i];
                }
                expect(fabs(ref - y1[0]) <= 1e-13 * ya[0], "row 0 by the scalar kernel");
                free(x); free(z); free(v); free(y1); free(y2); free(ya); free(yb);
            }
    /* Cholesky solve of K + sigma2 I (product form, d = 2) */
    {
        enum { n = 40 };
        double *x = malloc(sizeof(double) * n * 2), *a = malloc(sizeof(double) * n * n);
        double *k0 = malloc(sizeof(double) * n * n), *b = malloc(sizeof(double) * n * 2);
        double *b0 = malloc(sizeof(double) * n * 2);
        for (int i = 0; i < n * 2; ++i) x[i] = uniform();
        expect(oracle_kernel_matrix(n, 2, x, n, n, x, n, 3, 1, 0.2, 1.0, 0.05, 1, a, n) == 0, "kernel matrix");
        for (int i = 0; i < n * n; ++i) k0[i] = a[i];
        for (int i = 0; i < n * 2; ++i) b[i] = b0[i] = uniform() - 0.5;
        expect(oracle_cholesky(n, a, n) == 0, "cholesky");
        expect(oracle_cholesky_solve(n, a, n, b, n, 2) == 0, "cholesky solve");
        for (int r = 0; r < 2; ++r)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += k0[i + j * n] * b[j + r * n];
                expect(fabs(s - b0[i + r * n]) <= 1e-10, "residual of the solve");
            }
        /* a matrix that is not positive definite reports its pivot */
        double bad[4] = {1.0, 2.0, 2.0, 1.0};
        expect(oracle_cholesky(2, bad, 2) == 2, "non-positive pivot");
        free(x); free(a); free(k0); free(b); free(b0);
    }
    {
        double r[5] = {0.0, 0.1, 1.0, 5.0, 50.0}, out[5];
        for (int two_nu = 1; two_nu <= 5; two_nu += 2) {
            expect(oracle_profile_array(two_nu, 5, r, out) == 0, "profile array");
            for (int i = 0; i < 5; ++i) expect(out[i] == oracle_matern_profile(two_nu, r[i]), "profile values");
        }
        expect(isnan(oracle_matern_profile(2, 1.0)), "unsupported nu gives NaN");
    }
    expect(oracle_num_threads() >= 1, "thread count");
    double dummy = 0.0;
    expect(oracle_mvm(-1, 1, &dummy, 1, 1, &dummy, 1, 3, 1, 0.1, 1.0, &dummy, 1, 1, &dummy, 1, 0) == -1,
           "bad arguments refused");
    if (fails) return 1;
    printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
