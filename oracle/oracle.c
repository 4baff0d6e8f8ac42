/*
 * Dense FP64 CPU oracle for the Matern kernel matrix-vector product and the
 * direct Gaussian-process solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP implementation.
 *
 * What it computes is the plain definition, written out with no blocking,
 * reordering or decomposition:
 *
 *   y_j = sum_{i=1..N} K(z_j, x_i) v_i                  (Section 2, eq. Ky / kde)
 *
 * with the scaled multivariate Matern kernels
 *
 *   L1 form:      K(u) = s2 * k_nu(||u||_1 / ell)        (eq. L1_kernel, scaled_kernel;
 *                                                        eq. matern_l1_12 / _32 / _52)
 *   product form: K(u) = s2 * prod_k k_nu(|u_k| / ell)   (eq. product_kernel;
 *                                                        eq. eq:matern_product_32)
 *
 * and the univariate profiles of Appendix C (eq. matern_1_2, matern_3_2,
 * matern_5_2), where sqrt(2 nu) sits inside k_nu:
 *
 *   k_{1/2}(r) = exp(-r)
 *   k_{3/2}(r) = (1 + sqrt(3) r) exp(-sqrt(3) r)
 *   k_{5/2}(r) = (1 + sqrt(5) r + 5/3 r^2) exp(-sqrt(5) r)
 *
 * Each output row is accumulated with Neumaier's compensated summation so the
 * oracle's own rounding error stays near 2 eps (K|v|)_j independent of N; the
 * row sum of |K_ji v_i| is returned alongside for the componentwise error norm.
 *
 * The Cholesky factorisation is the textbook right-looking algorithm for a
 * symmetric positive definite matrix (used for the direct solve of
 * (K + sigma^2 I) alpha = y, Section 1, eq. gp_mean_system).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_FORM_L1 0
#define ORACLE_FORM_PRODUCT 1

/* Matern profile k_nu(r), r >= 0 (Appendix C, eq. matern_1_2 / 3_2 / 5_2). */
double oracle_matern_profile(int two_nu, double r)
{
    if (two_nu == 1) {
        return exp(-r);
    } else if (two_nu == 3) {
        double s3 = sqrt(3.0);
        return (1.0 + s3 * r) * exp(-s3 * r);
    } else if (two_nu == 5) {
        double s5 = sqrt(5.0);
        return (1.0 + s5 * r + (5.0 / 3.0) * r * r) * exp(-s5 * r);
    }
    return NAN;
}

/* Kernel value between points a and b (stride-addressed coordinates). */
static double kernel_value(int d, const double *a, int64_t sa, const double *b, int64_t sb,
                           int two_nu, int form, double ell, double s2)
{
    if (form == ORACLE_FORM_L1) {
        double l1 = 0.0;
        for (int k = 0; k < d; ++k)
            l1 += fabs(a[k * sa] - b[k * sb]);
        return s2 * oracle_matern_profile(two_nu, l1 / ell);
    } else {
        double prod = 1.0;
        for (int k = 0; k < d; ++k)
            prod *= oracle_matern_profile(two_nu, fabs(a[k * sa] - b[k * sb]) / ell);
        return s2 * prod;
    }
}

/* Scalar kernel value for two points given as d-vectors (unit stride). */
double oracle_kernel(int d, const double *a, const double *b, int two_nu, int form,
                     double ell, double s2)
{
    return kernel_value(d, a, 1, b, 1, two_nu, form, ell, s2);
}

/*
 * Rectangular dense MVM with compensated summation.
 *   x: source points, column-major n x d (x[k*ldx + i])
 *   z: target points, column-major m x d (z[k*ldz + j])
 *   v: n x nrhs column-major (v[r*ldv + i])
 *   y: m x nrhs column-major, y_j = sum_i K(z_j, x_i) v_i
 *   yabs (optional): m x nrhs, sum_i |K(z_j, x_i) v_i|
 * Returns 0 on success, -1 on bad arguments.
 */
int oracle_mvm(int64_t n, int d, const double *x, int64_t ldx,
               int64_t m, const double *z, int64_t ldz,
               int two_nu, int form, double ell, double s2,
               const double *v, int64_t ldv, int nrhs,
               double *y, int64_t ldy, double *yabs)
{
    if (n < 0 || m < 0 || d < 1 || nrhs < 1 || ell <= 0.0)
        return -1;
    if (two_nu != 1 && two_nu != 3 && two_nu != 5)
        return -1;
    if (form != ORACLE_FORM_L1 && form != ORACLE_FORM_PRODUCT)
        return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; ++j) {
        for (int r = 0; r < nrhs; ++r) {
            double sum = 0.0, comp = 0.0, sabs = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double term = kernel_value(d, z + j, ldz, x + i, ldx, two_nu, form, ell, s2)
                              * v[(int64_t)r * ldv + i];
                /* Neumaier: carry the low-order bits lost by the running sum. */
                double t = sum + term;
                if (fabs(sum) >= fabs(term))
                    comp += (sum - t) + term;
                else
                    comp += (term - t) + sum;
                sum = t;
                sabs += fabs(term);
            }
            y[(int64_t)r * ldy + j] = sum + comp;
            if (yabs)
                yabs[(int64_t)r * ldy + j] = sabs;
        }
    }
    return 0;
}

/*
 * Same as oracle_mvm but the kernel is evaluated once per (j, i) and applied
 * to every right-hand side; used for timing at many right-hand sides.
 */
int oracle_mvm_multi(int64_t n, int d, const double *x, int64_t ldx,
                     int64_t m, const double *z, int64_t ldz,
                     int two_nu, int form, double ell, double s2,
                     const double *v, int64_t ldv, int nrhs,
                     double *y, int64_t ldy, double *yabs)
{
    if (n < 0 || m < 0 || d < 1 || nrhs < 1 || nrhs > 256 || ell <= 0.0)
        return -1;
    if (two_nu != 1 && two_nu != 3 && two_nu != 5)
        return -1;
    if (form != ORACLE_FORM_L1 && form != ORACLE_FORM_PRODUCT)
        return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; ++j) {
        double sum[256], comp[256], sabs[256];
        for (int r = 0; r < nrhs; ++r) {
            sum[r] = 0.0;
            comp[r] = 0.0;
            sabs[r] = 0.0;
        }
        for (int64_t i = 0; i < n; ++i) {
            double kv = kernel_value(d, z + j, ldz, x + i, ldx, two_nu, form, ell, s2);
            for (int r = 0; r < nrhs; ++r) {
                double term = kv * v[(int64_t)r * ldv + i];
                double t = sum[r] + term;
                if (fabs(sum[r]) >= fabs(term))
                    comp[r] += (sum[r] - t) + term;
                else
                    comp[r] += (term - t) + sum[r];
                sum[r] = t;
                sabs[r] += fabs(term);
            }
        }
        for (int r = 0; r < nrhs; ++r) {
            y[(int64_t)r * ldy + j] = sum[r] + comp[r];
            if (yabs)
                yabs[(int64_t)r * ldy + j] = sabs[r];
        }
    }
    return 0;
}

/*
 * Dense kernel matrix Kmat[i + j*ldk] = K(z_i, x_j) (column-major m x n),
 * plus `diag` added where z_i and x_j are the same point index (i == j) when
 * add_diag is nonzero (used for K + sigma^2 I with z = x).
 */
int oracle_kernel_matrix(int64_t n, int d, const double *x, int64_t ldx,
                         int64_t m, const double *z, int64_t ldz,
                         int two_nu, int form, double ell, double s2,
                         double diag, int add_diag, double *kmat, int64_t ldk)
{
    if (n < 0 || m < 0 || d < 1 || ell <= 0.0)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double kv = kernel_value(d, z + i, ldz, x + j, ldx, two_nu, form, ell, s2);
            if (add_diag && i == j)
                kv += diag;
            kmat[i + j * ldk] = kv;
        }
    }
    return 0;
}

/*
 * In-place Cholesky factorisation A = L L^T of a symmetric positive definite
 * column-major n x n matrix (lower triangle used and overwritten by L; the
 * strict upper triangle is left untouched).  Textbook right-looking outer
 * product form: scale column k by the square root of its pivot, then subtract
 * l_k l_k^T from the trailing lower triangle.  Returns 0 on success, or k+1 if
 * the pivot of column k is not positive (not numerically positive definite).
 */
int oracle_cholesky(int64_t n, double *a, int64_t lda)
{
    for (int64_t k = 0; k < n; ++k) {
        double dkk = a[k + k * lda];
        if (!(dkk > 0.0))
            return (int)(k + 1);
        double lkk = sqrt(dkk);
        a[k + k * lda] = lkk;
        for (int64_t i = k + 1; i < n; ++i)
            a[i + k * lda] /= lkk;
        const double *lk = a + k * lda;
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t j = k + 1; j < n; ++j) {
            double ljk = lk[j];
            double *cj = a + j * lda;
            for (int64_t i = j; i < n; ++i)
                cj[i] -= lk[i] * ljk;
        }
    }
    return 0;
}

/*
 * Solve (L L^T) X = B in place for nrhs right-hand sides, given the lower
 * Cholesky factor from oracle_cholesky.  B is column-major n x nrhs.
 */
int oracle_cholesky_solve(int64_t n, const double *l, int64_t ldl, double *b, int64_t ldb,
                          int nrhs)
{
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrhs; ++r) {
        double *col = b + (int64_t)r * ldb;
        /* forward substitution L w = b (column by column) */
        for (int64_t p = 0; p < n; ++p) {
            col[p] /= l[p + p * ldl];
            double wp = col[p];
            for (int64_t i = p + 1; i < n; ++i)
                col[i] -= l[i + p * ldl] * wp;
        }
        /* back substitution L^T x = w */
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = col[i];
            for (int64_t p = i + 1; p < n; ++p)
                s -= l[p + i * ldl] * col[p];
            col[i] = s / l[i + i * ldl];
        }
    }
    return 0;
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void)
{
    int nt = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        nt = omp_get_num_threads();
    }
#endif
    return nt;
}

/* Elementwise Matern profile over an array (r >= 0). */
int oracle_profile_array(int two_nu, int64_t n, const double *r, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = oracle_matern_profile(two_nu, r[i]);
    return 0;
}
