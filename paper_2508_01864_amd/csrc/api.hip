// C entry points: plan lifecycle, the kernel product, conjugate gradients with
// the generalised-least-squares fixed effects, and the predictor.
#include "mm_internal.h"

#include <cmath>
#include <cstring>

namespace mm {
const char *last_error_str();
mm_status validate_kernel(const mm_kernel *k);
mm_status plan_build(mm_plan p, const double *x, int64_t ldx, hipStream_t s);
size_t plan_footprint(int64_t n, int d, int nrhs, const mm_kernel &k);

namespace {

constexpr int BS = 256;
constexpr int NRED = 256;  // blocks of the first reduction stage (fixed: deterministic sums)

inline unsigned grid1(int64_t n) {
    int64_t g = (n + BS - 1) / BS;
    if (g > 65535 * 8) g = 65535 * 8;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// layout conversion between the caller's column-major vectors and the
// point-major canonical work layout (row c = canonical point, W columns)
// ---------------------------------------------------------------------------
__global__ void gather_in_kernel(const double *v, int64_t ldv, int nrhs, const int32_t *perm,
                                 int64_t n, double *vin, int W) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / W;
        const int r = (int)(e - c * W);
        vin[e] = r < nrhs ? v[(int64_t)r * ldv + perm[c]] : 0.0;
    }
}

__global__ void scatter_out_kernel(const double *vin, const double *yacc, int W, int nrhs,
                                   const int32_t *perm, int64_t n, double s2, double shift,
                                   double *y, int64_t ldy) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n);
        const int64_t c = e - (int64_t)r * n;
        const double vv = vin[c * W + r];
        y[(int64_t)r * ldy + perm[c]] = s2 * (vv + yacc[c * W + r]) + shift * vv;
    }
}

__global__ void fill_int_kernel(int *p, int n, int val) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = val;
}

__global__ void fill_kernel(double *p, int64_t n, double val) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = val;
}

// ---------------------------------------------------------------------------
// conjugate-gradient kernels (W columns, point-major, W divides BS)
// ---------------------------------------------------------------------------
// partial column dot products: part[b*W + r] = sum over block b's rows of a[c,r]*b[c,r]
__device__ __forceinline__ void block_col_dot(double acc, int W, double *sm, double *part) {
    sm[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < W) {
        double s = 0.0;
        for (int t = threadIdx.x; t < BS; t += W) s += sm[t];
        part[blockIdx.x * W + threadIdx.x] = s;
    }
}

__device__ __forceinline__ void row_range(int64_t n, int64_t &lo, int64_t &hi) {
    const int64_t chunk = (n + NRED - 1) / NRED;
    lo = blockIdx.x * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
}

// Q = s2 (P + Y) + sigma2 P, and partial dots P.Q
__global__ void cg_apply_kernel(const double *P, const double *Y, double *Q, int64_t n, int W,
                                double s2, double sigma2, double *part) {
    __shared__ double sm[BS];
    int64_t lo, hi;
    row_range(n, lo, hi);
    double acc = 0.0;
    for (int64_t e = lo * W + threadIdx.x; e < hi * W; e += BS) {
        const double p = P[e];
        const double q = s2 * (p + Y[e]) + sigma2 * p;
        Q[e] = q;
        acc += p * q;
    }
    block_col_dot(acc, W, sm, part);
}

// scalars per column: [0] rr, [1] pAp, [2] alpha, [3] beta, [4] bnorm, [5] active, [6] iters
constexpr int NS = 8;

__global__ void cg_alpha_kernel(const double *part, int W, double *sc, int *flags) {
    const int r = threadIdx.x;
    if (r >= W) return;
    double s = 0.0;
    for (int b = 0; b < NRED; ++b) s += part[b * W + r];
    double *c = sc + r * NS;
    c[1] = s;
    if (c[5] != 0.0) {
        if (!(s > 0.0)) {
            flags[1] = 1;  // breakdown: non-positive curvature
            c[2] = 0.0;
            c[5] = 0.0;
        } else {
            c[2] = c[0] / s;
        }
    } else {
        c[2] = 0.0;
    }
}

// X += alpha P ; R -= alpha Q ; partial dots R.R
__global__ void cg_update_kernel(double *X, double *R, const double *P, const double *Q, int64_t n,
                                 int W, const double *sc, double *part) {
    __shared__ double sm[BS];
    int64_t lo, hi;
    row_range(n, lo, hi);
    const int r = threadIdx.x % W;
    const double al = sc[r * NS + 2];
    double acc = 0.0;
    for (int64_t e = lo * W + threadIdx.x; e < hi * W; e += BS) {
        const double xr = X[e] + al * P[e];
        const double rr = R[e] - al * Q[e];
        X[e] = xr;
        R[e] = rr;
        acc += rr * rr;
    }
    block_col_dot(acc, W, sm, part);
}

__global__ void cg_beta_kernel(const double *part, int W, double *sc, int *flags, double rtol,
                               int iter) {
    const int r = threadIdx.x;
    if (r >= W) return;
    double s = 0.0;
    for (int b = 0; b < NRED; ++b) s += part[b * W + r];
    double *c = sc + r * NS;
    if (c[5] != 0.0) {
        c[6] = (double)iter;
        if (sqrt(s) <= rtol * c[4]) {
            c[5] = 0.0;  // converged: freeze this column
            c[3] = 0.0;
        } else {
            c[3] = s / c[0];
            atomicAdd(&flags[0], 1);  // still active (integer count)
        }
        c[7] = sqrt(s);
        c[0] = s;
    } else {
        c[3] = 0.0;
    }
}

// P = R + beta P for active columns
__global__ void cg_dir_kernel(double *P, const double *R, int64_t n, int W, const double *sc) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % W);
        if (sc[r * NS + 5] != 0.0) P[e] = R[e] + sc[r * NS + 3] * P[e];
    }
}

// initial scalars from B: rr = bnorm^2, active where b != 0
__global__ void cg_init_kernel(const double *part, int W, double *sc, int nactive_cols) {
    const int r = threadIdx.x;
    if (r >= W) return;
    double s = 0.0;
    for (int b = 0; b < NRED; ++b) s += part[b * W + r];
    double *c = sc + r * NS;
    c[0] = s;
    c[1] = 0.0;
    c[2] = 0.0;
    c[3] = 0.0;
    c[4] = sqrt(s);
    c[5] = (r < nactive_cols && s > 0.0) ? 1.0 : 0.0;
    c[6] = 0.0;
    c[7] = sqrt(s);
}

__global__ void col_dot_kernel(const double *A, const double *B, int64_t n, int W, double *part) {
    __shared__ double sm[BS];
    int64_t lo, hi;
    row_range(n, lo, hi);
    double acc = 0.0;
    for (int64_t e = lo * W + threadIdx.x; e < hi * W; e += BS) acc += A[e] * B[e];
    block_col_dot(acc, W, sm, part);
}

// fixed-effects right-hand side B = [y, 1, x_1..x_d] in canonical order (W columns)
__global__ void fe_rhs_kernel(const double *y, const int32_t *perm, const double *xc, int64_t n,
                              int d, int fe, int W, double *B) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        double *row = B + c * W;
        row[0] = y[perm[c]];
        int col = 1;
        if (fe) {
            row[col++] = 1.0;
            for (int k = 0; k < d; ++k) row[col++] = xc[k * n + c];
        }
        for (; col < W; ++col) row[col] = 0.0;
    }
}

// partial sums of H^T X for the (d+1) x W Gram block, H = [1, x_1..x_d]
__global__ void fe_gram_kernel(const double *X, const double *xc, int64_t n, int d, int W,
                               double *part) {
    __shared__ double sm[BS];
    int64_t lo, hi;
    row_range(n, lo, hi);
    const int r = threadIdx.x % W;
    for (int i = 0; i <= d; ++i) {
        double acc = 0.0;
        for (int64_t e = lo * W + threadIdx.x; e < hi * W; e += BS) {
            const int64_t c = e / W;
            const double h = i == 0 ? 1.0 : xc[(int64_t)(i - 1) * n + c];
            acc += h * X[e];
        }
        (void)r;
        __syncthreads();
        sm[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x < W) {
            double s = 0.0;
            for (int t = threadIdx.x; t < BS; t += W) s += sm[t];
            part[((int64_t)blockIdx.x * (d + 1) + i) * W + threadIdx.x] = s;
        }
    }
}

// alpha (caller order) = X[:,0] - sum_j X[:,1+j] beta_j
__global__ void fe_alpha_kernel(const double *X, const int32_t *perm, int64_t n, int W, int nb,
                                double b0, double b1, double b2, double b3, double *alpha) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const double *row = X + c * W;
        double a = row[0];
        if (nb > 0) a -= row[1] * b0;
        if (nb > 1) a -= row[2] * b1;
        if (nb > 2) a -= row[3] * b2;
        if (nb > 3) a -= row[4] * b3;
        alpha[perm[c]] = a;
    }
}

__global__ void col_out_kernel(const double *X, const int32_t *perm, int64_t n, int W, int nrhs,
                               double *out, int64_t ldo) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n);
        const int64_t c = e - (int64_t)r * n;
        out[(int64_t)r * ldo + perm[c]] = X[c * W + r];
    }
}

// union points for prediction: [canonical x ; z] column-major, and weights [alpha ; 0]
__global__ void union_kernel(const double *xc, int64_t n, const double *z, int64_t m, int64_t ldz,
                             int d, const double *alpha, const int32_t *perm, double *U, double *u) {
    const int64_t nm = n + m;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nm;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < d; ++k)
            U[k * nm + i] = i < n ? xc[k * n + i] : z[k * ldz + (i - n)];
        u[i] = i < n ? alpha[perm[i]] : 0.0;
    }
}

__global__ void predict_out_kernel(const double *out, int64_t n, int64_t m, const double *z,
                                   int64_t ldz, int d, int has_beta, double b0, double b1,
                                   double b2, double b3, double *mean) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
         j += (int64_t)gridDim.x * blockDim.x) {
        double v = out[n + j];
        if (has_beta) {
            const double b[4] = {b0, b1, b2, b3};
            v += b[0];
            for (int k = 0; k < d; ++k) v += b[k + 1] * z[k * ldz + j];
        }
        mean[j] = v;
    }
}

int pow2ceil(int v) {
    int w = 1;
    while (w < v) w <<= 1;
    return w;
}

}  // namespace

void launch_gather_in(const double *v, int64_t ldv, int nrhs, const int32_t *perm, int64_t n,
                      double *vin, int W, hipStream_t s) {
    hipLaunchKernelGGL(gather_in_kernel, dim3(grid1(n * W)), dim3(BS), 0, s, v, ldv, nrhs, perm, n, vin, W);
}

void launch_scatter_out(const double *vin, const double *yacc, int W, int nrhs, const int32_t *perm,
                        int64_t n, double s2, double shift, double *y, int64_t ldy, hipStream_t s) {
    hipLaunchKernelGGL(scatter_out_kernel, dim3(grid1(n * nrhs)), dim3(BS), 0, s, vin, yacc, W, nrhs,
                       perm, n, s2, shift, y, ldy);
}

// Fold the recorded event pairs into the running totals (waits for them).
mm_status profile_flush(mm_plan p, double *ms_out, int64_t *cnt_out) {
    double ms = p->prof_ms;
    int64_t cnt = p->prof_launches;
    for (size_t i = 0; i < p->prof_used; ++i) {
        MM_HIP_TRY(hipEventSynchronize(p->prof_events[i].second));
        float t = 0.f;
        MM_HIP_TRY(hipEventElapsedTime(&t, p->prof_events[i].first, p->prof_events[i].second));
        ms += t;
        ++cnt;
    }
    p->prof_ms = ms;
    p->prof_launches = cnt;
    p->prof_used = 0;
    *ms_out = ms;
    *cnt_out = cnt;
    return MM_OK;
}

mm_status ensure_work(mm_plan p, int W) {
    const size_t vbytes = (size_t)p->n * W * sizeof(double);
    MM_TRY(dev_reserve(p->vin, vbytes));
    MM_TRY(dev_reserve(p->yacc, vbytes));
    MM_TRY(dev_reserve(p->agg, sweep_agg_bytes(p->n, p->d, W, p->kernel)));
    MM_TRY(dev_reserve(p->part, sweep_part_bytes(p->n, (int)p->passes.size(), W)));
    return MM_OK;
}

// yacc <- sum over passes of the off-diagonal kernel sums of vin (unscaled)
mm_status sweep_into(mm_plan p, const double *vin, double *yacc, int W, int R, hipStream_t s) {
    return sweep_all(p, vin, yacc, W, R, s);
}

}  // namespace mm

using namespace mm;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *mm_version(void) { return "maternmvm 0.1 (gfx950)"; }

const char *mm_status_str(mm_status st) {
    switch (st) {
        case MM_OK: return "MM_OK";
        case MM_ERR_ARG: return "MM_ERR_ARG";
        case MM_ERR_NOMEM: return "MM_ERR_NOMEM";
        case MM_ERR_HIP: return "MM_ERR_HIP";
        case MM_ERR_NOTPD: return "MM_ERR_NOTPD";
        case MM_ERR_BREAKDOWN: return "MM_ERR_BREAKDOWN";
        case MM_ERR_NOCONV: return "MM_ERR_NOCONV";
    }
    return "MM_ERR_UNKNOWN";
}

const char *mm_last_error(void) { return last_error_str(); }

size_t mm_plan_footprint_bytes(int64_t n, int32_t d, int32_t nrhs, const mm_kernel *kernel) {
    if (n < 1 || d < 1 || d > 3 || nrhs < 1 || nrhs > 256 || validate_kernel(kernel) != MM_OK) return 0;
    clear_error();
    return plan_footprint(n, d, nrhs, *kernel);
}

mm_status mm_plan_create(const double *x, int64_t n, int32_t d, int64_t ldx, const mm_kernel *kernel,
                         void *stream, mm_plan *out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return MM_ERR_ARG;
    }
    *out = nullptr;
    if (!x) {
        set_error("x is NULL");
        return MM_ERR_ARG;
    }
    if (n < 1 || n > (int64_t(1) << 30)) {
        set_error("n must be in [1, 2^30] (got %lld)", (long long)n);
        return MM_ERR_ARG;
    }
    if (d < 1 || d > 3) {
        set_error("d must be 1, 2 or 3 (got %d)", d);
        return MM_ERR_ARG;
    }
    if (ldx < n) {
        set_error("ldx (%lld) must be >= n (%lld)", (long long)ldx, (long long)n);
        return MM_ERR_ARG;
    }
    MM_TRY(validate_kernel(kernel));
    mm_plan p = new (std::nothrow) mm_plan_s();
    if (!p) {
        set_error("host allocation failed");
        return MM_ERR_NOMEM;
    }
    (void)hipGetDevice(&p->device);
    p->n = n;
    p->d = d;
    p->kernel = *kernel;
    hipStream_t s = static_cast<hipStream_t>(stream);
    p->last_stream = s;
    mm_status st = plan_build(p, x, ldx, s);
    if (st != MM_OK) {
        mm_plan_destroy(p);
        return st;
    }
    *out = p;
    return MM_OK;
}

mm_status mm_plan_set_kernel(mm_plan plan, const mm_kernel *kernel) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    MM_TRY(validate_kernel(kernel));
    plan->kernel = *kernel;
    return MM_OK;
}

mm_status mm_plan_info(mm_plan plan, int64_t *n, int32_t *d, mm_kernel *kernel) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    if (n) *n = plan->n;
    if (d) *d = plan->d;
    if (kernel) *kernel = plan->kernel;
    return MM_OK;
}

mm_status mm_plan_destroy(mm_plan plan) {
    if (!plan) return MM_OK;
    (void)hipDeviceSynchronize();
    dev_free(plan->xc);
    dev_free(plan->perm);
    dev_free(plan->structure);
    dev_free(plan->vin);
    dev_free(plan->yacc);
    dev_free(plan->agg);
    dev_free(plan->part);
    dev_free(plan->pass_dev);
    dev_free(plan->pass_xt);
    dev_free(plan->cgbuf);
    dev_free(plan->redbuf);
    for (auto &e : plan->prof_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete plan;
    return MM_OK;
}

mm_status matern_mvm(mm_plan plan, const double *v, int64_t ldv, double *y, int64_t ldy, int32_t nrhs,
                     double diag_shift, void *stream) {
    clear_error();
    if (!plan || !v || !y) {
        set_error("plan, v and y must be non-NULL");
        return MM_ERR_ARG;
    }
    if (nrhs < 1 || nrhs > 256) {
        set_error("nrhs must be in [1, 256] (got %d)", nrhs);
        return MM_ERR_ARG;
    }
    if (ldv < plan->n || ldy < plan->n) {
        set_error("ldv and ldy must be >= n");
        return MM_ERR_ARG;
    }
    if (!std::isfinite(diag_shift)) {
        set_error("diag_shift must be finite");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int R = rhs_block(plan->kernel, plan->d, nrhs);
    const int W = (nrhs + R - 1) / R * R;
    MM_TRY(ensure_work(plan, W));
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    double *vin = static_cast<double *>(plan->vin.ptr);
    double *yacc = static_cast<double *>(plan->yacc.ptr);
    launch_gather_in(v, ldv, nrhs, perm, plan->n, vin, W, s);
    MM_TRY(sweep_into(plan, vin, yacc, W, R, s));
    launch_scatter_out(vin, yacc, W, nrhs, perm, plan->n, plan->kernel.outputscale2, diag_shift, y, ldy, s);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

// Core CG on canonical point-major columns.  B (n x W) is read, X (n x W) written.
static mm_status cg_core(mm_plan p, const double *B, double *X, int W, int ncols, double sigma2,
                         double rtol, int maxit, mm_solve_info *info, hipStream_t s, int *conv_cols,
                         bool *breakdown, int *iters_out, double *relres_out) {
    const int64_t n = p->n;
    const int R = rhs_block(p->kernel, p->d, W);
    if (W % R != 0) {
        set_error("internal: CG width");
        return MM_ERR_ARG;
    }
    MM_TRY(ensure_work(p, W));
    const size_t vec = (size_t)n * W;
    MM_TRY(dev_reserve(p->cgbuf, 3 * vec * sizeof(double)));
    MM_TRY(dev_reserve(p->redbuf, (size_t)(NRED * W * 8 + W * NS + 16) * sizeof(double)));
    double *Rr = static_cast<double *>(p->cgbuf.ptr);
    double *Pp = Rr + vec;
    double *Q = Pp + vec;
    double *part = static_cast<double *>(p->redbuf.ptr);
    double *sc = part + (size_t)NRED * W * 8;
    int *flags = reinterpret_cast<int *>(sc + W * NS);
    double *yacc = static_cast<double *>(p->yacc.ptr);
    const double s2 = p->kernel.outputscale2;

    // x0 = 0, r0 = b, p0 = r0
    hipLaunchKernelGGL(fill_kernel, dim3(grid1(vec)), dim3(BS), 0, s, X, (int64_t)vec, 0.0);
    MM_HIP_TRY(hipMemcpyAsync(Rr, B, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    MM_HIP_TRY(hipMemcpyAsync(Pp, B, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(col_dot_kernel, dim3(NRED), dim3(BS), 0, s, B, B, n, W, part);
    hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(BS), 0, s, part, W, sc, ncols);
    MM_HIP_TRY(hipGetLastError());

    int it = 0;
    int hflags[2] = {1, 0};   // [0] columns still active, [1] breakdown seen (sticky)
    const int check_every = 8;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(32), 0, s, flags, 2, 0);
    while (it < maxit) {
        const int batch = (maxit - it) < check_every ? (maxit - it) : check_every;
        for (int b = 0; b < batch; ++b) {
            ++it;
            MM_TRY(sweep_into(p, Pp, yacc, W, R, s));
            hipLaunchKernelGGL(cg_apply_kernel, dim3(NRED), dim3(BS), 0, s, Pp, yacc, Q, n, W, s2, sigma2, part);
            hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(BS), 0, s, part, W, sc, flags);
            hipLaunchKernelGGL(cg_update_kernel, dim3(NRED), dim3(BS), 0, s, X, Rr, Pp, Q, n, W, sc, part);
            if (b == batch - 1)  // count the columns still active after the last iteration of the batch
                hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(32), 0, s, flags, 1, 0);
            hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(BS), 0, s, part, W, sc, flags, rtol, it);
            hipLaunchKernelGGL(cg_dir_kernel, dim3(grid1(vec)), dim3(BS), 0, s, Pp, Rr, n, W, sc);
        }
        MM_HIP_TRY(hipGetLastError());
        MM_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, s));
        MM_HIP_TRY(hipStreamSynchronize(s));
        if (hflags[1] || hflags[0] == 0) break;
    }
    std::vector<double> hsc((size_t)W * NS);
    MM_HIP_TRY(hipMemcpyAsync(hsc.data(), sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    int conv = 0;
    double relmax = 0.0;
    for (int r = 0; r < ncols; ++r) {
        const double bn = hsc[r * NS + 4];
        const double rn = hsc[r * NS + 7];
        const double rel = bn > 0.0 ? rn / bn : 0.0;
        if (rel > relmax) relmax = rel;
        if (bn == 0.0 || rel <= rtol) ++conv;
    }
    *conv_cols = conv;
    *breakdown = hflags[1] != 0;
    *iters_out = it;
    *relres_out = relmax;
    if (info) {
        info->iters = it;
        info->converged_cols = conv;
        info->relres_max = relmax;
    }
    return MM_OK;
}

static mm_status check_solve_args(mm_plan plan, double sigma2, double rtol, int32_t maxit) {
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) {
        set_error("sigma2 must be positive and finite");
        return MM_ERR_ARG;
    }
    if (!(rtol > 0.0) || !std::isfinite(rtol)) {
        set_error("rtol must be positive and finite");
        return MM_ERR_ARG;
    }
    if (maxit < 1) {
        set_error("maxit must be >= 1");
        return MM_ERR_ARG;
    }
    const KParams kp = kparams(plan->kernel, plan->d);
    if (!kp.prod && plan->d >= 2 && kp.P >= 2) {
        set_error("the L1 Matern form with nu >= 3/2 in d >= 2 is not positive definite; use the product form");
        return MM_ERR_NOTPD;
    }
    return MM_OK;
}

mm_status gp_cg_solve(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                      int32_t maxit, double *alpha, double *beta, mm_solve_info *info, void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol, maxit));
    if (!y || !alpha) {
        set_error("y and alpha must be non-NULL");
        return MM_ERR_ARG;
    }
    if (fixed_effects && !beta) {
        set_error("beta must be non-NULL when fixed_effects is set");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int64_t n = plan->n;
    const int d = plan->d;
    const int ncols = fixed_effects ? d + 2 : 1;
    const int R = rhs_block(plan->kernel, d, ncols);
    int W = pow2ceil(ncols > R ? ncols : R);
    DevBuf bx;
    MM_TRY(dev_alloc(bx, 2 * (size_t)n * W * sizeof(double)));
    double *B = static_cast<double *>(bx.ptr);
    double *X = B + (size_t)n * W;
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    const double *xc = static_cast<const double *>(plan->xc.ptr);
    hipLaunchKernelGGL(fe_rhs_kernel, dim3(grid1(n)), dim3(BS), 0, s, y, perm, xc, n, d, fixed_effects ? 1 : 0, W, B);
    int conv = 0, iters = 0;
    bool brk = false;
    double rel = 0.0;
    mm_status st = cg_core(plan, B, X, W, ncols, sigma2, rtol, maxit, info, s, &conv, &brk, &iters, &rel);
    if (st != MM_OK) {
        dev_free(bx);
        return st;
    }
    double hb[4] = {0.0, 0.0, 0.0, 0.0};
    if (fixed_effects) {
        // G = H^T A^-1 H, g = H^T A^-1 y  from the (d+1) x W block H^T X
        const int nb = d + 1;
        double *part = static_cast<double *>(plan->redbuf.ptr);
        hipLaunchKernelGGL(fe_gram_kernel, dim3(NRED), dim3(BS), 0, s, X, xc, n, d, W, part);
        std::vector<double> hp((size_t)NRED * nb * W);
        if (hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            dev_free(bx);
            set_error("HIP error in the GLS reduction");
            return MM_ERR_HIP;
        }
        std::vector<double> HX((size_t)nb * W, 0.0);  // HX[i*W + j] = h_i^T X_j
        for (int b = 0; b < NRED; ++b)
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < W; ++j) HX[i * W + j] += hp[((size_t)b * nb + i) * W + j];
        // G (nb x nb, symmetrised) and right-hand side g
        double G[4][4], g[4];
        for (int i = 0; i < nb; ++i) {
            g[i] = HX[i * W + 0];
            for (int j = 0; j < nb; ++j) G[i][j] = 0.5 * (HX[i * W + 1 + j] + HX[j * W + 1 + i]);
        }
        // Cholesky solve of the small SPD system
        double Lm[4][4] = {{0}};
        for (int j = 0; j < nb; ++j) {
            double dsum = G[j][j];
            for (int k = 0; k < j; ++k) dsum -= Lm[j][k] * Lm[j][k];
            if (!(dsum > 0.0)) {
                dev_free(bx);
                set_error("GLS Gram matrix H^T A^-1 H is not positive definite (collinear features?)");
                return MM_ERR_NOTPD;
            }
            Lm[j][j] = sqrt(dsum);
            for (int i = j + 1; i < nb; ++i) {
                double t = G[i][j];
                for (int k = 0; k < j; ++k) t -= Lm[i][k] * Lm[j][k];
                Lm[i][j] = t / Lm[j][j];
            }
        }
        double w[4];
        for (int i = 0; i < nb; ++i) {
            double t = g[i];
            for (int k = 0; k < i; ++k) t -= Lm[i][k] * w[k];
            w[i] = t / Lm[i][i];
        }
        for (int i = nb - 1; i >= 0; --i) {
            double t = w[i];
            for (int k = i + 1; k < nb; ++k) t -= Lm[k][i] * hb[k];
            hb[i] = t / Lm[i][i];
        }
        for (int i = 0; i < nb; ++i) beta[i] = hb[i];
        hipLaunchKernelGGL(fe_alpha_kernel, dim3(grid1(n)), dim3(BS), 0, s, X, perm, n, W, nb, hb[0], hb[1], hb[2],
                           hb[3], alpha);
    } else {
        hipLaunchKernelGGL(col_out_kernel, dim3(grid1(n)), dim3(BS), 0, s, X, perm, n, W, 1, alpha, n);
    }
    hipError_t e = hipStreamSynchronize(s);
    dev_free(bx);
    if (e != hipSuccess) {
        set_error("HIP error after the solve: %s", hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    if (brk) {
        set_error("conjugate gradients broke down (p^T A p <= 0)");
        return MM_ERR_BREAKDOWN;
    }
    if (conv < ncols) {
        set_error("conjugate gradients did not reach rtol in %d iterations (relres %.3e)", iters, rel);
        return MM_ERR_NOCONV;
    }
    return MM_OK;
}

mm_status gp_cg_solve_multi(mm_plan plan, const double *Bc, int64_t ldb, int32_t nrhs, double sigma2,
                            double rtol, int32_t maxit, double *Xc, int64_t ldx, mm_solve_info *info,
                            void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol, maxit));
    if (!Bc || !Xc) {
        set_error("B and X must be non-NULL");
        return MM_ERR_ARG;
    }
    if (nrhs < 1 || nrhs > 64) {
        set_error("nrhs must be in [1, 64]");
        return MM_ERR_ARG;
    }
    if (ldb < plan->n || ldx < plan->n) {
        set_error("ldb and ldx must be >= n");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int64_t n = plan->n;
    const int R = rhs_block(plan->kernel, plan->d, nrhs);
    const int W = pow2ceil(nrhs > R ? nrhs : R);
    DevBuf bx;
    MM_TRY(dev_alloc(bx, 2 * (size_t)n * W * sizeof(double)));
    double *B = static_cast<double *>(bx.ptr);
    double *X = B + (size_t)n * W;
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    launch_gather_in(Bc, ldb, nrhs, perm, n, B, W, s);
    int conv = 0, iters = 0;
    bool brk = false;
    double rel = 0.0;
    mm_status st = cg_core(plan, B, X, W, nrhs, sigma2, rtol, maxit, info, s, &conv, &brk, &iters, &rel);
    if (st != MM_OK) {
        dev_free(bx);
        return st;
    }
    hipLaunchKernelGGL(col_out_kernel, dim3(grid1(n * nrhs)), dim3(BS), 0, s, X, perm, n, W, nrhs, Xc, ldx);
    hipError_t e = hipStreamSynchronize(s);
    dev_free(bx);
    if (e != hipSuccess) {
        set_error("HIP error after the solve: %s", hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    if (brk) {
        set_error("conjugate gradients broke down (p^T A p <= 0)");
        return MM_ERR_BREAKDOWN;
    }
    if (conv < nrhs) {
        set_error("conjugate gradients did not reach rtol in %d iterations (relres %.3e)", iters, rel);
        return MM_ERR_NOCONV;
    }
    return MM_OK;
}

mm_status gp_predict(mm_plan plan, const double *alpha, const double *beta, const double *z, int64_t m,
                     int64_t ldz, double *mean, void *stream) {
    clear_error();
    if (!plan || !alpha || !z || !mean) {
        set_error("plan, alpha, z and mean must be non-NULL");
        return MM_ERR_ARG;
    }
    if (m < 1 || ldz < m) {
        set_error("m must be >= 1 and ldz >= m");
        return MM_ERR_ARG;
    }
    const int64_t n = plan->n;
    const int d = plan->d;
    if (n + m > (int64_t(1) << 30)) {
        set_error("n + m exceeds 2^30");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int64_t nm = n + m;
    DevBuf ub;
    MM_TRY(dev_alloc(ub, ((size_t)d + 2) * nm * sizeof(double)));
    double *U = static_cast<double *>(ub.ptr);
    double *u = U + (size_t)d * nm;
    double *out = u + nm;
    hipLaunchKernelGGL(union_kernel, dim3(grid1(nm)), dim3(BS), 0, s, static_cast<const double *>(plan->xc.ptr), n,
                       z, m, ldz, d, alpha, static_cast<const int32_t *>(plan->perm.ptr), U, u);
    mm_plan up = nullptr;
    mm_status st = mm_plan_create(U, nm, d, nm, &plan->kernel, stream, &up);
    if (st == MM_OK) st = matern_mvm(up, u, nm, out, nm, 1, 0.0, stream);
    if (st == MM_OK) {
        double b[4] = {0, 0, 0, 0};
        if (beta)
            for (int i = 0; i <= d; ++i) b[i] = beta[i];
        hipLaunchKernelGGL(predict_out_kernel, dim3(grid1(m)), dim3(BS), 0, s, out, n, m, z, ldz, d, beta ? 1 : 0,
                           b[0], b[1], b[2], b[3], mean);
        if (hipStreamSynchronize(s) != hipSuccess) {
            set_error("HIP error in predict: %s", hipGetErrorString(hipGetLastError()));
            st = MM_ERR_HIP;
        }
    }
    if (up) mm_plan_destroy(up);
    dev_free(ub);
    return st;
}

mm_status mm_plan_profile_enable(mm_plan plan, int32_t enable) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    plan->profile = enable != 0;
    return MM_OK;
}

mm_status mm_plan_profile_read(mm_plan plan, double *sweep_ms, int64_t *sweep_launches,
                               int64_t *sweep_passes, int32_t reset) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    double ms = 0.0;
    int64_t cnt = 0;
    MM_TRY(profile_flush(plan, &ms, &cnt));
    if (sweep_ms) *sweep_ms = ms;
    if (sweep_launches) *sweep_launches = cnt;
    if (sweep_passes) *sweep_passes = plan->prof_units;
    if (reset) {
        plan->prof_ms = 0.0;
        plan->prof_launches = 0;
        plan->prof_units = 0;
    }
    return MM_OK;
}

}  // extern "C"
