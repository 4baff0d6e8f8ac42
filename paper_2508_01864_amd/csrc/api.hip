// C entry points: plan lifecycle, the kernel product and the predictor
// (the conjugate-gradient solvers are in solver.hip).
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

inline unsigned grid1(int64_t n) {
    int64_t g = (n + BS - 1) / BS;
    if (g > 65535 * 8) g = 65535 * 8;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// layout conversion between the caller's column-major vectors and the
// point-major canonical work layout (row c = canonical point, W columns)
// ---------------------------------------------------------------------------
// y[r * ldy + i] = scale * yacc[iperm[i], r]: the derivative product has no
// diagonal term (threads take (caller point, column), column fastest)
__global__ void scale_out_kernel(const double *yacc, int W, int nrhs, const int32_t *iperm, int64_t n,
                                 double scale, double *y, int64_t ldy) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / W;
        const int r = (int)(e - i * W);
        if (r < nrhs) y[(int64_t)r * ldy + i] = scale * yacc[(int64_t)iperm[i] * W + r];
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


// vin[iperm[i] * W + r] = v[r * ldv + i] (0 for the padding columns r >= nrhs).
// Threads take (caller point i, column r) with r fastest: each thread group
// writes a whole canonical row, and the reads of a wave revisit the same few
// lines of the W caller columns, which stay in cache between neighbouring waves.
// I is the index type of the element counter (32 bits when n W fits).
template <class I>
__global__ void gather_caller_kernel(const double *v, int64_t ldv, int nrhs, const int32_t *iperm, int64_t n,
                                     double *vin, int W) {
    const I total = (I)(n * W);
    const I w = (I)W;
    for (I e = (I)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (I)gridDim.x * blockDim.x) {
        const I i = e / w;
        const int r = (int)(e - i * w);
        vin[(int64_t)iperm[i] * W + r] = r < nrhs ? v[(int64_t)r * ldv + i] : 0.0;
    }
}

// gather_caller_kernel for W = WT (16 or 32) through LDS: a workgroup reads 64
// consecutive caller points of every column (contiguous loads), then writes
// each point's WT-column row of vin (whole rows).
template <int WT>
__global__ __launch_bounds__(256) void gather_tile_kernel(const double *v, int64_t ldv, int nrhs, const int32_t *iperm,
                                                          int64_t n, double *vin) {
    constexpr int TI = 64;
    __shared__ double tile[WT][TI + 1];
    const int64_t i0 = (int64_t)blockIdx.x * TI;
    for (int k = threadIdx.x; k < WT * TI; k += 256) {
        const int r = k / TI, ii = k % TI;
        const int64_t i = i0 + ii;
        tile[r][ii] = (r < nrhs && i < n) ? v[(int64_t)r * ldv + i] : 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < WT * TI; k += 256) {
        const int ii = k / WT, r = k % WT;
        const int64_t i = i0 + ii;
        if (i < n) vin[(int64_t)iperm[i] * WT + r] = tile[r][ii];
    }
}

// acc + the G slabs' entries at q, added in pass order; the loads go out 8
// at a time ahead of their additions.
__device__ __forceinline__ double slab_sum(const double *part, int G, int64_t len, int64_t q, double acc) {
    int g = 0;
    for (; g + 8 <= G; g += 8) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = part[(int64_t)(g + k) * len + q];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += t[k];
    }
    for (; g < G; ++g) acc += part[(int64_t)g * len + q];
    return acc;
}

// y[r * ldy + i] = s2 (vin[c, r] + sum_g part_g[c, r]) + shift vin[c, r] with
// c = iperm[i]; the pass slabs are added in pass order (after yacc when not
// first).  Threads take (caller point i, column r) with r fastest: reads are
// whole canonical rows, writes fill the W caller columns a few points at a time.
template <class I>
__global__ void finish_caller_kernel(const double *vin, const double *part, int G, int first, const double *yacc,
                                     int W, int nrhs, const int32_t *iperm, int64_t n, double s2, double shift,
                                     double *y, int64_t ldy) {
    const I total = (I)(n * W);
    const I w = (I)W;
    const int64_t len = n * W;
    for (I e = (I)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (I)gridDim.x * blockDim.x) {
        const I i = e / w;
        const int r = (int)(e - i * w);
        if (r >= nrhs) continue;
        const int64_t q = (int64_t)iperm[i] * W + r;
        const double acc = slab_sum(part, G, len, q, first ? 0.0 : yacc[q]);
        const double vv = vin[q];
        y[(int64_t)r * ldy + i] = fma(shift, vv, s2 * (vv + acc));
    }
}

// The same in canonical order for narrow widths (rows of 1 or 2 doubles): the
// slab reads are sequential, the writes land at perm[c].
template <class I>
__global__ void finish_canon_kernel(const double *vin, const double *part, int G, int first, const double *yacc,
                                    int W, int nrhs, const int32_t *perm, int64_t n, double s2, double shift,
                                    double *y, int64_t ldy) {
    const I total = (I)(n * W);
    const I w = (I)W;
    const int64_t len = n * W;
    for (I q = (I)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (I)gridDim.x * blockDim.x) {
        const I c = q / w;
        const int r = (int)(q - c * w);
        if (r >= nrhs) continue;
        const double acc = slab_sum(part, G, len, (int64_t)q, first ? 0.0 : yacc[q]);
        const double vv = vin[q];
        y[(int64_t)r * ldy + perm[c]] = fma(shift, vv, s2 * (vv + acc));
    }
}

inline bool fits32(int64_t n, int W) { return (uint64_t)n * (uint64_t)W + 65536u * 8u * BS < (uint64_t(1) << 32); }

}  // namespace

void launch_gather_caller(mm_plan p, const double *v, int64_t ldv, int nrhs, double *vin, int W, hipStream_t s) {
    const int32_t *ip = static_cast<const int32_t *>(p->iperm.ptr);
    const int64_t ntile = (p->n + 63) / 64;
    if ((W == 32 || W == 16) && ntile <= INT32_MAX) {
        if (W == 32)
            hipLaunchKernelGGL(gather_tile_kernel<32>, dim3((unsigned)ntile), dim3(256), 0, s, v, ldv, nrhs, ip, p->n, vin);
        else
            hipLaunchKernelGGL(gather_tile_kernel<16>, dim3((unsigned)ntile), dim3(256), 0, s, v, ldv, nrhs, ip, p->n, vin);
    } else if (fits32(p->n, W))
        hipLaunchKernelGGL(gather_caller_kernel<uint32_t>, dim3(grid1(p->n * W)), dim3(BS), 0, s, v, ldv, nrhs, ip,
                           p->n, vin, W);
    else
        hipLaunchKernelGGL(gather_caller_kernel<int64_t>, dim3(grid1(p->n * W)), dim3(BS), 0, s, v, ldv, nrhs, ip,
                           p->n, vin, W);
}

void launch_finish_out(mm_plan p, const double *vin, const double *part, int G, int first, const double *yacc,
                       int W, int nrhs, double s2, double shift, double *y, int64_t ldy, hipStream_t s) {
    const bool small = fits32(p->n, W);
    const dim3 g(grid1(p->n * W)), b(BS);
    if (W >= 4) {
        const int32_t *ip = static_cast<const int32_t *>(p->iperm.ptr);
        if (small)
            hipLaunchKernelGGL(finish_caller_kernel<uint32_t>, g, b, 0, s, vin, part, G, first, yacc, W, nrhs, ip,
                               p->n, s2, shift, y, ldy);
        else
            hipLaunchKernelGGL(finish_caller_kernel<int64_t>, g, b, 0, s, vin, part, G, first, yacc, W, nrhs, ip,
                               p->n, s2, shift, y, ldy);
    } else {
        const int32_t *pm = static_cast<const int32_t *>(p->perm.ptr);
        if (small)
            hipLaunchKernelGGL(finish_canon_kernel<uint32_t>, g, b, 0, s, vin, part, G, first, yacc, W, nrhs, pm,
                               p->n, s2, shift, y, ldy);
        else
            hipLaunchKernelGGL(finish_canon_kernel<int64_t>, g, b, 0, s, vin, part, G, first, yacc, W, nrhs, pm,
                               p->n, s2, shift, y, ldy);
    }
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

mm_status ensure_work(mm_plan p, int W, bool der) {
    const size_t vbytes = (size_t)p->n * W * sizeof(double);
    MM_TRY(dev_reserve(p->vin, vbytes));
    MM_TRY(dev_reserve(p->yacc, vbytes));
    MM_TRY(dev_reserve(p->agg, sweep_agg_bytes(p->n, p->d, W, p->kernel, der)));
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
namespace {
// Release every buffer of a plan (no error state is touched).
void plan_free(mm_plan plan) {
    (void)hipDeviceSynchronize();
    dev_free(plan->xc);
    dev_free(plan->perm);
    dev_free(plan->iperm);
    dev_free(plan->structure);
    dev_free(plan->geo);
    dev_free(plan->vin);
    dev_free(plan->yacc);
    dev_free(plan->agg);
    dev_free(plan->part);
    dev_free(plan->pass_dev);
    for (auto &b : plan->pass_xt) dev_free(b);
    for (auto &b : plan->pass_xtpos) dev_free(b);
    for (auto &b : plan->seg_tab) dev_free(b);
    for (auto &b : plan->seg_big) dev_free(b);
    for (auto &e : plan->prof_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete plan;
}
}  // namespace

extern "C" {

const char *mm_version(void) { return "maternmvm 0.1 (gfx950)"; }

mm_status mm_set_allocator(mm_alloc_fn alloc, mm_free_fn free, void *ctx) {
    clear_error();
    if ((alloc == nullptr) != (free == nullptr)) {
        set_error("alloc and free must both be set or both be NULL");
        return MM_ERR_ARG;
    }
    set_allocator(alloc, free, ctx);
    return MM_OK;
}

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
        plan_free(p);
        return st;
    }
    *out = p;
    return MM_OK;
}

mm_status mm_plan_set_kernel(mm_plan plan, const mm_kernel *kernel, void *stream) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    MM_TRY(validate_kernel(kernel));
    if (plan->npins > 0) {
        set_error("the plan is in use by %d solver(s) or batch(es); release them before changing its kernel", plan->npins);
        return MM_ERR_ARG;
    }
    plan->kernel = *kernel;
    plan->sched.clear();  // schedules belong to a kernel class
    plan->last_stream = static_cast<hipStream_t>(stream);
    return MM_OK;
}

mm_status mm_plan_set_schedule(mm_plan plan, int32_t width, int32_t wb, int32_t e, int32_t runex) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    if (plan->npins > 0) {
        set_error("the plan is in use by %d solver(s) or batch(es); release them before changing its schedule",
                  plan->npins);
        return MM_ERR_ARG;
    }
    if (width < 1 || width > 256) {
        set_error("width must be in [1, 256] (got %d)", width);
        return MM_ERR_ARG;
    }
    const Sched sc{wb, e, runex ? 1 : 0};
    const KParams kp = kparams(plan->kernel, plan->d);
    if (!sched_available(plan->d, kp, sc, width)) {
        set_error("no compiled schedule with %d-column blocks and runs of %d for this kernel at width %d", wb, e,
                  width);
        return MM_ERR_ARG;
    }
    for (auto &en : plan->sched)
        if (en.first == width) {
            en.second = sc;
            return MM_OK;
        }
    plan->sched.push_back({width, sc});
    return MM_OK;
}

mm_status mm_plan_get_schedule(mm_plan plan, int32_t width, int32_t *wb, int32_t *e, int32_t *runex) {
    clear_error();
    if (!plan || width < 1 || width > 256) {
        set_error("plan is NULL or width outside [1, 256]");
        return MM_ERR_ARG;
    }
    Sched sc = plan_sched(plan, width, rhs_block(plan->kernel, plan->d, width));
    if (sc.e == 0)  // the default run length of the block (tiles of 256; 512 for 4-column blocks above 8 columns in d = 2)
        sc.e = sc.wb == 32 ? 128 : (sc.wb == 4 ? (plan->d == 2 && width > 8 ? 32 : 16) : (sc.wb == 2 ? 8 : 4));
    if (wb) *wb = sc.wb;
    if (e) *e = sc.e;
    if (runex) *runex = sc.runex;
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
    clear_error();
    if (!plan) return MM_OK;
    if (plan->npins > 0) {
        set_error("the plan is in use by %d solver(s) or batch(es); release them first", plan->npins);
        return MM_ERR_ARG;
    }
    plan_free(plan);
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
    (void)perm;
    launch_gather_caller(plan, v, ldv, nrhs, vin, W, s);
    int tail[2] = {0, 1};
    MM_TRY(sweep_all(plan, vin, yacc, W, R, s, tail));
    launch_finish_out(plan, vin, static_cast<const double *>(plan->part.ptr), tail[0], tail[1], yacc, W, nrhs,
                      plan->kernel.outputscale2, diag_shift, y, ldy, s);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

mm_status matern_mvm_dlengthscale(mm_plan plan, const double *v, int64_t ldv, double *y, int64_t ldy,
                                  int32_t nrhs, void *stream) {
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
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int R = rhs_block(plan->kernel, plan->d, nrhs);
    const int W = (nrhs + R - 1) / R * R;
    MM_TRY(ensure_work(plan, W, true));
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    double *vin = static_cast<double *>(plan->vin.ptr);
    double *yacc = static_cast<double *>(plan->yacc.ptr);
    (void)perm;
    launch_gather_caller(plan, v, ldv, nrhs, vin, W, s);
    MM_TRY(sweep_all_dl(plan, vin, yacc, W, R, s));
    // dK/dl = outputscale2 / l * (l dk/dl sums)
    const double scale = plan->kernel.outputscale2 / plan->kernel.lengthscale;
    hipLaunchKernelGGL(scale_out_kernel, dim3(grid1(plan->n * W)), dim3(BS), 0, s, yacc, W, nrhs,
                       static_cast<const int32_t *>(plan->iperm.ptr), plan->n, scale, y, ldy);
    MM_HIP_TRY(hipGetLastError());
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
