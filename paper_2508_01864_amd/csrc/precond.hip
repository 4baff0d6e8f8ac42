// Rank-k pivoted Cholesky of the kernel matrix, the preconditioner of
// Appendix A ("Preconditioning"): P = L L^T + sigma^2 I with L L^T the pivoted
// Cholesky decomposition of K (after Harbrecht, Peters and Schneider), applied
// through the Woodbury identity inside conjugate gradients (solver.hip).
//
// The factorisation is greedy on the residual diagonal d = diag(K - L L^T):
// each step picks the largest residual (the smallest caller index among equal
// values), evaluates one kernel column directly, removes the previous
// columns' contribution and updates d.  All of it stays on the device: a
// step is a column launch followed by a one-block selection launch that
// writes the next pivot, so the host does not wait inside the loop.  L is
// stored row-major (point-major) in canonical order, which makes both
// products of the Woodbury apply read it with coalesced or contiguous
// accesses.
#include "mm_internal.h"

#include <cmath>

namespace mm {
namespace {

constexpr int BS = 256;
constexpr int PNB = 256;  // blocks of the pivot reductions (fixed: deterministic)
constexpr int GCH = 32;   // row chunks of the Gram product (fixed: deterministic)

struct PcState {
    int64_t p;      // pivot of the next column (canonical index)
    double dp;      // its residual diagonal
    double trace;   // residual trace sum(d)
    double trace0;  // trace of K
    int stop;       // no further columns
    int rank;       // columns computed
};

// Matern profile in units t = a r (a = sqrt(2 nu) / lengthscale), Appendix C
// eq. matern_1_2 / 3_2 / 5_2.
__device__ __forceinline__ double profile_t(int P, double t) {
    const double e = exp(-t);
    if (P == 1) return e;
    if (P == 2) return fma(t, e, e);
    return e * fma(t, fma(t, 1.0 / 3.0, 1.0), 1.0);
}

// K(x_i, x_j) in canonical indices (product or L1 form), with outputscale2.
__device__ __forceinline__ double kval(const double *xc, int64_t n, int d, int64_t i, int64_t j, int P, bool prod,
                                       double a, double s2) {
    if (prod) {
        double k = 1.0;
        for (int c = 0; c < d; ++c) k *= profile_t(P, a * fabs(xc[(int64_t)c * n + i] - xc[(int64_t)c * n + j]));
        return s2 * k;
    }
    double r = 0.0;
    for (int c = 0; c < d; ++c) r += fabs(xc[(int64_t)c * n + i] - xc[(int64_t)c * n + j]);
    return s2 * profile_t(P, a * r);
}

// (value, caller index, canonical index): larger value wins, then smaller caller index.
__device__ __forceinline__ bool better(double v, int32_t ci, double bv, int32_t bci) {
    return v > bv || (v == bv && ci < bci);
}

// Block-level argmax and sum of d over the block's rows, written to the partials.
__device__ __forceinline__ void block_argmax_sum(double v, int32_t ci, int64_t i, double sumv, double *pv, int32_t *pci,
                                                 int64_t *pi, double *ps, int blk) {
    __shared__ double sv[BS], ss[BS];
    __shared__ int32_t sci[BS];
    __shared__ int64_t si[BS];
    const int t = threadIdx.x;
    sv[t] = v;
    sci[t] = ci;
    si[t] = i;
    ss[t] = sumv;
    __syncthreads();
    for (int h = BS / 2; h > 0; h >>= 1) {
        if (t < h) {
            if (better(sv[t + h], sci[t + h], sv[t], sci[t])) {
                sv[t] = sv[t + h];
                sci[t] = sci[t + h];
                si[t] = si[t + h];
            }
            ss[t] += ss[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        pv[blk] = sv[0];
        pci[blk] = sci[0];
        pi[blk] = si[0];
        ps[blk] = ss[0];
    }
}

// d = diag K = outputscale2 (the profile is 1 at zero distance).
__global__ void pc_init(double *d, const int32_t *perm, int64_t n, double s2, double *pv, int32_t *pci, int64_t *pi,
                        double *ps) {
    const int64_t chunk = (n + PNB - 1) / PNB;
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double bv = -1.0, sum = 0.0;
    int32_t bci = 0x7fffffff;
    int64_t bi = -1;
    for (int64_t i = lo + threadIdx.x; i < hi; i += BS) {
        d[i] = s2;
        sum += s2;
        if (better(s2, perm[i], bv, bci)) {
            bv = s2;
            bci = perm[i];
            bi = i;
        }
    }
    block_argmax_sum(bv, bci, bi, sum, pv, pci, pi, ps, blockIdx.x);
}

// Next pivot from the block partials (one block; fixed-order tree).
__global__ void pc_select(const double *pv, const int32_t *pci, const int64_t *pi, const double *ps, PcState *st,
                          int first, int kmax, double tol) {
    __shared__ double sv[BS], ss[BS];
    __shared__ int32_t sci[BS];
    __shared__ int64_t si[BS];
    const int t = threadIdx.x;
    static_assert(PNB == BS, "one partial per thread");
    sv[t] = pv[t];
    sci[t] = pci[t];
    si[t] = pi[t];
    ss[t] = ps[t];
    __syncthreads();
    for (int h = BS / 2; h > 0; h >>= 1) {
        if (t < h) {
            if (better(sv[t + h], sci[t + h], sv[t], sci[t])) {
                sv[t] = sv[t + h];
                sci[t] = sci[t + h];
                si[t] = si[t + h];
            }
            ss[t] += ss[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (first) {
            st->trace0 = ss[0];
            st->rank = 0;
            st->stop = 0;
        }
        st->trace = ss[0];
        st->p = si[0];
        st->dp = sv[0];
        if (st->rank >= kmax || !(sv[0] > 0.0) || si[0] < 0 || ss[0] <= tol * st->trace0) st->stop = 1;
    }
}

// Column m of L and the residual-diagonal update, then the partials of the next pivot.
__global__ void pc_column(const double *xc, const int32_t *perm, int64_t n, int d, int P, int prod, double a, double s2,
                          double *L, int kmax, int m, double *dg, PcState *st, double *pv, int32_t *pci, int64_t *pi,
                          double *ps, int32_t *piv) {
    const int stop = st->stop;
    const int64_t chunk = (n + PNB - 1) / PNB;
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double bv = -1.0, sum = 0.0;
    int32_t bci = 0x7fffffff;
    int64_t bi = -1;
    if (!stop) {
        const int64_t p = st->p;
        const double sq = sqrt(st->dp);
        const double *rowp = L + p * kmax;
        for (int64_t i = lo + threadIdx.x; i < hi; i += BS) {
            double l;
            if (i == p) {
                l = sq;
            } else {
                double dot = 0.0;
                const double *rowi = L + i * kmax;
                for (int j = 0; j < m; ++j) dot = fma(rowi[j], rowp[j], dot);
                l = (kval(xc, n, d, i, p, P, prod != 0, a, s2) - dot) / sq;
            }
            L[i * kmax + m] = l;
            double di = (i == p) ? 0.0 : dg[i] - l * l;
            di = di > 0.0 ? di : 0.0;
            dg[i] = di;
            sum += di;
            if (better(di, perm[i], bv, bci)) {
                bv = di;
                bci = perm[i];
                bi = i;
            }
        }
    }
    block_argmax_sum(bv, bci, bi, sum, pv, pci, pi, ps, blockIdx.x);
    if (!stop && blockIdx.x == 0 && threadIdx.x == 0) {
        st->rank = m + 1;
        piv[m] = perm[st->p];
    }
}

// Partial Gram products part[ch][a][b] = sum over the chunk's rows of L[i][a] L[i][b].
__global__ void pc_gram_partial(const double *L, int64_t n, int kmax, int rank, double *part) {
    const int ch = blockIdx.x;
    const int a = blockIdx.y * 16 + threadIdx.x / 16;
    const int b = blockIdx.z * 16 + threadIdx.x % 16;
    const int64_t chunk = (n + GCH - 1) / GCH;
    const int64_t lo = ch * chunk, hi = lo + chunk < n ? lo + chunk : n;
    if (a >= rank || b >= rank) return;
    double acc = 0.0;
    for (int64_t i = lo; i < hi; ++i) acc = fma(L[i * kmax + a], L[i * kmax + b], acc);
    part[((int64_t)ch * rank + a) * rank + b] = acc;
}

__global__ void pc_gram_reduce(const double *part, int rank, double *G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rank * rank) return;
    double s = 0.0;
    for (int ch = 0; ch < GCH; ++ch) s += part[(int64_t)ch * rank * rank + e];
    G[e] = s;
}

__global__ void pc_export(const double *L, const int32_t *perm, int64_t n, int kmax, int rank, double *out, int64_t ld) {
    const int64_t total = n * rank;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / rank;
        const int j = (int)(e - i * rank);
        out[(int64_t)j * ld + perm[i]] = L[i * kmax + j];
    }
}

}  // namespace
}  // namespace mm

using namespace mm;

extern "C" {

mm_status mm_precond_create(mm_plan plan, int32_t max_rank, double tol, void *stream, mm_precond *out) {
    clear_error();
    if (!out || !plan) {
        set_error("plan and out are required");
        return MM_ERR_ARG;
    }
    *out = nullptr;
    if (max_rank < 1 || max_rank > MM_PRECOND_MAX_RANK) {
        set_error("max_rank must be in [1, %d]", MM_PRECOND_MAX_RANK);
        return MM_ERR_ARG;
    }
    if (!(tol >= 0.0) || !std::isfinite(tol)) {
        set_error("tol must be finite and >= 0");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = plan->n;
    const int kmax = max_rank < n ? max_rank : (int)n;
    mm_precond pc = new (std::nothrow) mm_precond_s();
    if (!pc) {
        set_error("host allocation failed");
        return MM_ERR_NOMEM;
    }
    pc->plan = plan;
    pc->kmax = kmax;
    auto fail = [&](mm_status st) {
        dev_free(pc->L);
        dev_free(pc->work);
        delete pc;
        return st;
    };
    mm_status st = dev_alloc(pc->L, (size_t)n * kmax * sizeof(double));
    // work: d (n) | partial values, sums (PNB each) | caller indices (PNB int32) |
    //       canonical indices (PNB int64) | state
    const size_t wbytes = (size_t)n * 8 + (size_t)PNB * (8 + 8 + 4 + 8) + sizeof(PcState) + 64 + (size_t)kmax * 4;
    if (st == MM_OK) st = dev_alloc(pc->work, wbytes);
    if (st != MM_OK) return fail(st);
    char *w = static_cast<char *>(pc->work.ptr);
    double *dg = reinterpret_cast<double *>(w);
    double *pv = dg + n;
    double *psum = pv + PNB;
    int64_t *pi = reinterpret_cast<int64_t *>(psum + PNB);
    int32_t *pci = reinterpret_cast<int32_t *>(pi + PNB);
    PcState *state = reinterpret_cast<PcState *>(reinterpret_cast<char *>(pci + PNB) + 8);
    int32_t *piv = reinterpret_cast<int32_t *>(state + 1);
    const KParams kp = kparams(plan->kernel, plan->d);
    const double *xc = static_cast<const double *>(plan->xc.ptr);
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    double *L = static_cast<double *>(pc->L.ptr);
    hipLaunchKernelGGL(pc_init, dim3(PNB), dim3(BS), 0, s, dg, perm, n, kp.s2, pv, pci, pi, psum);
    hipLaunchKernelGGL(pc_select, dim3(1), dim3(BS), 0, s, pv, pci, pi, psum, state, 1, kmax, tol);
    for (int m = 0; m < kmax; ++m) {
        hipLaunchKernelGGL(pc_column, dim3(PNB), dim3(BS), 0, s, xc, perm, n, plan->d, kp.P, kp.prod ? 1 : 0, kp.a,
                           kp.s2, L, kmax, m, dg, state, pv, pci, pi, psum, piv);
        hipLaunchKernelGGL(pc_select, dim3(1), dim3(BS), 0, s, pv, pci, pi, psum, state, 0, kmax, tol);
    }
    if (hipGetLastError() != hipSuccess) {
        set_error("pivoted Cholesky launch failed");
        return fail(MM_ERR_HIP);
    }
    PcState hs{};
    if (hipMemcpyAsync(&hs, state, sizeof hs, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("HIP error in the pivoted Cholesky");
        return fail(MM_ERR_HIP);
    }
    pc->rank = hs.rank;
    pc->trace0 = hs.trace0;
    pc->trace_res = hs.trace;
    pc->pivots.resize(hs.rank);
    if (hs.rank > 0 &&
        (hipMemcpy(pc->pivots.data(), piv, (size_t)hs.rank * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)) {
        set_error("HIP error reading the pivots");
        return fail(MM_ERR_HIP);
    }
    // Gram matrix L^T L of the computed columns
    if (pc->rank > 0) {
        const int r = pc->rank;
        DevBuf gp;
        st = dev_alloc(gp, ((size_t)GCH + 1) * r * r * sizeof(double));
        if (st != MM_OK) return fail(st);
        double *part = static_cast<double *>(gp.ptr);
        double *G = part + (size_t)GCH * r * r;
        const unsigned nt = (unsigned)((r + 15) / 16);
        hipLaunchKernelGGL(pc_gram_partial, dim3(GCH, nt, nt), dim3(BS), 0, s, L, n, kmax, r, part);
        hipLaunchKernelGGL(pc_gram_reduce, dim3((unsigned)((r * r + BS - 1) / BS)), dim3(BS), 0, s, part, r, G);
        pc->gram.resize((size_t)r * r);
        hipError_t e = hipMemcpyAsync(pc->gram.data(), G, (size_t)r * r * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dev_free(gp);
        if (e != hipSuccess) {
            set_error("HIP error in the Gram product: %s", hipGetErrorString(e));
            return fail(MM_ERR_HIP);
        }
    }
    plan->npins++;
    *out = pc;
    return MM_OK;
}

mm_status mm_precond_info(mm_precond pc, int32_t *rank, double *trace_residual, double *trace_k) {
    clear_error();
    if (!pc) {
        set_error("preconditioner is NULL");
        return MM_ERR_ARG;
    }
    if (rank) *rank = pc->rank;
    if (trace_residual) *trace_residual = pc->trace_res;
    if (trace_k) *trace_k = pc->trace0;
    return MM_OK;
}

mm_status mm_precond_factor(mm_precond pc, double *L, int64_t ldl, int32_t *pivots, void *stream) {
    clear_error();
    if (!pc || (!L && !pivots)) {
        set_error("preconditioner and L or pivots are required");
        return MM_ERR_ARG;
    }
    if (pivots)
        for (int m = 0; m < pc->rank; ++m) pivots[m] = pc->pivots[m];
    if (!L) return MM_OK;
    const int64_t n = pc->plan->n;
    if (ldl < n) {
        set_error("ldl must be >= n");
        return MM_ERR_ARG;
    }
    if (pc->rank == 0) return MM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t g = (n * pc->rank + BS - 1) / BS;
    if (g > 65535 * 8) g = 65535 * 8;
    hipLaunchKernelGGL(pc_export, dim3((unsigned)g), dim3(BS), 0, s, static_cast<const double *>(pc->L.ptr),
                       static_cast<const int32_t *>(pc->plan->perm.ptr), n, pc->kmax, pc->rank, L, ldl);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

mm_status mm_precond_destroy(mm_precond pc) {
    clear_error();
    if (!pc) return MM_OK;
    if (pc->npins > 0) {
        set_error("the preconditioner is in use by %d solver(s); destroy them first", pc->npins);
        return MM_ERR_ARG;
    }
    (void)hipDeviceSynchronize();
    pc->plan->npins--;
    dev_free(pc->L);
    dev_free(pc->work);
    delete pc;
    return MM_OK;
}

}  // extern "C"
