// Conjugate gradients as solver objects (Appendix A, Algorithm 2 with the
// identity preconditioner and a null initial guess), iterated alone or many
// at once.  A solver keeps its right-hand sides, iterate, residual, direction
// and scalars on the device in the plan's canonical point order, so
// iterations need no permutation and no host round trip.  Batched iterations
// run every solver's product in the batched sweeps (one launch per kernel
// configuration and phase) and every CG update in one launch per step over a
// table of (solver, block) items; a single solver runs the very same kernels
// with a table of one, so a problem's arithmetic does not depend on its
// batch-mates (results are bitwise identical alone and in a batch).
#include "mm_internal.h"

#include <cmath>
#include <cstring>

namespace mm {

namespace {

constexpr int BS = 256;
constexpr int WAVE = 64;   // lanes per wavefront
constexpr int NRED = 1024;  // row blocks of the column dot products (fixed: deterministic sums)
constexpr int NS = 11;     // scalars per column: [0] r.r [1] p.Ap [2] alpha [3] beta
                           // [4] |b| [5] active [6] iterations while active [7] |r|
                           // [8] r.r and [9] active as the update left them (read by
                           //     every workgroup of the direction step, which rewrites [0], [5])
                           // [10] the column's stopping tolerance (relative to |b|): rtol,
                           //     tightened when a recomputed residual misses rtol
constexpr int CHUNK = 1024;
constexpr int PUB = 1024;     // row blocks of the partial products L^T r (fixed: deterministic)
constexpr int PC_MAXW = 8;    // columns of a preconditioned solver
// Solvers of at most FUSE_W columns reduce the CG dot-product partials inside
// every workgroup of the update and direction steps; wider ones have them
// reduced once by a separate launch (a redundant reduction would read
// NRED x W partials in each of the NRED workgroups).
constexpr int FUSE_W = 8;
static_assert(NRED % BS == 0, "whole row-block partials per thread in the scalar kernels");

struct CgDesc {
    const double *B;
    double *X, *R, *P, *Q, *Y;
    double *part;  // NRED x W partial column sums (p.Ap of the apply step, |b|^2 at the start)
    double *part2; // NRED x W partial r.r of the update step
    double *red;   // 3 x W reduced sums of wide solvers: p.Ap, r.r, r.z
    const double *slabs;  // per-pass partial products of P (nslab of n x W), or
    int nslab;            //   nslab < 0: the product is already summed in Y
    double *sc;    // W x NS
    int *flags;    // [0] active columns after the last update, [1] breakdown seen
    // pivoted Cholesky preconditioner (rank 0: none)
    const double *Lpc;    // n x kmax row-major, canonical order
    const double *Minv;   // rank x rank: (I + L^T L / sigma2)^{-1}, formed as Rinv^T Rinv (Rinv: inverse Cholesky factor)
    double *ub;           // rank x W: L^T R
    double *Z;            // P^{-1} R
    double *part_rz;      // NRED x W partial r.z
    double *part_u;       // PUB x rank x W partial L^T r
    double *wv;           // rank x W
    int kmax, rank;
    // Lanczos coefficients (Algorithm 2): alpha_k, beta_k of column r at [(k * W + r) * 2 + {0, 1}]
    double *tlog;
    int tlog_cap;
    int64_t n;
    int W;
    int ncols;
    double s2, sigma2, rtol;
};

__device__ __forceinline__ void row_range(int64_t n, int blk, int64_t &lo, int64_t &hi) {
    const int64_t chunk = (n + NRED - 1) / NRED;
    lo = blk * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
}

// part[blk][r] = sum over the block's rows of acc (one value per thread, W | BS)
__device__ __forceinline__ void block_col_sum(double acc, int W, double *sm, double *part, int blk) {
    sm[threadIdx.x] = acc;
    __syncthreads();
    if ((int)threadIdx.x < W) {
        double s = 0.0;
        for (int t = threadIdx.x; t < BS; t += W) s += sm[t];
        part[(int64_t)blk * W + threadIdx.x] = s;
    }
    __syncthreads();
}

// tot[r] = sum over the NRED row blocks of part[b][r] for every column r < W:
// each thread adds NRED/BS partials in a fixed order, then a fixed binary tree
// (deterministic); one workgroup of BS threads.
__device__ __forceinline__ void reduce_cols(const double *part, int W, double *red, double *tot) {
    const int t = threadIdx.x;
    for (int r = 0; r < W; ++r) {
        double v = 0.0;
        for (int j = 0; j < NRED / BS; ++j) v += part[(int64_t)(t + j * BS) * W + r];
        red[t] = v;
        __syncthreads();
        for (int h = BS / 2; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) tot[r] = red[0];
        __syncthreads();
    }
}

// The same sums for a workgroup that needs them for its own work: each thread
// adds NRED/BS partials per column in a fixed order, each wave adds its lanes
// by a fixed shuffle tree and the four wave sums are added in order.  Every
// workgroup that calls it gets bitwise the same tot.  wred: 4 x 4 doubles.
__device__ __forceinline__ void reduce_cols_w(const double *part, int W, double *wred, double *tot, int c0 = 0,
                                              int c1 = -1) {
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    static_assert(BS == 4 * WAVE, "four waves per workgroup");
    if (c1 < 0) c1 = W;
    for (int r0 = c0; r0 < c1; r0 += 4) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = 0.0;
            if (r0 + q < c1)
                for (int j = 0; j < NRED / BS; ++j) v[q] += part[(int64_t)(t + j * BS) * W + r0 + q];
        }
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += __shfl_down(v[q], o, WAVE);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) wred[wv * 4 + q] = v[q];
        __syncthreads();
        if (t < 4 && r0 + t < c1) tot[r0 + t] = ((wred[t] + wred[4 + t]) + wred[8 + t]) + wred[12 + t];
        __syncthreads();
    }
}

// x0 = 0, r0 = b, p0 = r0, partial |b|^2
__global__ void cg_init_b(const CgDesc *ds, const int2 *items, int nitems) {
    __shared__ double sm[BS];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        int64_t lo, hi;
        row_range(d.n, it.y, lo, hi);
        double acc = 0.0;
        for (int64_t e = lo * d.W + threadIdx.x; e < hi * d.W; e += BS) {
            const double b = d.B[e];
            d.X[e] = 0.0;
            d.R[e] = b;
            d.P[e] = b;
            acc = fma(b, b, acc);
        }
        block_col_sum(acc, d.W, sm, d.part, it.y);
    }
}

__global__ void cg_init_scalars_b(const CgDesc *ds, int nsol) {
    __shared__ double red[BS];
    __shared__ double tot[64];
    for (int k = blockIdx.x; k < nsol; k += gridDim.x) {
        const CgDesc d = ds[k];
        reduce_cols(d.part, d.W, red, tot);
        __shared__ double tz[64];
        if (d.rank > 0) reduce_cols(d.part_rz, d.W, red, tz);
        const int r = threadIdx.x;
        if (r < d.W) {
            const double s = tot[r];
            double *c = d.sc + r * NS;
            c[0] = d.rank > 0 ? tz[r] : s;  // r.z (= r.r without preconditioner)
            c[1] = 0.0;
            c[2] = 0.0;
            c[3] = 0.0;
            c[4] = sqrt(s);
            c[5] = (r < d.ncols && s > 0.0) ? 1.0 : 0.0;
            c[6] = 0.0;
            c[7] = sqrt(s);
            c[8] = c[0];
            c[9] = c[5];
            c[10] = d.rtol;
        }
        if (r == 0) {
            d.flags[0] = 0;
            d.flags[1] = 0;
        }
        __syncthreads();
    }
}

// The scalars of column r after the alpha step (p.Ap = s); non-positive
// curvature = breakdown.  Written by one workgroup per solver; the others
// compute the same alpha from the same sums.  [8], [9] keep r.z and the active
// flag for the direction step; the active-column count restarts.
__device__ __forceinline__ void alpha_record(const CgDesc &d, int r, double s) {
    double *c = d.sc + r * NS;
    c[1] = s;
    if (c[5] != 0.0) {
        if (!(s > 0.0)) {
            d.flags[1] = 1;
            c[2] = 0.0;
            c[5] = 0.0;
        } else {
            c[2] = c[0] / s;
            const int it = (int)c[6];
            if (d.tlog && it < d.tlog_cap) d.tlog[((int64_t)it * d.W + r) * 2] = c[2];
            c[6] += 1.0;
        }
    } else {
        c[2] = 0.0;
    }
    c[8] = c[0];
    c[9] = c[5];
    if (r == 0) d.flags[0] = 0;
}

// The scalars of column r after the direction step (new r.r = s, r.z = rz):
// beta = r.z(new) / r.z(old); columns reaching the tolerance are frozen.
// Written by one workgroup per solver from the snapshots [8], [9].
__device__ __forceinline__ void beta_record(const CgDesc &d, int r, double s, double rz) {
    double *c = d.sc + r * NS;
    if (c[9] != 0.0) {
        if (sqrt(s) <= c[10] * c[4]) {
            c[5] = 0.0;
            c[3] = 0.0;
        } else {
            c[3] = rz / c[8];
            const int it = (int)c[6] - 1;
            if (d.tlog && it >= 0 && it < d.tlog_cap) d.tlog[((int64_t)it * d.W + r) * 2 + 1] = c[3];
            atomicAdd(&d.flags[0], 1);  // integer count of still-active columns
        }
        c[7] = sqrt(s);
        c[0] = rz;
    } else {
        c[3] = 0.0;
    }
}

// Q = s2 (P + K~ P) + sigma2 P (K~ P: the product's off-diagonal sums) and
// partial P.Q
__global__ void cg_apply_b(const CgDesc *ds, const int2 *items, int nitems) {
    __shared__ double sm[BS];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        int64_t lo, hi;
        row_range(d.n, it.y, lo, hi);
        double acc = 0.0;
        const int64_t len = d.n * d.W;
        for (int64_t e = lo * d.W + threadIdx.x; e < hi * d.W; e += BS) {
            const double p = d.P[e];
            double y;
            if (d.nslab < 0) {
                y = d.Y[e];
            } else {  // the product's per-pass partials, summed in pass order
                // (loads issued four at a time, the additions stay in order)
                y = 0.0;
                const double *sp = d.slabs + e;
                int g = 0;
                for (; g + 4 <= d.nslab; g += 4) {
                    const double a0 = sp[(int64_t)g * len], a1 = sp[(int64_t)(g + 1) * len];
                    const double a2 = sp[(int64_t)(g + 2) * len], a3 = sp[(int64_t)(g + 3) * len];
                    y += a0;
                    y += a1;
                    y += a2;
                    y += a3;
                }
                for (; g < d.nslab; ++g) y += sp[(int64_t)g * len];
            }
            const double q = fma(d.sigma2, p, d.s2 * (p + y));
            d.Q[e] = q;
            acc = fma(p, q, acc);
        }
        block_col_sum(acc, d.W, sm, d.part, it.y);
    }
}

// The CG sums of the solvers wider than FUSE_W, once per step: which = 0 the
// p.Ap partials (before the update), 1 the r.r and r.z partials (before the
// direction step).  Items: (solver, group of four columns).
__global__ void cg_reduce_b(const CgDesc *ds, const int2 *items, int nitems, int which) {
    __shared__ double wred[16];
    __shared__ double tot[64];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const int c0 = 4 * it.y, c1 = c0 + 4 < d.W ? c0 + 4 : d.W;
        if (which == 0) {
            reduce_cols_w(d.part, d.W, wred, tot, c0, c1);
            if ((int)threadIdx.x < c1 - c0) d.red[c0 + threadIdx.x] = tot[c0 + threadIdx.x];
        } else {
            reduce_cols_w(d.part2, d.W, wred, tot, c0, c1);
            if ((int)threadIdx.x < c1 - c0) d.red[d.W + c0 + threadIdx.x] = tot[c0 + threadIdx.x];
            if (d.rank > 0) {
                reduce_cols_w(d.part_rz, d.W, wred, tot, c0, c1);
                if ((int)threadIdx.x < c1 - c0) d.red[2 * d.W + c0 + threadIdx.x] = tot[c0 + threadIdx.x];
            }
        }
        __syncthreads();
    }
}

// alpha = r.z / p.Ap per active column from the p.Ap partials (every
// workgroup reduces them; the solver's first row block records the scalars),
// then X += alpha P, R -= alpha Q and partial R.R
__global__ void cg_update_b(const CgDesc *ds, const int2 *items, int nitems) {
    __shared__ double sm[BS];
    __shared__ double wred[16];
    __shared__ double tot[64];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        if (d.W <= FUSE_W) reduce_cols_w(d.part, d.W, wred, tot);
        int64_t lo, hi;
        row_range(d.n, it.y, lo, hi);
        const int r = threadIdx.x % d.W;  // W divides BS: the thread's column is fixed
        const double s = d.W <= FUSE_W ? tot[r] : d.red[r];
        const double *c = d.sc + r * NS;
        const double al = (c[5] != 0.0 && s > 0.0) ? c[0] / s : 0.0;
        __syncthreads();  // every thread has read the scalars before they are recorded
        if (it.y == 0 && (int)threadIdx.x < d.W) alpha_record(d, r, s);
        double acc = 0.0;
        for (int64_t e = lo * d.W + threadIdx.x; e < hi * d.W; e += BS) {
            const double xr = fma(al, d.P[e], d.X[e]);
            const double rr = fma(-al, d.Q[e], d.R[e]);
            d.X[e] = xr;
            d.R[e] = rr;
            acc = fma(rr, rr, acc);
        }
        block_col_sum(acc, d.W, sm, d.part2, it.y);
    }
}

// beta = r.z(new) / r.z(old) from the r.r (and r.z) partials, columns reaching
// the tolerance frozen (every workgroup reduces the partials; the solver's
// first chunk records the scalars), then P = R + beta P (Z for R with a
// preconditioner) on the still-active columns
__global__ void cg_dir_b(const CgDesc *ds, const int2 *items, int nitems) {
    __shared__ double wred[16];
    __shared__ double tot[64];
    __shared__ double tz[64];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const bool fused = d.W <= FUSE_W;
        if (fused) {
            reduce_cols_w(d.part2, d.W, wred, tot);
            if (d.rank > 0) reduce_cols_w(d.part_rz, d.W, wred, tz);
        }
        const int64_t lo = (int64_t)it.y * CHUNK;
        const int64_t len = d.n * d.W;
        const int64_t hi = lo + CHUNK < len ? lo + CHUNK : len;
        // W divides CHUNK and the stride: the thread's column is fixed
        const int r = (int)((lo + threadIdx.x) & (d.W - 1));
        const double s = fused ? tot[r] : d.red[d.W + r];
        const double rz = d.rank > 0 ? (fused ? tz[r] : d.red[2 * d.W + r]) : s;
        const double *c = d.sc + r * NS;
        const bool on = c[9] != 0.0 && !(sqrt(s) <= c[10] * c[4]);
        const double be = on ? rz / c[8] : 0.0;
        if (it.y == 0 && (int)threadIdx.x < d.W) beta_record(d, r, s, rz);
        if (!on) continue;
        const double *src = d.rank > 0 ? d.Z : d.R;
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) d.P[e] = fma(be, d.P[e], src[e]);
    }
}

// ---- recomputed residual and restart (residual replacement) ----
// After Q = A X (the product of the iterate, through the same sweeps and
// apply step): R = B - Q, partial r.r per column into part2 and, for the
// fixed-effects combination of Section 3.2, partial |r_0 - sum_i beta_i r_{1+i}|^2
// into column 0 of part (y - H beta - A alpha = r_0 - sum_i beta_i r_{1+i}).
__global__ void cg_resid_b(const CgDesc *ds, const int2 *items, int nitems, int nb, double b0, double b1, double b2,
                           double b3) {
    __shared__ double sm[BS];
    __shared__ double sr[BS];
    const double bt[4] = {b0, b1, b2, b3};
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        int64_t lo, hi;
        row_range(d.n, it.y, lo, hi);
        double acc = 0.0, comb = 0.0;
        // BS / W whole rows per step (W divides BS): thread t holds column t mod W
        for (int64_t base = lo * d.W; base < hi * d.W; base += BS) {
            const int64_t e = base + threadIdx.x;
            double r = 0.0;
            if (e < hi * d.W) {
                r = d.B[e] - d.Q[e];
                d.R[e] = r;
            }
            acc = fma(r, r, acc);
            sr[threadIdx.x] = r;
            __syncthreads();
            const int row = threadIdx.x;
            if (nb > 0 && row < BS / d.W && base + (int64_t)row * d.W < hi * d.W) {
                double t = sr[row * d.W];
                for (int k = 0; k < nb; ++k) t = fma(-bt[k], sr[row * d.W + 1 + k], t);
                comb = fma(t, t, comb);
            }
            __syncthreads();
        }
        block_col_sum(acc, d.W, sm, d.part2, it.y);
        block_col_sum(comb, 1, sm, d.part, it.y);  // one column: the sum of every thread's value
    }
}

// P = R: the restart direction without a preconditioner
__global__ void cg_restart_dir_b(const CgDesc *ds, const int2 *items, int nitems) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const int64_t lo = (int64_t)it.y * CHUNK;
        const int64_t len = d.n * d.W;
        const int64_t hi = lo + CHUNK < len ? lo + CHUNK : len;
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) d.P[e] = d.R[e];
    }
}

// Scalars of a restart from the recomputed residual: r.z (r.r without a
// preconditioner), |r|, the tolerances tol[r] (host-chosen), and the active
// flags: a column is active while |r| > tol |b|, unless freeze (every column
// frozen: the solve has met its tolerance).  |b| and the iteration counts stay.
__global__ void cg_restart_scalars_b(const CgDesc *ds, const double *tol, int freeze) {
    __shared__ double red[BS];
    __shared__ double tot[64];
    __shared__ double tz[64];
    const CgDesc d = ds[0];
    reduce_cols(d.part2, d.W, red, tot);
    if (d.rank > 0) reduce_cols(d.part_rz, d.W, red, tz);
    const int r = threadIdx.x;
    if (r < d.W) {
        double *c = d.sc + r * NS;
        const double rr = tot[r];
        c[0] = d.rank > 0 ? tz[r] : rr;
        c[1] = 0.0;
        c[2] = 0.0;
        c[3] = 0.0;
        c[7] = sqrt(rr);
        c[10] = tol[r];
        c[5] = (!freeze && r < d.ncols && c[4] > 0.0 && c[7] > c[10] * c[4]) ? 1.0 : 0.0;
        c[8] = c[0];
        c[9] = c[5];
    }
    if (r == 0) {
        d.flags[0] = 0;
        d.flags[1] = 0;
    }
}

// ---- preconditioner solve s_P (Woodbury, Appendix A "Preconditioning") ----
// partial L^T R over the rows of block it.y (of PUB): thread t takes the
// (column of L, column of R) pairs t, t + BS, ...; rows are read 8 at a time
__global__ void cg_pa_b(const CgDesc *ds, const int2 *items, int nitems) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const int64_t chunk = (d.n + PUB - 1) / PUB;
        const int64_t lo = it.y * chunk;
        const int64_t hi = lo + chunk < d.n ? lo + chunk : d.n;
        const int rw = d.rank * d.W;
        for (int e = threadIdx.x; e < rw; e += BS) {
            const int j = e / d.W, c = e - (e / d.W) * d.W;
            double acc = 0.0;
            int64_t row = lo;
            for (; row + 8 <= hi; row += 8) {
                double l8[8], r8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    l8[q] = d.Lpc[(row + q) * d.kmax + j];
                    r8[q] = d.R[(row + q) * d.W + c];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) acc = fma(l8[q], r8[q], acc);
            }
            for (; row < hi; ++row) acc = fma(d.Lpc[row * d.kmax + j], d.R[row * d.W + c], acc);
            d.part_u[(int64_t)it.y * rw + e] = acc;
        }
    }
}

// u[e] = sum of the PUB partials of element e (one block per element, fixed tree)
__global__ void cg_pu_b(const CgDesc *ds, const int2 *items, int nitems) {
    __shared__ double red[BS];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const int rw = d.rank * d.W;
        const int e = it.y;
        double v = 0.0;
        for (int b = threadIdx.x; b < PUB; b += BS) v += d.part_u[(int64_t)b * rw + e];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int h = BS / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) d.ub[e] = red[0];
        __syncthreads();
    }
}

// w = (I + L^T L / sigma2)^{-1} u with the stored inverse Minv = Rinv^T Rinv:
// one block per (solver, row j of Minv), fixed-tree dot products
__global__ void cg_pb_b(const CgDesc *ds, const int2 *items, int nitems) {
    __shared__ double red[BS];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const int j = it.y / d.W, c = it.y - (it.y / d.W) * d.W;
        double v = 0.0;
        for (int l = threadIdx.x; l < d.rank; l += BS) v = fma(d.Minv[j * d.rank + l], d.ub[l * d.W + c], v);
        red[threadIdx.x] = v;
        __syncthreads();
        for (int h = BS / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) d.wv[it.y] = red[0];
        __syncthreads();
    }
}

// Z = R / sigma2 - L w / sigma2^2 on the rows of block it.y (of NRED), partial
// R.Z per column; at initialisation also P = Z
__global__ void cg_pc_b(const CgDesc *ds, const int2 *items, int nitems, int init) {
    __shared__ double sw[MM_PRECOND_MAX_RANK * PC_MAXW];
    __shared__ double red[BS];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const CgDesc d = ds[it.x];
        const int rw = d.rank * d.W;
        for (int e = threadIdx.x; e < rw; e += BS) sw[e] = d.wv[e];
        __syncthreads();
        int64_t lo, hi;
        row_range(d.n, it.y, lo, hi);
        const double inv = 1.0 / d.sigma2;
        double rz[PC_MAXW];
#pragma unroll
        for (int c = 0; c < PC_MAXW; ++c) rz[c] = 0.0;
        for (int64_t row = lo + threadIdx.x; row < hi; row += BS) {
            double acc[PC_MAXW];
#pragma unroll
            for (int c = 0; c < PC_MAXW; ++c) acc[c] = 0.0;
            const double *lr = d.Lpc + row * d.kmax;
            int j = 0;
            for (; j + 8 <= d.rank; j += 8) {  // the row's entries are loaded 8 at a time
                double l8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) l8[q] = lr[j + q];
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int c = 0; c < PC_MAXW; ++c)
                        if (c < d.W) acc[c] = fma(l8[q], sw[(j + q) * d.W + c], acc[c]);
            }
            for (; j < d.rank; ++j) {
                const double l = lr[j];
#pragma unroll
                for (int c = 0; c < PC_MAXW; ++c)
                    if (c < d.W) acc[c] = fma(l, sw[j * d.W + c], acc[c]);
            }
#pragma unroll
            for (int c = 0; c < PC_MAXW; ++c) {
                if (c >= d.W) break;
                const double rv = d.R[row * d.W + c];
                const double z = fma(-acc[c], inv * inv, rv * inv);
                d.Z[row * d.W + c] = z;
                if (init) d.P[row * d.W + c] = z;
                rz[c] = fma(rv, z, rz[c]);
            }
        }
        for (int c = 0; c < d.W; ++c) {
            red[threadIdx.x] = rz[c < PC_MAXW ? c : 0];
            __syncthreads();
            for (int h = BS / 2; h > 0; h >>= 1) {
                if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
                __syncthreads();
            }
            if (threadIdx.x == 0) d.part_rz[(int64_t)it.y * d.W + c] = red[0];
            __syncthreads();
        }
    }
}

// status[k] = (active columns, breakdown) of every solver, for one host read
__global__ void cg_collect_b(const CgDesc *ds, int nsol, int2 *status) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nsol; k += gridDim.x * blockDim.x)
        status[k] = make_int2(ds[k].flags[0], ds[k].flags[1]);
}

// right-hand sides [y, 1, x_1..x_d] (fixed effects) or [y] in canonical order
__global__ void fe_rhs_kernel(const double *y, const int32_t *perm, const double *xc, int64_t n, int d,
                              int fe, int W, double *B) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        double *row = B + c * W;
        row[0] = y[perm[c]];
        int col = 1;
        if (fe) {
            row[col++] = 1.0;
            for (int k = 0; k < d; ++k) row[col++] = xc[(int64_t)k * n + c];
        }
        for (; col < W; ++col) row[col] = 0.0;
    }
}

__global__ void gather_cols_kernel(const double *v, int64_t ldv, int nrhs, const int32_t *perm, int64_t n,
                                   double *out, int W) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / W;
        const int r = (int)(e - c * W);
        out[e] = r < nrhs ? v[(int64_t)r * ldv + perm[c]] : 0.0;
    }
}

// Preconditioned log-determinant probes z = L g1 + sigma g2 (N(0, L L^T +
// sigma^2 I) draws from standard normal g1, g2), canonical rows, W columns
// (the padding zero): L is the preconditioner's factor (canonical rows of kmax,
// rank columns used), g1 rank x nb and g2 (caller rows) n x nb, column-major.
__global__ void pc_probe_kernel(const double *Lpc, int kmax, int rank, const double *G1, int64_t ldg1,
                                const double *G2, int64_t ldg2, int nb, double sigma, const int32_t *perm,
                                int64_t n, double *B, int W) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / W;
        const int r = (int)(e - c * W);
        double z = 0.0;
        if (r < nb) {
            const double *lr = Lpc + c * kmax;
            const double *g = G1 + (int64_t)r * ldg1;
            for (int j = 0; j < rank; ++j) z = fma(lr[j], g[j], z);
            z = fma(sigma, G2[(int64_t)r * ldg2 + perm[c]], z);
        }
        B[e] = z;
    }
}

// partial sums of H^T X for the (d+1) x W block, H = [1, x_1..x_d]
__global__ void fe_gram_kernel(const double *X, const double *xc, int64_t n, int d, int W, double *part) {
    __shared__ double sm[BS];
    int64_t lo, hi;
    row_range(n, blockIdx.x, lo, hi);
    for (int i = 0; i <= d; ++i) {
        double acc = 0.0;
        for (int64_t e = lo * W + threadIdx.x; e < hi * W; e += BS) {
            const int64_t c = e / W;
            const double h = i == 0 ? 1.0 : xc[(int64_t)(i - 1) * n + c];
            acc = fma(h, X[e], acc);
        }
        sm[threadIdx.x] = acc;
        __syncthreads();
        if ((int)threadIdx.x < W) {
            double s = 0.0;
            for (int t = threadIdx.x; t < BS; t += W) s += sm[t];
            part[((int64_t)blockIdx.x * (d + 1) + i) * W + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// alpha (caller order) = X[:,0] - sum_j X[:,1+j] beta_j
__global__ void fe_alpha_kernel(const double *X, const int32_t *perm, int64_t n, int W, int nb, double b0, double b1,
                                double b2, double b3, double *alpha) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const double *row = X + c * W;
        double a = row[0];
        if (nb > 0) a -= row[1] * b0;
        if (nb > 1) a -= row[2] * b1;
        if (nb > 2) a -= row[3] * b2;
        if (nb > 3) a -= row[4] * b3;
        alpha[perm[c]] = a;
    }
}

__global__ void col_out_kernel(const double *X, const int32_t *perm, int64_t n, int W, int nrhs, double *out,
                               int64_t ldo) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n);
        const int64_t c = e - (int64_t)r * n;
        out[(int64_t)r * ldo + perm[c]] = X[c * W + r];
    }
}

inline unsigned grid1(int64_t n) {
    int64_t g = (n + BS - 1) / BS;
    if (g > 65535 * 8) g = 65535 * 8;
    return (unsigned)(g < 1 ? 1 : g);
}

inline unsigned pgrid(int nitems, int cap) {
    return (unsigned)(nitems < cap ? (nitems < 1 ? 1 : nitems) : cap);
}

int pow2ceil(int v) {
    int w = 1;
    while (w < v) w <<= 1;
    return w;
}

template <class T>
mm_status upload_vec(DevBuf &b, const std::vector<T> &v) {
    if (v.empty()) return MM_OK;
    MM_TRY(dev_alloc(b, v.size() * sizeof(T)));
    MM_HIP_TRY(hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return MM_OK;
}

// Right-hand sides of the likelihood solve: column 0 the targets, columns
// 1..l the probes, the padding zero (canonical rows).
__global__ void gather_lml_kernel(const double *y, const double *Z, int64_t ldz, int l, const int32_t *perm,
                                  int64_t n, double *B, int W) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / W;
        const int r = (int)(e - c * W);
        const int64_t i = perm[c];
        B[e] = r == 0 ? y[i] : (r <= l ? Z[(int64_t)(r - 1) * ldz + i] : 0.0);
    }
}

// Inputs of the derivative product: alpha = X[:, 0] and the probes B[:, 1..].
__global__ void lml_mix_kernel(const double *X, const double *B, int64_t n, int W, double *V) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        V[e] = (e % W) == 0 ? X[e] : B[e];
}

// Coordinates of the union of the training points (canonical order) and the
// prediction points, column-major with leading dimension n + m.
__global__ void union_coords_kernel(const double *xc, int64_t n, const double *z, int64_t m, int64_t ldz, int d,
                                    double *U) {
    const int64_t nm = n + m;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nm; i += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < d; ++k) U[k * nm + i] = i < n ? xc[k * n + i] : z[k * ldz + (i - n)];
}

// Unit weights on prediction points j0 .. j0 + b - 1: column r of V (leading
// dimension nm) is the indicator of union point n + j0 + r.
__global__ void unit_cols_kernel(double *V, int64_t nm, int64_t n, int64_t j0, int b) {
    const int64_t total = nm * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / nm, i = e - r * nm;
        V[e] = i == n + j0 + r ? 1.0 : 0.0;
    }
}

// Right-hand sides k_z of the variance solves: the first n rows of the union
// products (the union's first n points are the training points in canonical
// order), point-major with W columns, the padding zero.
__global__ void kz_rhs_kernel(const double *KV, int64_t nm, int64_t n, int b, double *B, int W) {
    const int64_t total = n * W;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / W;
        const int r = (int)(e - c * W);
        B[e] = r < b ? KV[(int64_t)r * nm + c] : 0.0;
    }
}

// Per row block and column: partial sums of X.B, X.D and X.X (three NRED x W
// slabs of part).
__global__ void lml_dots_kernel(const double *X, const double *B, const double *D, int64_t n, int W, double *part) {
    __shared__ double sm[BS];
    int64_t lo, hi;
    row_range(n, blockIdx.x, lo, hi);
    double xb = 0.0, xd = 0.0, xx = 0.0;
    for (int64_t e = lo * W + threadIdx.x; e < hi * W; e += BS) {
        const double x = X[e];
        xb = fma(x, B[e], xb);
        xd = fma(x, D[e], xd);
        xx = fma(x, x, xx);
    }
    block_col_sum(xb, W, sm, part, blockIdx.x);
    block_col_sum(xd, W, sm, part + (size_t)NRED * W, blockIdx.x);
    block_col_sum(xx, W, sm, part + (size_t)2 * NRED * W, blockIdx.x);
}

}  // namespace
}  // namespace mm

using namespace mm;

struct mm_solver_s {
    mm_plan plan = nullptr;
    int W = 1, ncols = 1, fe = 0, d = 1;
    double sigma2 = 0.0, rtol = 0.0;
    DevBuf buf;
    CgDesc desc{};
    DevBuf ws;                       // sweep workspaces (aggregates, partial slabs)
    double *agg = nullptr, *part = nullptr;
    bool batchable = true;           // all passes fit one group: may join batches
    int64_t iters = 0;
    mm_solver_batch self = nullptr;  // batch of one for solitary iterations
    mm_precond pc = nullptr;         // preconditioner (pinned while the solver lives)
    double true_rel = -1.0;          // residual recomputed by the last check (-1: none)
    int64_t checked_iters = -1;      // iterations at that check
    int2 *poll_host = nullptr;       // pinned: the status after each of two chunks in flight
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
};

struct mm_solver_batch_s {
    std::vector<mm_solver> members;
    std::vector<SweepBatch> sweeps;      // one per distinct width among the members
    DevBuf cg_desc, items_blk, items_chunk, items_red, status;
    int n_blk = 0, n_chunk = 0, n_red = 0;  // n_red: (solver, column group) items of the wide members
    DevBuf items_pa, items_pu, items_pc;  // preconditioned members only
    int n_pa = 0, n_pu = 0, n_pc = 0;
    bool plain = false;                  // lone solver too large for a batch workspace
    hipStream_t bs = nullptr;            // private stream for graph capture and replay
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
    int use_graph = 1;
    int grid_cap = 2048;                 // persistent grid of the CG step kernels
    int wg_per_cu = 24;                  // persistent sweep grids: workgroups per compute unit
                                         // (24 measured 1-2% faster than 16 for the d = 2 solves)
};

namespace mm {
namespace {

// Z = P^{-1} R for the preconditioned members (and P = Z when init).
mm_status precond_enqueue(mm_solver_batch b, hipStream_t s, int init) {
    const CgDesc *ds = static_cast<const CgDesc *>(b->cg_desc.ptr);
    hipLaunchKernelGGL(cg_pa_b, dim3(pgrid(b->n_pa, b->grid_cap)), dim3(BS), 0, s, ds,
                       static_cast<const int2 *>(b->items_pa.ptr), b->n_pa);
    hipLaunchKernelGGL(cg_pu_b, dim3(pgrid(b->n_pu, b->grid_cap)), dim3(BS), 0, s, ds,
                       static_cast<const int2 *>(b->items_pu.ptr), b->n_pu);
    hipLaunchKernelGGL(cg_pb_b, dim3(pgrid(b->n_pu, b->grid_cap)), dim3(BS), 0, s, ds,
                       static_cast<const int2 *>(b->items_pu.ptr), b->n_pu);
    hipLaunchKernelGGL(cg_pc_b, dim3(pgrid(b->n_pc, b->grid_cap)), dim3(BS), 0, s, ds,
                       static_cast<const int2 *>(b->items_pc.ptr), b->n_pc, init);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

// Enqueue `iters` CG iterations of every member of the batch on stream s.
mm_status batch_enqueue(mm_solver_batch b, int iters, hipStream_t s) {
    const CgDesc *ds = static_cast<const CgDesc *>(b->cg_desc.ptr);
    const int2 *ib = static_cast<const int2 *>(b->items_blk.ptr);
    const int2 *ic = static_cast<const int2 *>(b->items_chunk.ptr);
    const int nsol = (int)b->members.size();
    for (int it = 0; it < iters; ++it) {
        if (b->plain) {
            mm_solver m = b->members[0];
            MM_TRY(sweep_all(m->plan, m->desc.P, m->desc.Y, m->W, rhs_block(m->plan->kernel, m->d, m->W), s));
        } else {
            for (SweepBatch &sb : b->sweeps) MM_TRY(sweep_batch_run(sb, s));
        }
        const int2 *ir = static_cast<const int2 *>(b->items_red.ptr);
        hipLaunchKernelGGL(cg_apply_b, dim3(pgrid(b->n_blk, b->grid_cap)), dim3(BS), 0, s, ds, ib, b->n_blk);
        if (b->n_red > 0) hipLaunchKernelGGL(cg_reduce_b, dim3(pgrid(b->n_red, 1024)), dim3(BS), 0, s, ds, ir, b->n_red, 0);
        hipLaunchKernelGGL(cg_update_b, dim3(pgrid(b->n_blk, b->grid_cap)), dim3(BS), 0, s, ds, ib, b->n_blk);
        if (b->n_pa > 0) MM_TRY(precond_enqueue(b, s, 0));
        if (b->n_red > 0) hipLaunchKernelGGL(cg_reduce_b, dim3(pgrid(b->n_red, 1024)), dim3(BS), 0, s, ds, ir, b->n_red, 1);
        hipLaunchKernelGGL(cg_dir_b, dim3(pgrid(b->n_chunk, b->grid_cap)), dim3(BS), 0, s, ds, ic, b->n_chunk);
    }
    hipLaunchKernelGGL(cg_collect_b, dim3(pgrid((nsol + BS - 1) / BS, 64)), dim3(BS), 0, s, ds, nsol,
                       static_cast<int2 *>(b->status.ptr));
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

mm_status batch_build(mm_solver_batch b) {
    std::vector<CgDesc> descs;
    std::vector<int2> ib, ic, ir, ipa, ipu, ipc;
    std::vector<int> widths;
    for (size_t k = 0; k < b->members.size(); ++k) {
        mm_solver s = b->members[k];
        if (!s->batchable) {
            if (b->members.size() > 1) {
                set_error("solver %zu is too large to share a batch (its partial sums exceed 16 GiB)", k);
                return MM_ERR_ARG;
            }
            b->plain = true;
        }
        size_t w = 0;
        while (w < widths.size() && widths[w] != s->W) ++w;
        if (w == widths.size()) widths.push_back(s->W);
        descs.push_back(s->desc);
        for (int blk = 0; blk < NRED; ++blk) ib.push_back(make_int2((int)k, blk));
        if (s->W > FUSE_W)
            for (int g = 0; 4 * g < s->W; ++g) ir.push_back(make_int2((int)k, g));
        if (s->desc.rank > 0) {
            for (int blk = 0; blk < PUB; ++blk) ipa.push_back(make_int2((int)k, blk));
            for (int e = 0; e < s->desc.rank * s->W; ++e) ipu.push_back(make_int2((int)k, e));
            for (int blk = 0; blk < NRED; ++blk) ipc.push_back(make_int2((int)k, blk));
        }
        const int64_t nch = (s->desc.n * s->W + CHUNK - 1) / CHUNK;
        for (int64_t c = 0; c < nch; ++c) ic.push_back(make_int2((int)k, (int)c));
    }
    if (descs.empty()) return MM_OK;
    if (!b->plain) {
        b->sweeps.resize(widths.size());
        for (size_t w = 0; w < widths.size(); ++w) {
            std::vector<BatchEntry> ent;
            const mm_solver *first = nullptr;
            for (const mm_solver &s : b->members)
                if (s->W == widths[w]) {
                    if (!first) first = &s;
                    ent.push_back(BatchEntry{s->plan, s->desc.P, s->desc.Y, s->agg, s->part});
                }
            const int WB = rhs_block((*first)->plan->kernel, (*first)->d, widths[w]);
            MM_TRY(sweep_batch_build(ent, widths[w], WB, b->sweeps[w]));
            b->sweeps[w].grid_per_cu = b->wg_per_cu;
            b->sweeps[w].skip_accum = true;  // cg_apply sums the per-pass partials itself
        }
    }
    MM_TRY(upload_vec(b->cg_desc, descs));
    MM_TRY(upload_vec(b->items_blk, ib));
    MM_TRY(upload_vec(b->items_chunk, ic));
    MM_TRY(upload_vec(b->items_red, ir));
    b->n_blk = (int)ib.size();
    b->n_chunk = (int)ic.size();
    b->n_red = (int)ir.size();
    MM_TRY(upload_vec(b->items_pa, ipa));
    MM_TRY(upload_vec(b->items_pu, ipu));
    b->n_pu = (int)ipu.size();
    MM_TRY(upload_vec(b->items_pc, ipc));
    b->n_pa = (int)ipa.size();
    b->n_pc = (int)ipc.size();
    MM_TRY(dev_alloc(b->status, b->members.size() * sizeof(int2)));
    return MM_OK;
}

// Release a batch's executable graph once its last launch (on the batch's
// private stream) has finished: a graph whose branches run side by side owns
// the streams they run on, so it must not go while it executes.
void drop_graph(mm_solver_batch b) {
    if (!b->graph) return;
    if (b->bs) (void)hipStreamSynchronize(b->bs);
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

void batch_free(mm_solver_batch b) {
    drop_graph(b);
    for (SweepBatch &sb : b->sweeps) sweep_batch_free(sb);
    b->sweeps.clear();
    dev_free(b->cg_desc);
    dev_free(b->items_blk);
    dev_free(b->items_chunk);
    dev_free(b->items_red);
    dev_free(b->items_pa);
    dev_free(b->items_pu);
    dev_free(b->items_pc);
    dev_free(b->status);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->bs) (void)hipStreamDestroy(b->bs);
}

}  // namespace

mm_status solver_batch_iterate(mm_solver_batch b, int iters, hipStream_t user) {
    if (b->members.empty() || iters < 1) return MM_OK;
    if (!b->use_graph) {
        MM_TRY(batch_enqueue(b, iters, user));
    } else {
        if (!b->bs) {
            MM_HIP_TRY(hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking));
            MM_HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
            MM_HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
        }
        if (!b->graph || b->graph_iters != iters) {
            drop_graph(b);
            hipGraph_t g = nullptr;
            MM_HIP_TRY(hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal));
            mm_status st = batch_enqueue(b, iters, b->bs);
            hipError_t e = hipStreamEndCapture(b->bs, &g);
            if (st != MM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) {
                set_error("graph capture failed: %s", hipGetErrorString(e));
                return MM_ERR_HIP;
            }
            e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                set_error("graph instantiation failed: %s", hipGetErrorString(e));
                b->graph = nullptr;
                return MM_ERR_HIP;
            }
            b->graph_iters = iters;
        }
        MM_HIP_TRY(hipEventRecord(b->ev_in, user));
        MM_HIP_TRY(hipStreamWaitEvent(b->bs, b->ev_in, 0));
        MM_HIP_TRY(hipGraphLaunch(b->graph, b->bs));
        MM_HIP_TRY(hipEventRecord(b->ev_out, b->bs));
        MM_HIP_TRY(hipStreamWaitEvent(user, b->ev_out, 0));
    }
    for (mm_solver s : b->members) s->iters += iters;
    return MM_OK;
}

}  // namespace mm

// ---------------------------------------------------------------------------
// helpers shared by the C entry points
// ---------------------------------------------------------------------------
namespace {

mm_status check_solve_args(mm_plan plan, double sigma2, double rtol) {
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
    const KParams kp = kparams(plan->kernel, plan->d);
    if (!kp.prod && plan->d >= 2 && kp.P >= 2) {
        set_error("the L1 Matern form with nu >= 3/2 in d >= 2 is not positive definite; use the product form");
        return MM_ERR_NOTPD;
    }
    return MM_OK;
}

// e_1^T log(T) e_1 for the Lanczos matrix T of CG coefficients (Algorithm 2):
// T[k][k] = 1/alpha_k + beta_{k-1}/alpha_{k-1}, T[k][k+1] = sqrt(beta_k)/alpha_k.
// The eigenvalues come from implicit symmetric QR steps with Wilkinson shifts
// on the tridiagonal matrix (Golub & Van Loan, the symmetric tridiagonal QR
// algorithm), accumulating only the first row q of the eigenvector matrix, so
// that e_1^T log(T) e_1 = sum_k q_k^2 log(lambda_k).  False if it does not
// converge or an eigenvalue is not positive.
bool lanczos_logquad(const std::vector<double> &alpha, const std::vector<double> &beta, int m, double *out) {
    std::vector<double> a(m), b(m > 1 ? m - 1 : 1, 0.0), q(m, 0.0);
    for (int k = 0; k < m; ++k) {
        a[k] = 1.0 / alpha[k] + (k > 0 ? beta[k - 1] / alpha[k - 1] : 0.0);
        if (k + 1 < m) b[k] = std::sqrt(beta[k]) / alpha[k];
    }
    q[0] = 1.0;
    const double eps = 2.220446049250313e-16;
    int hi = m - 1, iter = 0;
    while (hi > 0) {
        if (std::fabs(b[hi - 1]) <= eps * (std::fabs(a[hi - 1]) + std::fabs(a[hi]))) {
            b[hi - 1] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(b[lo - 1]) > eps * (std::fabs(a[lo - 1]) + std::fabs(a[lo]))) --lo;
        if (++iter > 200) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2x2 block closer to a[hi]
        const double dd = 0.5 * (a[hi - 1] - a[hi]);
        const double bb = b[hi - 1] * b[hi - 1];
        const double den = dd + std::copysign(std::sqrt(dd * dd + bb), dd);
        const double mu = den != 0.0 ? a[hi] - bb / den : a[hi];
        double x = a[lo] - mu, z = b[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation J = [c s; -s c] on coordinates (k, k+1) with J [x; z] = [r; 0]
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? z / r : 0.0;
            if (k > lo) b[k - 1] = r;
            const double ak = a[k], ak1 = a[k + 1], bk = b[k];
            a[k] = c * c * ak + 2.0 * c * sn * bk + sn * sn * ak1;
            a[k + 1] = sn * sn * ak - 2.0 * c * sn * bk + c * c * ak1;
            b[k] = c * sn * (ak1 - ak) + (c * c - sn * sn) * bk;
            if (k + 1 < hi) {
                x = b[k];
                z = sn * b[k + 1];
                b[k + 1] = c * b[k + 1];
            }
            // Q <- Q J^T on columns k, k+1 (first row only)
            const double qk = q[k], qk1 = q[k + 1];
            q[k] = c * qk + sn * qk1;
            q[k + 1] = -sn * qk + c * qk1;
        }
    }
    double sum = 0.0;
    for (int k = 0; k < m; ++k) {
        if (!(a[k] > 0.0)) return false;
        sum += q[k] * q[k] * std::log(a[k]);
    }
    *out = sum;
    return true;
}

// ||z||^2 e_1^T log(T) e_1 of solver column r from its recorded CG
// coefficients: c the column's scalars (NS), tl the coefficient log
// [iteration][W][alpha, beta].  The iterations that continued past their
// alpha define T (Algorithm 2).  False if T has no positive spectrum.
bool column_logquad(const double *c, const std::vector<double> &tl, int W, int r, double *q, int *msteps,
                    double norm2 = -1.0) {
    const int na = (int)c[6];                  // alphas recorded
    const int m = c[5] != 0.0 ? na : na - 1;   // iterations that continued
    // ||z||^2 of the probe, or z^T P^{-1} z for the preconditioned estimator
    const double znorm2 = norm2 >= 0.0 ? norm2 : c[4] * c[4];
    *q = 0.0;
    *msteps = m > 0 ? m : na;
    if (m >= 1) {
        std::vector<double> al(m), be(m, 0.0);
        for (int k = 0; k < m; ++k) {
            al[k] = tl[((size_t)k * W + r) * 2];
            if (k + 1 < m) be[k] = tl[((size_t)k * W + r) * 2 + 1];
        }
        if (!lanczos_logquad(al, be, m, q)) return false;
        *q *= znorm2;
    } else if (na == 1) {
        // solved exactly in one step: T = [1 / alpha_1]
        *q = znorm2 * std::log(1.0 / tl[(size_t)r * 2]);
    }
    return true;
}

template <class F>
mm_status solver_new(mm_plan plan, int ncols, int fe, double sigma2, double rtol, mm_precond pc, hipStream_t s,
                     F &&fill, mm_solver *out, int tlog_cap = 0) {
    const int64_t n = plan->n;
    const int R = rhs_block(plan->kernel, plan->d, ncols);
    const int W = pow2ceil(ncols > R ? ncols : R);
    const int rank = pc ? pc->rank : 0;
    if (pc && pc->plan != plan) {
        set_error("the preconditioner was built for another plan");
        return MM_ERR_ARG;
    }
    if (rank > 0 && W > PC_MAXW) {
        set_error("a preconditioned solver takes at most %d columns (got %d)", PC_MAXW, W);
        return MM_ERR_ARG;
    }
    // Woodbury factors for this noise level: Rinv = inverse of the Cholesky factor
    // of I + L^T L / sigma2 (host, rank x rank)
    std::vector<double> rinv, minv;
    if (rank > 0) {
        const int r = rank;
        std::vector<double> M((size_t)r * r), C((size_t)r * r, 0.0);
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) M[i * r + j] = (i == j ? 1.0 : 0.0) + pc->gram[i * r + j] / sigma2;
        for (int j = 0; j < r; ++j) {
            double dj = M[j * r + j];
            for (int k = 0; k < j; ++k) dj -= C[j * r + k] * C[j * r + k];
            if (!(dj > 0.0)) {
                set_error("preconditioner Gram factor is not positive definite");
                return MM_ERR_NOTPD;
            }
            C[j * r + j] = std::sqrt(dj);
            for (int i = j + 1; i < r; ++i) {
                double t = M[i * r + j];
                for (int k = 0; k < j; ++k) t -= C[i * r + k] * C[j * r + k];
                C[i * r + j] = t / C[j * r + j];
            }
        }
        rinv.assign((size_t)r * r, 0.0);  // forward substitution on the identity
        for (int c = 0; c < r; ++c)
            for (int i = c; i < r; ++i) {
                double t = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) t -= C[i * r + k] * rinv[k * r + c];
                rinv[i * r + c] = t / C[i * r + i];
            }
        // M^{-1} = Rinv^T Rinv: symmetric positive definite by construction
        minv.assign((size_t)r * r, 0.0);
        for (int i = 0; i < r; ++i)
            for (int j = 0; j <= i; ++j) {
                double t = 0.0;
                for (int k = i; k < r; ++k) t += rinv[k * r + i] * rinv[k * r + j];
                minv[i * r + j] = t;
                minv[j * r + i] = t;
            }
    }
    mm_solver sv = new (std::nothrow) mm_solver_s();
    if (!sv) {
        set_error("host allocation failed");
        return MM_ERR_NOMEM;
    }
    sv->plan = plan;
    sv->W = W;
    sv->ncols = ncols;
    sv->fe = fe;
    sv->d = plan->d;
    sv->sigma2 = sigma2;
    sv->rtol = rtol;
    const size_t vec = (size_t)n * W;
    size_t agg_b = 0, part_b = 0;
    sv->batchable = sweep_batch_bytes(plan, W, &agg_b, &part_b);
    agg_b = (agg_b + 255) & ~size_t(255);
    const size_t pcd = rank > 0 ? vec + (size_t)NRED * W + (size_t)PUB * rank * W + (size_t)2 * rank * W +
                                      (size_t)rank * rank
                                : 0;
    const size_t tld = (size_t)tlog_cap * W * 2;
    mm_status st =
        dev_alloc(sv->buf, (6 * vec + (size_t)NRED * W * 8 + (size_t)W * NS + 8 + pcd + tld) * sizeof(double));
    if (st == MM_OK) {
        if (sv->batchable) {
            st = dev_alloc(sv->ws, agg_b + part_b);
            if (st == MM_OK) {
                sv->agg = static_cast<double *>(sv->ws.ptr);
                sv->part = reinterpret_cast<double *>(static_cast<char *>(sv->ws.ptr) + agg_b);
            }
        } else {
            st = ensure_work(plan, W);  // a lone solver sweeps in the plan's own work buffers
        }
    }
    if (st != MM_OK) {
        dev_free(sv->ws);
        dev_free(sv->buf);
        delete sv;
        return st;
    }
    double *base = static_cast<double *>(sv->buf.ptr);
    CgDesc &d = sv->desc;
    double *Bm = base;
    d.B = Bm;
    d.X = base + vec;
    d.R = base + 2 * vec;
    d.P = base + 3 * vec;
    d.Q = base + 4 * vec;
    d.Y = base + 5 * vec;
    d.part = base + 6 * vec;
    d.part2 = d.part + (size_t)NRED * W;
    d.red = d.part + (size_t)2 * NRED * W;
    d.sc = d.part + (size_t)NRED * W * 8;
    d.flags = reinterpret_cast<int *>(d.sc + (size_t)W * NS);
    if (tlog_cap > 0) {
        d.tlog = d.sc + (size_t)W * NS + 8 + pcd;
        d.tlog_cap = tlog_cap;
    }
    if (rank > 0) {
        double *q = d.sc + (size_t)W * NS + 8;
        d.Z = q;
        d.part_rz = q + vec;
        d.part_u = d.part_rz + (size_t)NRED * W;
        d.wv = d.part_u + (size_t)PUB * rank * W;
        d.ub = d.wv + (size_t)rank * W;
        double *rv = d.ub + (size_t)rank * W;
        d.Minv = rv;
        d.Lpc = static_cast<const double *>(pc->L.ptr);
        d.kmax = pc->kmax;
        d.rank = rank;
        if (hipMemcpyAsync(rv, minv.data(), minv.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            dev_free(sv->ws);
            dev_free(sv->buf);
            delete sv;
            set_error("copy of the preconditioner factors failed");
            return MM_ERR_HIP;
        }
        sv->pc = pc;
    }
    d.slabs = sv->part;
    d.nslab = sv->batchable ? (int)plan->passes.size() : -1;
    d.n = n;
    d.W = W;
    d.ncols = ncols;
    d.s2 = plan->kernel.outputscale2;
    d.sigma2 = sigma2;
    d.rtol = rtol;
    fill(Bm, W);
    // a batch of one for solitary iterations; the init runs through the batched kernels too
    mm_solver_batch b = new (std::nothrow) mm_solver_batch_s();
    if (!b) {
        dev_free(sv->ws);
        dev_free(sv->buf);
        delete sv;
        set_error("host allocation failed");
        return MM_ERR_NOMEM;
    }
    b->members.push_back(sv);
    // solitary iterations are enqueued directly: replaying captured chunks of 8
    // iterations measured 4.6% slower per iteration on the headline solve
    b->use_graph = 0;
    st = batch_build(b);
    if (st == MM_OK) {
        const CgDesc *ds = static_cast<const CgDesc *>(b->cg_desc.ptr);
        hipLaunchKernelGGL(cg_init_b, dim3(pgrid(b->n_blk, 2048)), dim3(BS), 0, s, ds,
                           static_cast<const int2 *>(b->items_blk.ptr), b->n_blk);
        if (b->n_pa > 0) st = precond_enqueue(b, s, 1);  // z0 = P^{-1} r0, p0 = z0
        hipLaunchKernelGGL(cg_init_scalars_b, dim3(1), dim3(BS), 0, s, ds, 1);
        if (hipGetLastError() != hipSuccess) {
            set_error("solver initialisation launch failed");
            st = MM_ERR_HIP;
        }
    }
    if (st != MM_OK) {
        batch_free(b);
        delete b;
        dev_free(sv->ws);
        dev_free(sv->buf);
        delete sv;
        return st;
    }
    sv->self = b;
    plan->npins++;
    if (sv->pc) sv->pc->npins++;
    plan->last_stream = s;
    *out = sv;
    return MM_OK;
}

// Host-side convergence summary from the device scalars (synchronises s).
mm_status solver_summary(mm_solver sv, hipStream_t s, int *conv, int *brk, double *relmax, mm_solve_info *info) {
    std::vector<double> hsc((size_t)sv->W * NS);
    int fl[2] = {0, 0};
    MM_HIP_TRY(hipMemcpyAsync(hsc.data(), sv->desc.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipMemcpyAsync(fl, sv->desc.flags, sizeof fl, hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    int c = 0;
    double rel = 0.0, itmax = 0.0;
    for (int r = 0; r < sv->ncols; ++r) {
        const double bn = hsc[r * NS + 4];
        const double rn = hsc[r * NS + 7];
        const double rr = bn > 0.0 ? rn / bn : 0.0;
        if (rr > rel) rel = rr;
        if (hsc[r * NS + 6] > itmax) itmax = hsc[r * NS + 6];
        if (bn == 0.0 || rr <= sv->rtol) ++c;
    }
    *conv = c;
    *brk = fl[1];
    *relmax = rel;
    if (info) {
        info->iters = (int32_t)itmax;
        info->converged_cols = c;
        info->relres_max = rel;
    }
    return MM_OK;
}

// Iterate a single solver until convergence, breakdown or maxit.
// The host reads the convergence status of every chunk of 8 iterations while the
// next chunk is already queued, so the stream does not drain at each check.  A
// chunk queued after the last active column has met its tolerance changes
// nothing: converged columns are frozen (no update, their iteration counts stay).
mm_status solver_run(mm_solver sv, int maxit, hipStream_t s) {
    const int check_every = 8;
    if (sv->iters >= maxit) return MM_OK;
    if (!sv->poll_host) {
        MM_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&sv->poll_host), 2 * sizeof(int2), hipHostMallocDefault));
        for (hipEvent_t &e : sv->poll_ev) MM_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    auto enqueue = [&](int slot) -> mm_status {
        const int k = (int)(maxit - sv->iters < check_every ? maxit - sv->iters : check_every);
        MM_TRY(solver_batch_iterate(sv->self, k, s));
        MM_HIP_TRY(hipMemcpyAsync(sv->poll_host + slot, sv->self->status.ptr, sizeof(int2), hipMemcpyDeviceToHost, s));
        MM_HIP_TRY(hipEventRecord(sv->poll_ev[slot], s));
        return MM_OK;
    };
    int slot = 0;  // the oldest chunk whose status is not read yet
    MM_TRY(enqueue(slot));
    for (;;) {
        const bool ahead = sv->iters < maxit;
        if (ahead) MM_TRY(enqueue(slot ^ 1));
        MM_HIP_TRY(hipEventSynchronize(sv->poll_ev[slot]));
        const int2 st = sv->poll_host[slot];
        if (st.y || st.x == 0 || !ahead) break;
        slot ^= 1;
    }
    MM_HIP_TRY(hipStreamSynchronize(s));
    return MM_OK;
}

// GLS estimate beta = (H^T A^-1 H)^{-1} H^T A^-1 y from the solved columns
// [A^-1 y, A^-1 H] (Section 3.2), on the host: hb[0..d].
mm_status solver_gls(mm_solver sv, double *hb, hipStream_t s) {
    mm_plan plan = sv->plan;
    const int64_t n = plan->n;
    const int d = plan->d;
    const int W = sv->W;
    const double *xc = static_cast<const double *>(plan->xc.ptr);
    const int nb = d + 1;
    double *part = sv->desc.part;
    hipLaunchKernelGGL(fe_gram_kernel, dim3(NRED), dim3(BS), 0, s, sv->desc.X, xc, n, d, W, part);
    std::vector<double> hp((size_t)NRED * nb * W);
    MM_HIP_TRY(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    std::vector<double> HX((size_t)nb * W, 0.0);  // HX[i*W + j] = h_i^T X_j
    for (int b = 0; b < NRED; ++b)
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < W; ++j) HX[i * W + j] += hp[((size_t)b * nb + i) * W + j];
    double G[4][4], g[4], Lm[4][4] = {{0}}, w[4];
    for (int i = 0; i < 4; ++i) hb[i] = 0.0;
    for (int i = 0; i < nb; ++i) {
        g[i] = HX[i * W + 0];
        for (int j = 0; j < nb; ++j) G[i][j] = 0.5 * (HX[i * W + 1 + j] + HX[j * W + 1 + i]);
    }
    for (int j = 0; j < nb; ++j) {
        double dsum = G[j][j];
        for (int k = 0; k < j; ++k) dsum -= Lm[j][k] * Lm[j][k];
        if (!(dsum > 0.0)) {
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
    return MM_OK;
}

// GLS from the solved columns and alpha = A^-1 y - (A^-1 H) beta in caller order.
mm_status solver_output(mm_solver sv, double *alpha, double *beta, hipStream_t s) {
    mm_plan plan = sv->plan;
    const int64_t n = plan->n;
    const int W = sv->W;
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    if (!sv->fe) {
        hipLaunchKernelGGL(col_out_kernel, dim3(grid1(n)), dim3(BS), 0, s, sv->desc.X, perm, n, W, 1, alpha, n);
        MM_HIP_TRY(hipGetLastError());
        return MM_OK;
    }
    const int nb = plan->d + 1;
    double hb[4];
    MM_TRY(solver_gls(sv, hb, s));
    for (int i = 0; i < nb; ++i) beta[i] = hb[i];
    hipLaunchKernelGGL(fe_alpha_kernel, dim3(grid1(n)), dim3(BS), 0, s, sv->desc.X, perm, n, W, nb, hb[0], hb[1],
                       hb[2], hb[3], alpha);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

// The residual of the current iterate recomputed with a fresh product (the
// recurrence residual of Algorithm 2 drifts from it, and with fixed effects
// the solved columns combine into y - H beta - A alpha = r_0 - sum_i beta_i r_i),
// then a restart from it: R = B - A X, P = R (P^{-1} R with a preconditioner),
// the scalars recomputed.  *rel_out is |y - H beta - A alpha| / |y| with fixed
// effects, else the largest |b_j - A x_j| / |b_j|; *passed is rel_out <= rtol,
// and then every column is frozen.  Otherwise, with tighten and every column
// converged by the recurrence, the column tolerances shrink by
// 0.5 rtol / rel_out (within [0.05, 0.5]: the columns that missed, or all
// of them with fixed effects), so further iterations continue the solve.
mm_status solver_check(mm_solver sv, hipStream_t s, bool tighten, int *passed, double *rel_out) {
    mm_plan plan = sv->plan;
    mm_solver_batch b = sv->self;
    const int64_t n = plan->n;
    const int W = sv->W;
    CgDesc &d = sv->desc;
    std::vector<double> hsc((size_t)W * NS);
    MM_HIP_TRY(hipMemcpyAsync(hsc.data(), d.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    bool all_conv = true;
    for (int r = 0; r < sv->ncols; ++r)
        if (hsc[r * NS + 5] != 0.0) all_conv = false;
    double hb[4] = {0.0, 0.0, 0.0, 0.0};
    const int nb = sv->fe ? plan->d + 1 : 0;
    if (sv->fe) MM_TRY(solver_gls(sv, hb, s));
    // Q = A X through the solver's own product (its sweeps read P)
    MM_HIP_TRY(hipMemcpyAsync(d.P, d.X, (size_t)n * W * sizeof(double), hipMemcpyDeviceToDevice, s));
    const CgDesc *ds = static_cast<const CgDesc *>(b->cg_desc.ptr);
    const int2 *ib = static_cast<const int2 *>(b->items_blk.ptr);
    if (b->plain) {
        MM_TRY(sweep_all(plan, d.P, d.Y, W, rhs_block(plan->kernel, sv->d, W), s));
    } else {
        for (SweepBatch &sb : b->sweeps) MM_TRY(sweep_batch_run(sb, s));
    }
    hipLaunchKernelGGL(cg_apply_b, dim3(pgrid(b->n_blk, b->grid_cap)), dim3(BS), 0, s, ds, ib, b->n_blk);
    hipLaunchKernelGGL(cg_resid_b, dim3(pgrid(b->n_blk, b->grid_cap)), dim3(BS), 0, s, ds, ib, b->n_blk, nb, hb[0],
                       hb[1], hb[2], hb[3]);
    std::vector<double> hr((size_t)NRED * W), hc(NRED);
    MM_HIP_TRY(hipMemcpyAsync(hr.data(), d.part2, hr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipMemcpyAsync(hc.data(), d.part, hc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    std::vector<double> rn(W, 0.0);
    double comb = 0.0;
    for (int blk = 0; blk < NRED; ++blk) {
        for (int r = 0; r < W; ++r) rn[r] += hr[(size_t)blk * W + r];
        comb += hc[blk];
    }
    std::vector<double> rel(W, 0.0), tol(W);
    double worst = 0.0;
    for (int r = 0; r < W; ++r) {
        const double bn = hsc[r * NS + 4];
        rel[r] = bn > 0.0 ? std::sqrt(rn[r]) / bn : 0.0;
        tol[r] = hsc[r * NS + 10];
        if (r < sv->ncols && rel[r] > worst) worst = rel[r];
    }
    const double bn0 = hsc[4];
    const double trel = sv->fe ? (bn0 > 0.0 ? std::sqrt(comb) / bn0 : 0.0) : worst;
    const bool ok = trel <= sv->rtol;
    if (!ok && tighten && all_conv) {
        double f = 0.5 * sv->rtol / trel;
        f = f < 0.05 ? 0.05 : (f > 0.5 ? 0.5 : f);
        for (int r = 0; r < sv->ncols; ++r)
            if (sv->fe || rel[r] > sv->rtol) tol[r] *= f;
    }
    if (b->n_pa > 0) {
        MM_TRY(precond_enqueue(b, s, 1));  // Z = P^{-1} R, P = Z, partial r.z
    } else {
        hipLaunchKernelGGL(cg_restart_dir_b, dim3(pgrid(b->n_chunk, b->grid_cap)), dim3(BS), 0, s, ds,
                           static_cast<const int2 *>(b->items_chunk.ptr), b->n_chunk);
    }
    double *tstage = d.part + (size_t)4 * NRED * W;  // unused part of the partial-sum area
    MM_HIP_TRY(hipMemcpyAsync(tstage, tol.data(), W * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(cg_restart_scalars_b, dim3(1), dim3(BS), 0, s, ds, static_cast<const double *>(tstage),
                       ok ? 1 : 0);
    MM_HIP_TRY(hipGetLastError());
    MM_HIP_TRY(hipStreamSynchronize(s));
    sv->true_rel = trel;
    sv->checked_iters = sv->iters;
    if (passed) *passed = ok ? 1 : 0;
    if (rel_out) *rel_out = trel;
    return MM_OK;
}

mm_status status_of(int conv, int ncols, int brk, int iters, double rel, double true_rel = -1.0,
                    double rtol = 0.0) {
    if (brk) {
        set_error("conjugate gradients broke down (p^T A p <= 0)");
        return MM_ERR_BREAKDOWN;
    }
    if (conv < ncols) {
        set_error("conjugate gradients did not reach rtol in %d iterations (relres %.3e)", iters, rel);
        return MM_ERR_NOCONV;
    }
    if (true_rel > rtol) {
        set_error("the recomputed residual %.3e misses rtol %.3e after %d iterations", true_rel, rtol, iters);
        return MM_ERR_NOCONV;
    }
    return MM_OK;
}

// Iterate until the recurrence converges, then check the recomputed residual;
// a miss tightens the column tolerances and the solve continues from the
// recomputed residual (at most MAX_CHECKS checks, within maxit iterations).
constexpr int MAX_CHECKS = 8;

mm_status solver_solve(mm_solver sv, int maxit, hipStream_t s) {
    for (int chk = 0;; ++chk) {
        MM_TRY(solver_run(sv, maxit, s));
        int conv = 0, brk = 0;
        double rel = 0.0;
        MM_TRY(solver_summary(sv, s, &conv, &brk, &rel, nullptr));
        if (brk || conv < sv->ncols) return MM_OK;  // breakdown or maxit: finish reports it
        const bool more = chk + 1 < MAX_CHECKS && sv->iters < maxit;
        int passed = 0;
        double tr = 0.0;
        MM_TRY(solver_check(sv, s, more, &passed, &tr));
        if (passed || !more) return MM_OK;
    }
}

}  // namespace

extern "C" {

size_t mm_solver_footprint_bytes(int64_t n, int32_t d, int32_t fixed_effects, const mm_kernel *kernel) {
    if (n < 1 || d < 1 || d > 3 || !kernel) return 0;
    if (kernel->two_nu != 1 && kernel->two_nu != 3 && kernel->two_nu != 5) return 0;
    const int ncols = fixed_effects ? d + 2 : 1;
    const int R = rhs_block(*kernel, d, ncols);
    const int W = pow2ceil(ncols > R ? ncols : R);
    int L = 0;
    while ((int64_t(1) << L) < n) ++L;
    const int npass = n < 2 ? 0 : (d == 1 ? 1 : (d == 2 ? L : L * (L + 1) / 2));
    size_t b = ((size_t)6 * n * W + (size_t)NRED * W * 8 + (size_t)W * NS + 8) * sizeof(double);
    size_t agg_b = 0, part_b = 0;
    if (sweep_batch_bytes_n(n, d, *kernel, npass, W, &agg_b, &part_b)) {
        b += ((agg_b + 255) & ~size_t(255)) + part_b;
    } else {  // a lone solver sweeps in the plan's work buffers
        b += 2 * (size_t)n * W * sizeof(double) + sweep_agg_bytes(n, d, W, *kernel) + sweep_part_bytes(n, npass, W);
    }
    // work tables of a batch: sweep items (at most three per pass, tile of 256 and
    // column block) and the vector-update items
    const int64_t ntile = (n + 127) / 128;
    b += (size_t)3 * (npass + 1) * (ntile + 1) * W * 16 + (size_t)NRED * 8 + (size_t)(n * W / CHUNK + 1) * 8;
    return b;
}

namespace {
mm_status solver_create_impl(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                             mm_precond pc, void *stream, mm_solver *out) {
    if (!out) {
        set_error("out is NULL");
        return MM_ERR_ARG;
    }
    *out = nullptr;
    MM_TRY(check_solve_args(plan, sigma2, rtol));
    if (!y) {
        set_error("y is NULL");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ncols = fixed_effects ? plan->d + 2 : 1;
    return solver_new(plan, ncols, fixed_effects ? 1 : 0, sigma2, rtol, pc, s,
                      [&](double *B, int W) {
                          hipLaunchKernelGGL(fe_rhs_kernel, dim3(grid1(plan->n)), dim3(BS), 0, s, y,
                                             static_cast<const int32_t *>(plan->perm.ptr),
                                             static_cast<const double *>(plan->xc.ptr), plan->n, plan->d,
                                             fixed_effects ? 1 : 0, W, B);
                      },
                      out);
}
}  // namespace

mm_status mm_solver_create(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                           void *stream, mm_solver *out) {
    clear_error();
    return solver_create_impl(plan, y, sigma2, fixed_effects, rtol, nullptr, stream, out);
}

mm_status mm_solver_create_pc(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                              mm_precond pc, void *stream, mm_solver *out) {
    clear_error();
    return solver_create_impl(plan, y, sigma2, fixed_effects, rtol, pc, stream, out);
}

mm_status mm_solver_iterate(mm_solver solver, int32_t iters, void *stream) {
    clear_error();
    if (!solver || iters < 0) {
        set_error("solver is NULL or iters < 0");
        return MM_ERR_ARG;
    }
    return solver_batch_iterate(solver->self, iters, static_cast<hipStream_t>(stream));
}

mm_status mm_solver_poll(mm_solver solver, int32_t *active_cols, int32_t *breakdown, mm_solve_info *info,
                         void *stream) {
    clear_error();
    if (!solver) {
        set_error("solver is NULL");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int conv = 0, brk = 0;
    double rel = 0.0;
    MM_TRY(solver_summary(solver, s, &conv, &brk, &rel, info));
    if (active_cols) *active_cols = solver->ncols - conv;
    if (breakdown) *breakdown = brk;
    return MM_OK;
}

mm_status mm_solver_finish(mm_solver solver, double *alpha, double *beta, mm_solve_info *info, void *stream) {
    clear_error();
    if (!solver || !alpha || (solver->fe && !beta)) {
        set_error("solver and alpha (and beta with fixed effects) must be non-NULL");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int conv = 0, brk = 0;
    double rel = 0.0;
    mm_solve_info inf{};
    MM_TRY(solver_summary(solver, s, &conv, &brk, &rel, &inf));
    if (!brk && solver->checked_iters != solver->iters) {
        // the residual of the returned iterate, recomputed (no tightening)
        MM_TRY(solver_check(solver, s, false, nullptr, nullptr));
        MM_TRY(solver_summary(solver, s, &conv, &brk, &rel, &inf));
    }
    inf.true_relres = brk ? -1.0 : solver->true_rel;
    if (info) *info = inf;
    MM_TRY(solver_output(solver, alpha, beta, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    return status_of(conv, solver->ncols, brk, inf.iters, rel, inf.true_relres, solver->rtol);
}

mm_status mm_solver_check(mm_solver solver, int32_t tighten, int32_t *passed, double *true_relres, void *stream) {
    clear_error();
    if (!solver) {
        set_error("solver is NULL");
        return MM_ERR_ARG;
    }
    int ok = 0;
    double tr = 0.0;
    MM_TRY(solver_check(solver, static_cast<hipStream_t>(stream), tighten != 0, &ok, &tr));
    if (passed) *passed = ok;
    if (true_relres) *true_relres = tr;
    return MM_OK;
}

mm_status mm_solver_destroy(mm_solver solver) {
    if (!solver) return MM_OK;
    (void)hipDeviceSynchronize();
    if (solver->self) {
        batch_free(solver->self);
        delete solver->self;
    }
    solver->plan->npins--;
    if (solver->pc) solver->pc->npins--;
    for (hipEvent_t e : solver->poll_ev)
        if (e) (void)hipEventDestroy(e);
    if (solver->poll_host) (void)hipHostFree(solver->poll_host);
    dev_free(solver->ws);
    dev_free(solver->buf);
    delete solver;
    return MM_OK;
}

mm_status mm_solver_batch_create(mm_solver *solvers, int32_t count, int32_t use_graph, mm_solver_batch *out) {
    clear_error();
    if (!out || !solvers || count < 1) {
        set_error("solvers, count >= 1 and out are required");
        return MM_ERR_ARG;
    }
    *out = nullptr;
    mm_solver_batch b = new (std::nothrow) mm_solver_batch_s();
    if (!b) {
        set_error("host allocation failed");
        return MM_ERR_NOMEM;
    }
    for (int i = 0; i < count; ++i) {
        if (!solvers[i]) {
            delete b;
            set_error("solver %d is NULL", i);
            return MM_ERR_ARG;
        }
        b->members.push_back(solvers[i]);
    }
    b->use_graph = use_graph ? 1 : 0;
    mm_status st = batch_build(b);
    if (st != MM_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return MM_OK;
}

mm_status mm_solver_batch_set_schedule(mm_solver_batch batch, int32_t sweep_wg_per_cu, int32_t cg_grid) {
    clear_error();
    if (!batch || sweep_wg_per_cu < 1 || cg_grid < 1) {
        set_error("batch is NULL or schedule out of range");
        return MM_ERR_ARG;
    }
    batch->wg_per_cu = sweep_wg_per_cu;
    for (SweepBatch &sb : batch->sweeps) sb.grid_per_cu = sweep_wg_per_cu;
    batch->grid_cap = cg_grid;
    drop_graph(batch);
    return MM_OK;
}

mm_status mm_solver_batch_iterate(mm_solver_batch batch, int32_t iters, void *stream) {
    clear_error();
    if (!batch || iters < 0) {
        set_error("batch is NULL or iters < 0");
        return MM_ERR_ARG;
    }
    return solver_batch_iterate(batch, iters, static_cast<hipStream_t>(stream));
}

mm_status mm_solver_batch_poll(mm_solver_batch batch, int32_t *active, void *stream) {
    clear_error();
    if (!batch || !active) {
        set_error("batch and active are required");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int2> st(batch->members.size());
    MM_HIP_TRY(hipMemcpyAsync(st.data(), batch->status.ptr, st.size() * sizeof(int2), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    for (size_t k = 0; k < st.size(); ++k) active[k] = st[k].y ? -1 : st[k].x;
    return MM_OK;
}

mm_status mm_solver_batch_destroy(mm_solver_batch batch) {
    if (!batch) return MM_OK;
    (void)hipDeviceSynchronize();
    batch_free(batch);
    delete batch;
    return MM_OK;
}

namespace {
mm_status pcg_impl(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol, int32_t maxit,
                   mm_precond pc, double *alpha, double *beta, mm_solve_info *info, void *stream) {
    MM_TRY(check_solve_args(plan, sigma2, rtol));
    if (!y || !alpha) {
        set_error("y and alpha must be non-NULL");
        return MM_ERR_ARG;
    }
    if (fixed_effects && !beta) {
        set_error("beta must be non-NULL when fixed_effects is set");
        return MM_ERR_ARG;
    }
    if (maxit < 1) {
        set_error("maxit must be >= 1");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    mm_solver sv = nullptr;
    MM_TRY(solver_create_impl(plan, y, sigma2, fixed_effects, rtol, pc, stream, &sv));
    mm_status st = solver_solve(sv, maxit, s);
    if (st == MM_OK) st = mm_solver_finish(sv, alpha, beta, info, stream);
    if (st != MM_OK && st != MM_ERR_NOCONV && st != MM_ERR_BREAKDOWN) {
        mm_solver_destroy(sv);
        return st;
    }
    std::string msg = last_error_str();
    mm_solver_destroy(sv);
    if (st != MM_OK) set_error("%s", msg.c_str());
    return st;
}
}  // namespace

mm_status gp_cg_solve(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                      int32_t maxit, double *alpha, double *beta, mm_solve_info *info, void *stream) {
    clear_error();
    return pcg_impl(plan, y, sigma2, fixed_effects, rtol, maxit, nullptr, alpha, beta, info, stream);
}

mm_status gp_pcg_solve(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                       int32_t maxit, mm_precond pc, double *alpha, double *beta, mm_solve_info *info, void *stream) {
    clear_error();
    return pcg_impl(plan, y, sigma2, fixed_effects, rtol, maxit, pc, alpha, beta, info, stream);
}

mm_status mm_lanczos_logquad(const double *alpha, const double *beta, int32_t m, double *out) {
    clear_error();
    if (!alpha || !out || m < 1 || (m > 1 && !beta)) {
        set_error("alpha, out (and beta for m > 1) are required, m >= 1");
        return MM_ERR_ARG;
    }
    std::vector<double> al(alpha, alpha + m), be(m, 0.0);
    for (int k = 0; k + 1 < m; ++k) be[k] = beta[k];
    double q = 0.0;
    if (!lanczos_logquad(al, be, m, &q)) {
        set_error("the Lanczos matrix did not converge to a positive spectrum");
        return MM_ERR_BREAKDOWN;
    }
    *out = q;
    return MM_OK;
}

mm_status gp_logdet(mm_plan plan, double sigma2, const double *Zc, int64_t ldz, int32_t nprobes, int32_t steps,
                    double rtol, double *logdet, double *quad, int32_t *lanczos_steps, void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol > 0.0 ? rtol : 1.0));
    if (!Zc || !logdet) {
        set_error("Z and logdet must be non-NULL");
        return MM_ERR_ARG;
    }
    if (nprobes < 1 || nprobes > 64 || steps < 1 || ldz < plan->n || !(rtol >= 0.0)) {
        set_error("nprobes in [1, 64], steps >= 1, ldz >= n and rtol >= 0 are required");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    mm_solver sv = nullptr;
    MM_TRY(solver_new(plan, nprobes, 0, sigma2, rtol > 0.0 ? rtol : 1e-300, nullptr, s,
                      [&](double *B, int W) {
                          hipLaunchKernelGGL(gather_cols_kernel, dim3(grid1(plan->n * W)), dim3(BS), 0, s, Zc, ldz,
                                             nprobes, static_cast<const int32_t *>(plan->perm.ptr), plan->n, B, W);
                      },
                      &sv, steps));
    mm_status st = solver_run(sv, steps, s);
    const int W = sv->W;
    std::vector<double> hsc((size_t)W * NS), tl((size_t)steps * W * 2);
    if (st == MM_OK) {
        if (hipMemcpyAsync(hsc.data(), sv->desc.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipMemcpyAsync(tl.data(), sv->desc.tlog, tl.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("HIP error reading the Lanczos coefficients");
            st = MM_ERR_HIP;
        }
    }
    double sum = 0.0;
    for (int r = 0; r < nprobes && st == MM_OK; ++r) {
        double q = 0.0;
        int ms = 0;
        if (!column_logquad(hsc.data() + (size_t)r * NS, tl, W, r, &q, &ms)) {
            set_error("probe %d: the Lanczos matrix did not converge to a positive spectrum", r);
            st = MM_ERR_BREAKDOWN;
            break;
        }
        if (quad) quad[r] = q;
        if (lanczos_steps) lanczos_steps[r] = ms;
        sum += q;
    }
    if (st == MM_OK) *logdet = sum / nprobes;
    std::string msg = last_error_str();
    mm_solver_destroy(sv);
    if (st != MM_OK) set_error("%s", msg.c_str());
    return st;
}

mm_status gp_logdet_pc(mm_plan plan, double sigma2, mm_precond pc, const double *G1, int64_t ldg1, const double *G2,
                       int64_t ldg2, int32_t nprobes, int32_t steps, double rtol, double *logdet, double *quad,
                       int32_t *lanczos_steps, double *logdet_precond, void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol > 0.0 ? rtol : 1.0));
    if (!pc || !G2 || !logdet || (pc->rank > 0 && !G1)) {
        set_error("pc, G2 and logdet (and G1 for a preconditioner of rank > 0) must be non-NULL");
        return MM_ERR_ARG;
    }
    if (pc->plan != plan) {
        set_error("the preconditioner was built for another plan");
        return MM_ERR_ARG;
    }
    if (nprobes < 1 || nprobes > 64 || steps < 1 || ldg2 < plan->n || (pc->rank > 0 && ldg1 < pc->rank) ||
        !(rtol >= 0.0)) {
        set_error("nprobes in [1, 64], steps >= 1, ldg1 >= rank, ldg2 >= n and rtol >= 0 are required");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = plan->n;
    const int rank = pc->rank;
    // log det P = n log sigma2 + log det(I + L^T L / sigma2) (Sylvester), by Cholesky on the host
    double ldp = (double)n * std::log(sigma2);
    {
        const int r = rank;
        std::vector<double> C((size_t)r * r, 0.0);
        for (int j = 0; j < r; ++j) {
            double dj = 1.0 + pc->gram[(size_t)j * r + j] / sigma2;
            for (int k = 0; k < j; ++k) dj -= C[(size_t)j * r + k] * C[(size_t)j * r + k];
            if (!(dj > 0.0)) {
                set_error("preconditioner Gram factor is not positive definite");
                return MM_ERR_NOTPD;
            }
            C[(size_t)j * r + j] = std::sqrt(dj);
            ldp += 2.0 * std::log(C[(size_t)j * r + j]);
            for (int i = j + 1; i < r; ++i) {
                double t = pc->gram[(size_t)i * r + j] / sigma2;
                for (int k = 0; k < j; ++k) t -= C[(size_t)i * r + k] * C[(size_t)j * r + k];
                C[(size_t)i * r + j] = t / C[(size_t)j * r + j];
            }
        }
    }
    const double sigma = std::sqrt(sigma2);
    double sum = 0.0;
    mm_status st = MM_OK;
    // preconditioned solvers take at most PC_MAXW columns: blocks of probes
    for (int r0 = 0; r0 < nprobes && st == MM_OK; r0 += PC_MAXW) {
        const int nb = nprobes - r0 < PC_MAXW ? nprobes - r0 : PC_MAXW;
        mm_solver sv = nullptr;
        st = solver_new(plan, nb, 0, sigma2, rtol > 0.0 ? rtol : 1e-300, pc, s,
                        [&](double *B, int W) {
                            hipLaunchKernelGGL(pc_probe_kernel, dim3(grid1(n * W)), dim3(BS), 0, s,
                                               static_cast<const double *>(pc->L.ptr), pc->kmax, rank,
                                               G1 ? G1 + (size_t)r0 * ldg1 : nullptr, ldg1, G2 + (size_t)r0 * ldg2,
                                               ldg2, nb, sigma, static_cast<const int32_t *>(plan->perm.ptr), n, B,
                                               W);
                        },
                        &sv, steps);
        if (st != MM_OK) break;
        const int W = sv->W;
        // z^T P^{-1} z of each probe: the initial r.z
        std::vector<double> h0((size_t)W * NS), hsc((size_t)W * NS), tl((size_t)steps * W * 2);
        if (hipMemcpyAsync(h0.data(), sv->desc.sc, h0.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("HIP error reading the initial residuals");
            st = MM_ERR_HIP;
        }
        if (st == MM_OK) st = solver_run(sv, steps, s);
        if (st == MM_OK &&
            (hipMemcpyAsync(hsc.data(), sv->desc.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                 hipSuccess ||
             hipMemcpyAsync(tl.data(), sv->desc.tlog, tl.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                 hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess)) {
            set_error("HIP error reading the Lanczos coefficients");
            st = MM_ERR_HIP;
        }
        for (int r = 0; r < nb && st == MM_OK; ++r) {
            double q = 0.0;
            int ms = 0;
            if (!column_logquad(hsc.data() + (size_t)r * NS, tl, W, r, &q, &ms, h0[(size_t)r * NS + 0])) {
                set_error("probe %d: the Lanczos matrix did not converge to a positive spectrum", r0 + r);
                st = MM_ERR_BREAKDOWN;
                break;
            }
            if (quad) quad[r0 + r] = q;
            if (lanczos_steps) lanczos_steps[r0 + r] = ms;
            sum += q;
        }
        std::string msg = last_error_str();
        mm_solver_destroy(sv);
        if (st != MM_OK) set_error("%s", msg.c_str());
    }
    if (st != MM_OK) return st;
    *logdet = ldp + sum / nprobes;
    if (logdet_precond) *logdet_precond = ldp;
    return MM_OK;
}

mm_status gp_lml(mm_plan plan, const double *y, double sigma2, const double *Zc, int64_t ldz, int32_t nprobes,
                 int32_t maxit, double rtol, mm_lml_info *info, double *alpha, void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol));
    if (!y || !Zc || !info) {
        set_error("y, Z and info must be non-NULL");
        return MM_ERR_ARG;
    }
    if (nprobes < 1 || nprobes > 63 || maxit < 1 || ldz < plan->n) {
        set_error("nprobes in [1, 63], maxit >= 1 and ldz >= n are required");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = plan->n;
    const int32_t *perm = static_cast<const int32_t *>(plan->perm.ptr);
    mm_solver sv = nullptr;
    MM_TRY(solver_new(plan, 1 + nprobes, 0, sigma2, rtol, nullptr, s,
                      [&](double *B, int W) {
                          hipLaunchKernelGGL(gather_lml_kernel, dim3(grid1(n * W)), dim3(BS), 0, s, y, Zc, ldz,
                                             nprobes, perm, n, B, W);
                      },
                      &sv, maxit));
    const int W = sv->W;
    mm_status st = solver_run(sv, maxit, s);
    int conv = 0, brk = 0;
    double rel = 0.0;
    mm_solve_info inf{};
    if (st == MM_OK) st = solver_summary(sv, s, &conv, &brk, &rel, &inf);
    std::vector<double> hsc((size_t)W * NS), tl((size_t)maxit * W * 2), hp((size_t)3 * NRED * W);
    if (st == MM_OK && hipMemcpyAsync(hsc.data(), sv->desc.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                           hipSuccess) {
        set_error("HIP error reading the solver scalars");
        st = MM_ERR_HIP;
    }
    if (st == MM_OK && hipMemcpyAsync(tl.data(), sv->desc.tlog, tl.size() * sizeof(double), hipMemcpyDeviceToHost,
                                      s) != hipSuccess) {
        set_error("HIP error reading the Lanczos coefficients");
        st = MM_ERR_HIP;
    }
    // the derivative product of [alpha, z_1 .. z_l] in the plan's work buffers
    // (free again: the solve has finished), then the column dot products
    if (st == MM_OK) st = ensure_work(plan, W, true);
    if (st == MM_OK) {
        double *V = static_cast<double *>(plan->vin.ptr);
        double *D = static_cast<double *>(plan->yacc.ptr);
        hipLaunchKernelGGL(lml_mix_kernel, dim3(grid1(n * W)), dim3(BS), 0, s, sv->desc.X, sv->desc.B, n, W, V);
        st = sweep_all_dl(plan, V, D, W, rhs_block(plan->kernel, plan->d, W), s);
        if (st == MM_OK) {
            hipLaunchKernelGGL(lml_dots_kernel, dim3(NRED), dim3(BS), 0, s, sv->desc.X, sv->desc.B, D, n, W,
                               sv->desc.part);
            if (alpha)
                hipLaunchKernelGGL(col_out_kernel, dim3(grid1(n)), dim3(BS), 0, s, sv->desc.X, perm, n, W, 1, alpha, n);
            if (hipMemcpyAsync(hp.data(), sv->desc.part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("HIP error in the likelihood products");
                st = MM_ERR_HIP;
            }
        }
    }
    if (st == MM_OK) {
        // column sums of the row-block partials, in block order
        std::vector<double> xb(W, 0.0), xd(W, 0.0), xx(W, 0.0);
        for (int b = 0; b < NRED; ++b)
            for (int r = 0; r < W; ++r) {
                xb[r] += hp[(size_t)b * W + r];
                xd[r] += hp[(size_t)(NRED + b) * W + r];
                xx[r] += hp[(size_t)(2 * NRED + b) * W + r];
            }
        const double s2 = plan->kernel.outputscale2, ell = plan->kernel.lengthscale;
        double ld = 0.0, tr_inv = 0.0, tr_dk = 0.0, tr_k = 0.0;
        for (int r = 1; r <= nprobes && st == MM_OK; ++r) {
            double q = 0.0;
            int ms = 0;
            const double *c = hsc.data() + (size_t)r * NS;
            if (!column_logquad(c, tl, W, r, &q, &ms)) {
                set_error("probe %d: the Lanczos matrix did not converge to a positive spectrum", r - 1);
                st = MM_ERR_BREAKDOWN;
                break;
            }
            ld += q;
            tr_inv += xb[r];                               // z^T A^-1 z
            tr_dk += xd[r];                                // (A^-1 z)^T (l dK/dl / s2) z
            tr_k += c[4] * c[4] - sigma2 * xb[r];          // z^T A^-1 K z = |z|^2 - sigma2 z^T A^-1 z
        }
        if (st == MM_OK) {
            const double inv_l = 1.0 / nprobes;
            mm_lml_info o{};
            o.quad = xb[0];
            o.logdet = ld * inv_l;
            o.lml = -0.5 * o.quad - 0.5 * o.logdet - 0.5 * (double)n * std::log(2.0 * M_PI);
            o.trace_inv = tr_inv * inv_l;
            o.trace_dk_dlengthscale = s2 / ell * tr_dk * inv_l;
            o.dlml_dlengthscale = 0.5 * (s2 / ell) * xd[0] - 0.5 * o.trace_dk_dlengthscale;
            o.dlml_dsigma2 = 0.5 * xx[0] - 0.5 * o.trace_inv;
            // dK/d s2 = K / s2; alpha^T K alpha = y^T alpha - sigma2 alpha^T alpha
            o.dlml_doutputscale2 = (0.5 * (xb[0] - sigma2 * xx[0]) - 0.5 * tr_k * inv_l) / s2;
            o.relres_max = inf.relres_max;
            o.iters = inf.iters;
            o.converged = conv == 1 + nprobes ? 1 : 0;
            *info = o;
            st = status_of(conv, 1 + nprobes, brk, inf.iters, rel);
        }
    }
    std::string msg = last_error_str();
    mm_solver_destroy(sv);
    if (st != MM_OK) set_error("%s", msg.c_str());
    return st;
}

mm_status gp_variance(mm_plan plan, double sigma2, const double *z, int64_t m, int64_t ldz, double rtol,
                      int32_t maxit, double *var, mm_solve_info *info, void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol));
    if (!z || !var) {
        set_error("z and var must be non-NULL");
        return MM_ERR_ARG;
    }
    if (m < 1 || ldz < m || maxit < 1) {
        set_error("m >= 1, ldz >= m and maxit >= 1 are required");
        return MM_ERR_ARG;
    }
    const int64_t n = plan->n;
    const int d = plan->d;
    if (n + m > (int64_t(1) << 30)) {
        set_error("n + m exceeds 2^30");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nm = n + m;
    constexpr int BLK = 32;  // prediction points per block of solves
    DevBuf wb;
    MM_TRY(dev_alloc(wb, ((size_t)d * nm + (size_t)2 * nm * BLK) * sizeof(double)));
    double *U = static_cast<double *>(wb.ptr);
    double *V = U + (size_t)d * nm;
    double *KV = V + (size_t)nm * BLK;
    hipLaunchKernelGGL(union_coords_kernel, dim3(grid1(nm)), dim3(BS), 0, s, static_cast<const double *>(plan->xc.ptr),
                       n, z, m, ldz, d, U);
    mm_plan up = nullptr;
    mm_status st = mm_plan_create(U, nm, d, nm, &plan->kernel, stream, &up);
    const double s2 = plan->kernel.outputscale2;
    mm_solve_info worst{};
    int conv_all = 1, brk_any = 0;
    double rel_all = 0.0;
    std::vector<double> hv(BLK), hp((size_t)3 * NRED * BLK);
    for (int64_t j0 = 0; j0 < m && st == MM_OK; j0 += BLK) {
        const int b = (int)(m - j0 < BLK ? m - j0 : BLK);
        // k_z for the block: exact products of the union with unit weights
        hipLaunchKernelGGL(unit_cols_kernel, dim3(grid1(nm * b)), dim3(BS), 0, s, V, nm, n, j0, b);
        st = matern_mvm(up, V, nm, KV, nm, b, 0.0, stream);
        if (st != MM_OK) break;
        mm_solver sv = nullptr;
        st = solver_new(plan, b, 0, sigma2, rtol, nullptr, s,
                        [&](double *B, int W) {
                            hipLaunchKernelGGL(kz_rhs_kernel, dim3(grid1(n * W)), dim3(BS), 0, s, KV, nm, n, b, B, W);
                        },
                        &sv);
        if (st != MM_OK) break;
        st = solver_run(sv, maxit, s);
        int conv = 0, brk = 0;
        double rel = 0.0;
        mm_solve_info inf{};
        if (st == MM_OK) st = solver_summary(sv, s, &conv, &brk, &rel, &inf);
        if (st == MM_OK) {
            const int W = sv->W;
            // k_z^T A^-1 k_z per column (the X.B sums)
            hipLaunchKernelGGL(lml_dots_kernel, dim3(NRED), dim3(BS), 0, s, sv->desc.X, sv->desc.B, sv->desc.B, n, W,
                               sv->desc.part);
            if (hipMemcpyAsync(hp.data(), sv->desc.part, (size_t)NRED * W * sizeof(double), hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("HIP error in the variance products");
                st = MM_ERR_HIP;
            } else {
                for (int r = 0; r < b; ++r) {
                    double q = 0.0;
                    for (int blk = 0; blk < NRED; ++blk) q += hp[(size_t)blk * W + r];
                    hv[r] = s2 - q;
                }
                if (hipMemcpyAsync(var + j0, hv.data(), b * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    set_error("HIP error writing the variances");
                    st = MM_ERR_HIP;
                }
            }
            if (inf.iters > worst.iters) worst.iters = inf.iters;
            if (inf.relres_max > worst.relres_max) worst.relres_max = inf.relres_max;
            worst.converged_cols += inf.converged_cols;
            if (conv < b) conv_all = 0;
            if (brk) brk_any = 1;
            if (rel > rel_all) rel_all = rel;
        }
        std::string msg = last_error_str();
        mm_solver_destroy(sv);
        if (st != MM_OK) set_error("%s", msg.c_str());
    }
    if (up) mm_plan_destroy(up);
    dev_free(wb);
    if (st != MM_OK) return st;
    if (info) *info = worst;
    if (brk_any) {
        set_error("conjugate gradients broke down (p^T A p <= 0)");
        return MM_ERR_BREAKDOWN;
    }
    if (!conv_all) {
        set_error("conjugate gradients did not reach rtol in %d iterations (relres %.3e)", worst.iters, rel_all);
        return MM_ERR_NOCONV;
    }
    return MM_OK;
}

mm_status gp_cg_solve_multi(mm_plan plan, const double *Bc, int64_t ldb, int32_t nrhs, double sigma2, double rtol,
                            int32_t maxit, double *Xc, int64_t ldx, mm_solve_info *info, void *stream) {
    clear_error();
    MM_TRY(check_solve_args(plan, sigma2, rtol));
    if (!Bc || !Xc) {
        set_error("B and X must be non-NULL");
        return MM_ERR_ARG;
    }
    if (nrhs < 1 || nrhs > 64 || maxit < 1) {
        set_error("nrhs must be in [1, 64] and maxit >= 1");
        return MM_ERR_ARG;
    }
    if (ldb < plan->n || ldx < plan->n) {
        set_error("ldb and ldx must be >= n");
        return MM_ERR_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    mm_solver sv = nullptr;
    MM_TRY(solver_new(plan, nrhs, 0, sigma2, rtol, nullptr, s,
                      [&](double *B, int W) {
                          hipLaunchKernelGGL(gather_cols_kernel, dim3(grid1(plan->n * W)), dim3(BS), 0, s, Bc, ldb,
                                             nrhs, static_cast<const int32_t *>(plan->perm.ptr), plan->n, B, W);
                      },
                      &sv));
    mm_status st = solver_solve(sv, maxit, s);
    int conv = 0, brk = 0;
    double rel = 0.0;
    mm_solve_info inf{};
    if (st == MM_OK) st = solver_summary(sv, s, &conv, &brk, &rel, &inf);
    if (st == MM_OK && !brk && sv->checked_iters != sv->iters) {
        st = solver_check(sv, s, false, nullptr, nullptr);
        if (st == MM_OK) st = solver_summary(sv, s, &conv, &brk, &rel, &inf);
    }
    if (st == MM_OK) {
        inf.true_relres = brk ? -1.0 : sv->true_rel;
        if (info) *info = inf;
        hipLaunchKernelGGL(col_out_kernel, dim3(grid1(plan->n * nrhs)), dim3(BS), 0, s, sv->desc.X,
                           static_cast<const int32_t *>(plan->perm.ptr), plan->n, sv->W, nrhs, Xc, ldx);
        if (hipStreamSynchronize(s) != hipSuccess) {
            set_error("HIP error after the solve");
            st = MM_ERR_HIP;
        } else {
            st = status_of(conv, nrhs, brk, inf.iters, rel, inf.true_relres, rtol);
        }
    }
    std::string msg = last_error_str();
    mm_solver_destroy(sv);
    if (st != MM_OK) set_error("%s", msg.c_str());
    return st;
}

}  // extern "C"
