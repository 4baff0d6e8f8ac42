// Internal declarations shared by the HIP sources of libmaternmvm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/maternmvm.h"

namespace mm {

// ---------------------------------------------------------------------------
// Error reporting (thread-local message returned by mm_last_error()).
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();
const char *last_error_str();

#define MM_HIP_TRY(expr)                                                        \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ::mm::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                \
            return (e_ == hipErrorOutOfMemory) ? MM_ERR_NOMEM : MM_ERR_HIP;     \
        }                                                                       \
    } while (0)

#define MM_TRY(expr)                 \
    do {                             \
        mm_status s_ = (expr);       \
        if (s_ != MM_OK) return s_;  \
    } while (0)

// ---------------------------------------------------------------------------
// Device buffers owned by a plan.
// ---------------------------------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    mm_free_fn freefn = nullptr;  // the caller allocator that provided ptr (NULL: hipMalloc)
    void *ctx = nullptr;
};

mm_status dev_alloc(DevBuf &b, size_t bytes);
void set_allocator(mm_alloc_fn alloc, mm_free_fn free, void *ctx);
mm_status dev_reserve(DevBuf &b, size_t bytes);  // grow-only
void dev_free(DevBuf &b);

// ---------------------------------------------------------------------------
// One divide-and-conquer pass: a segmented bidirectional scan over a stored
// order of the points.
//   d = 1: the single pass scans the canonical (x1-sorted) order.
//   d = 2: level l; ord lists canonical indices, segments of 2^(l+1)
//          positions (the x1-rank nodes), each sorted by x2.
//   d = 3: level pair (l1, l2); ord lists positions q of the level-l1
//          (x1, x2) order ord2, segments of 2^(l2+1) positions, sorted by x3.
// ---------------------------------------------------------------------------
struct Pass {
    const int32_t *ord = nullptr;   // build only: position -> canonical index (d=2) or q (d=3)
    const int32_t *ord2 = nullptr;  // build only, d=3: q -> canonical index of level l1
    // geometry in pass order, read by the sweeps (d >= 2):
    const uint32_t *cf = nullptr;   // canonical index | x1 half << 30 | x2 half << 31
    const double *xs = nullptr;     // scan (last) coordinate
    const double *w1 = nullptr;     // |x1 - x1 of the node's split point|
    const double *w2 = nullptr;     // d=3: |x2 - x2 of the x2 node's split point|
    int l1 = -1;
    int l2 = -1;
    int seg_log2 = 0;               // segment size 2^seg_log2 positions
};

// Kernel constants derived from mm_kernel.
struct KParams {
    int P = 1;        // number of separable terms (nu + 1/2)
    bool prod = true; // product form (also used for d = 1 and nu = 1/2)
    double a = 1.0;   // sqrt(2 nu) / lengthscale
    double s2 = 1.0;  // outputscale^2
};

KParams kparams(const mm_kernel &k, int d);

// Scan schedule of the products at one padded width: wb columns per wave (the
// column block), runs of e positions per lane (tiles of 64 / wb * e
// positions), and whether the tile-aggregate pre-pass stores the runs'
// within-tile carries for the main launch (d <= 2, below 32 columns).  e = 0
// selects the default run length of the block.
struct Sched {
    int wb = 1;
    int e = 0;
    int runex = 1;
};

}  // namespace mm

// ---------------------------------------------------------------------------
// The plan object behind mm_plan.
// ---------------------------------------------------------------------------
struct mm_plan_s {
    int device = 0;
    int64_t n = 0;
    int d = 1;
    int L = 0;                    // ceil(log2 n) divide-and-conquer levels
    mm_kernel kernel{};
    hipStream_t last_stream = nullptr;

    mm::DevBuf xc;                // d x n canonical coordinates (SoA, x1-rank order)
    mm::DevBuf perm;              // n int32: canonical index -> caller index
    mm::DevBuf iperm;             // n int32: caller index -> canonical index
    mm::DevBuf structure;         // stored orders (int32; released once the pass geometry is built)
    mm::DevBuf geo;               // per-pass geometry in pass order (cf, xs, w1, w2)
    std::vector<mm::Pass> passes;
    mm::DevBuf pass_dev;          // device table of the passes
    static constexpr int NTS = 4;  // tile sizes 128, 256, 512, 1024 positions
    mm::DevBuf pass_xt[NTS];        // per tile size: passes whose segments span tiles
    mm::DevBuf pass_xtpos[NTS];     // per tile size: each pass's position in pass_xt (-1: none)
    std::vector<int> xt_host[NTS];
    mm::DevBuf seg_tab[NTS];        // per tile size: (pass, first tile, end tile) of those segments
    std::vector<int> seg_off[NTS];  //   offset of each cross-tile pass's first segment
    std::vector<int4> seg_host[NTS];  // host copy of seg_tab
    mm::DevBuf seg_big[NTS];        // per tile size: indices into seg_tab of the segments of more
                                    //   than CARRY_SMALL tiles (the carry scan's wave-per-slice path)
    std::vector<int> big_off[NTS];  //   offset of each cross-tile pass's first such segment

    // scan schedules chosen for particular widths (mm_plan_set_schedule; others: the default)
    std::vector<std::pair<int, mm::Sched>> sched;

    // product work buffers (grow on demand)
    mm::DevBuf vin;               // n x W point-major canonical input
    mm::DevBuf yacc;              // n x W point-major canonical accumulator
    mm::DevBuf agg;               // tile aggregates and anchors
    mm::DevBuf part;              // per-pass partial results of one pass group
    int64_t work_cols = 0;
    int npins = 0;                // live solvers and product batches reading this plan

    // measurement
    bool profile = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    size_t prof_used = 0;
    double prof_ms = 0.0;
    int64_t prof_launches = 0;
    int64_t prof_units = 0;       // passes covered by the bracketed launches
};

// Rank-k pivoted Cholesky preconditioner (precond.hip).
struct mm_precond_s {
    mm_plan plan = nullptr;
    int kmax = 0;                 // columns allocated (row stride of L)
    int rank = 0;                 // columns computed
    mm::DevBuf L;                 // n x kmax, row-major, canonical order
    mm::DevBuf work;              // residual diagonal, reduction partials, state
    std::vector<double> gram;     // rank x rank: L^T L (host)
    std::vector<int32_t> pivots;  // caller index of each column's pivot
    double trace0 = 0.0, trace_res = 0.0;
    int npins = 0;                // live solvers using it
};

namespace mm {

// sweep.hip
mm_status profile_flush(mm_plan p, double *ms, int64_t *launches);

// Batched sweeps over several problems of one width (one launch per kernel
// configuration and phase; the work tables are built once per problem set).
struct BatchEntry {
    mm_plan p;
    const double *vin;  // n x W point-major canonical input
    double *yacc;       // n x W point-major result (sum over passes)
    double *agg;        // workspaces of sweep_batch_bytes (owned by the caller)
    double *part;
};
// Workspace sizes of a batched product of plan p at width W, where all of the
// plan's passes run as one group; false if their partial slabs would exceed
// the group budget (such a problem runs alone through sweep_all).
bool sweep_batch_bytes(mm_plan p, int W, size_t *agg_bytes, size_t *part_bytes);
bool sweep_batch_bytes_n(int64_t n, int d, const mm_kernel &k, int npass, int W, size_t *agg_bytes,
                         size_t *part_bytes);
constexpr int ACC_CHUNK = 2048;
struct AccumDesc {
    const double *ypart;
    double *yacc;
    int64_t len;
    int G;
};
struct SweepBatch {
    struct Cls {
        int key = 0, d = 1;
        KParams kp;
        Sched sc;                  // the members' common schedule
        std::vector<int> members;
        DevBuf descs, items_agg, items_carry, items_main;
        int n_agg = 0, n_carry = 0, n_main = 0;
    };
    std::vector<Cls> classes;
    std::vector<mm_plan> plans;  // the problems' plans (a lone plan's profiling brackets the main launch)
    DevBuf acc_desc, acc_items;
    int n_acc = 0;
    int W = 1, WB = 1;
    int grid_per_cu = 16;  // persistent carry-scan grid: workgroups per compute unit (tuned)
    bool skip_accum = false;  // leave the per-pass partials unsummed (the consumer sums them)
};
mm_status sweep_batch_build(const std::vector<BatchEntry> &probs, int W, int WB, SweepBatch &out);
mm_status sweep_batch_run(SweepBatch &b, hipStream_t s);
void sweep_batch_free(SweepBatch &b);
// Workspaces of a product supplied by the caller instead of the plan's own
// (aggregates of sweep_agg_bytes, partial slabs of sweep_part_bytes).
struct SweepWs {
    double *agg;
    double *part;
};
// yacc <- the off-diagonal sums of K applied to vin (unscaled; canonical order).  With tail,
// the last pass group's slabs stay in the partial-slab workspace unsummed (see run_passes);
// ws replaces the plan's workspaces (no profiling then).
mm_status sweep_all(mm_plan p, const double *vin, double *yacc, int W, int R, hipStream_t s, int *tail = nullptr,
                    const SweepWs *ws = nullptr);
// yacc <- the off-diagonal sums of l dK/dl applied to vin (unscaled; canonical order)
mm_status sweep_all_dl(mm_plan p, const double *vin, double *yacc, int W, int R, hipStream_t s);
int rhs_block(const mm_kernel &k, int d, int nrhs);
// the schedule of plan p's products at width W (default column block WB)
Sched plan_sched(mm_plan p, int W, int WB);
// whether schedule sc is compiled for the kernel class (d, kp) at width W
bool sched_available(int d, const KParams &kp, const Sched &sc, int W);
size_t sweep_agg_bytes(int64_t n, int d, int W, const mm_kernel &k, bool der = false);
int agg_per_rhs(int d, const mm_kernel &k, bool der);
size_t sweep_part_bytes(int64_t n, int npass, int W);
int group_passes(mm_plan p, int W);
mm_status upload_pass_tables(mm_plan p);

// mvm.hip helpers
mm_status mvm_internal(mm_plan p, const double *vin, double *yout, int W, int nrhs,
                       double shift, hipStream_t s);
// reserve the plan's product buffers for W columns (der: also the lengthscale-derivative sweeps)
mm_status ensure_work(mm_plan p, int W, bool der = false);

// permutation kernels
// y (caller column-major) = s2 (vin + sum of the G pass slabs) + shift vin: the sum over
// passes in pass order, fused with the diagonal and the un-permutation
void launch_finish_out(mm_plan p, const double *vin, const double *part, int G, int first, const double *yacc,
                       int W, int nrhs, double s2, double shift, double *y, int64_t ldy, hipStream_t s);
// vin (canonical point-major, W columns, padding zero) from v (caller column-major)
void launch_gather_caller(mm_plan p, const double *v, int64_t ldv, int nrhs, double *vin, int W, hipStream_t s);

}  // namespace mm
