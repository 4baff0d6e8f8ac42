// Batched kernel products over many independent point sets (Section 2,
// eq. Ky, for each problem): one gather launch, the batched sweeps (one
// launch per kernel configuration and phase) and one scatter launch cover
// every problem of the batch.  Each problem runs exactly the arithmetic of
// matern_mvm on its own plan, so its result does not depend on the batch.
#include "mm_internal.h"

#include <cmath>

namespace mm {
namespace {

constexpr int BS = 256;
constexpr int CHUNK = 8192;

// Per-problem pointers of one call (updated by every run before the launches).
struct MvmIo {
    const double *v;
    double *y;
    int64_t ldv, ldy;
};

// Per-problem constants of the batch.
struct MvmDesc {
    const int32_t *perm;    // canonical index -> caller index
    const int32_t *iperm;   // caller index -> canonical index
    double *vin;
    const double *part;     // the G per-pass partial slabs (n x W each)
    int64_t n;
    int W, nrhs, G;
    double s2;
};

// vin[iperm[i], r] = v[r * ldv + i] (padding columns zero), as matern_mvm's
// gather: items are chunks of (caller point, column) pairs, column fastest.
__global__ void gather_batch_kernel(const MvmDesc *ds, const MvmIo *io, const int2 *items, int nitems) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const MvmDesc d = ds[it.x];
        const MvmIo q = io[it.x];
        const int64_t total = d.n * d.W;
        const int64_t lo = (int64_t)it.y * CHUNK;
        const int64_t hi = lo + CHUNK < total ? lo + CHUNK : total;
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            const int64_t pt = e / d.W;
            const int r = (int)(e - pt * d.W);
            d.vin[(int64_t)d.iperm[pt] * d.W + r] = r < d.nrhs ? q.v[(int64_t)r * q.ldv + pt] : 0.0;
        }
    }
}

// y[r * ldy + i] = s2 (vin + sum of the pass slabs in pass order) + shift vin at
// canonical row iperm[i]: the arithmetic of matern_mvm's output step.
__global__ void scatter_batch_kernel(const MvmDesc *ds, const MvmIo *io, const int2 *items, int nitems,
                                     double shift) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const MvmDesc d = ds[it.x];
        const MvmIo q = io[it.x];
        const int64_t total = d.n * d.W;
        const int64_t len = d.n * d.W;
        const int64_t lo = (int64_t)it.y * CHUNK;
        const int64_t hi = lo + CHUNK < total ? lo + CHUNK : total;
        if (d.W >= 4) {
            // caller order, whole canonical rows read (as matern_mvm's output step)
            for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
                const int64_t pt = e / d.W;
                const int r = (int)(e - pt * d.W);
                if (r >= d.nrhs) continue;
                const int64_t c = (int64_t)d.iperm[pt] * d.W + r;
                double acc = 0.0;
                for (int g = 0; g < d.G; ++g) acc += d.part[(int64_t)g * len + c];
                const double vv = d.vin[c];
                q.y[(int64_t)r * q.ldy + pt] = fma(shift, vv, d.s2 * (vv + acc));
            }
        } else {
            // narrow rows: canonical order, sequential slab reads, writes at perm[c]
            for (int64_t c = lo + threadIdx.x; c < hi; c += blockDim.x) {
                const int64_t pt = c / d.W;
                const int r = (int)(c - pt * d.W);
                if (r >= d.nrhs) continue;
                double acc = 0.0;
                for (int g = 0; g < d.G; ++g) acc += d.part[(int64_t)g * len + c];
                const double vv = d.vin[c];
                q.y[(int64_t)r * q.ldy + d.perm[pt]] = fma(shift, vv, d.s2 * (vv + acc));
            }
        }
    }
}

template <class T>
mm_status upload_tab(DevBuf &b, const std::vector<T> &v) {
    if (v.empty()) return MM_OK;
    MM_TRY(dev_alloc(b, v.size() * sizeof(T)));
    MM_HIP_TRY(hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return MM_OK;
}

inline unsigned pgrid(int nitems, int cap) {
    return (unsigned)(nitems < cap ? (nitems < 1 ? 1 : nitems) : cap);
}

}  // namespace
}  // namespace mm

using namespace mm;

struct mm_mvm_batch_s {
    std::vector<mm_plan> plans;
    int nrhs = 1, W = 1, WB = 1;
    DevBuf work;                 // per problem: vin, aggregates, partial slabs
    DevBuf desc, io_dev, items_in, items_out;
    int n_in = 0, n_out = 0;
    MvmIo *io_host = nullptr;    // pinned staging of the per-call pointers
    hipEvent_t io_done = nullptr;
    SweepBatch sweep;
    double shift = 0.0;
    int use_graph = 1;
    int grid_cap = 2048;
    hipStream_t bs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t graph = nullptr;
};

namespace {

// Release the executable graph once its last launch (on the batch's private
// stream) has finished: a graph whose branches run side by side owns the
// streams they run on, so it must not go while it executes.
void drop_graph(mm_mvm_batch b) {
    if (!b->graph) return;
    if (b->bs) (void)hipStreamSynchronize(b->bs);
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

void mvm_batch_release(mm_mvm_batch b) {
    drop_graph(b);
    sweep_batch_free(b->sweep);
    dev_free(b->work);
    dev_free(b->desc);
    dev_free(b->io_dev);
    dev_free(b->items_in);
    dev_free(b->items_out);
    if (b->io_host) (void)hipHostFree(b->io_host);
    if (b->io_done) (void)hipEventDestroy(b->io_done);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->bs) (void)hipStreamDestroy(b->bs);
    for (mm_plan p : b->plans) p->npins--;
    b->plans.clear();
}

mm_status mvm_batch_enqueue(mm_mvm_batch b, hipStream_t s) {
    const MvmDesc *ds = static_cast<const MvmDesc *>(b->desc.ptr);
    const MvmIo *io = static_cast<const MvmIo *>(b->io_dev.ptr);
    hipLaunchKernelGGL(gather_batch_kernel, dim3(pgrid(b->n_in, b->grid_cap)), dim3(BS), 0, s, ds, io,
                       static_cast<const int2 *>(b->items_in.ptr), b->n_in);
    MM_TRY(sweep_batch_run(b->sweep, s));
    hipLaunchKernelGGL(scatter_batch_kernel, dim3(pgrid(b->n_out, b->grid_cap)), dim3(BS), 0, s, ds, io,
                       static_cast<const int2 *>(b->items_out.ptr), b->n_out, b->shift);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

mm_status mvm_batch_build(mm_mvm_batch b) {
    const size_t count = b->plans.size();
    std::vector<size_t> aggb(count), partb(count);
    size_t total = 0;
    for (size_t k = 0; k < count; ++k) {
        mm_plan p = b->plans[k];
        if (!sweep_batch_bytes(p, b->W, &aggb[k], &partb[k])) {
            set_error("problem %zu is too large for a batched product at %d columns (its partial sums exceed 16 GiB)",
                      k, b->nrhs);
            return MM_ERR_ARG;
        }
        const size_t vec = ((size_t)p->n * b->W * sizeof(double) + 255) & ~size_t(255);
        total += vec + ((aggb[k] + 255) & ~size_t(255)) + ((partb[k] + 255) & ~size_t(255));
    }
    MM_TRY(dev_alloc(b->work, total));
    char *base = static_cast<char *>(b->work.ptr);
    std::vector<BatchEntry> ent;
    std::vector<MvmDesc> descs;
    std::vector<int2> ii, io;
    for (size_t k = 0; k < count; ++k) {
        mm_plan p = b->plans[k];
        const size_t vec = ((size_t)p->n * b->W * sizeof(double) + 255) & ~size_t(255);
        double *vin = reinterpret_cast<double *>(base);
        double *agg = reinterpret_cast<double *>(base + vec);
        base += vec + ((aggb[k] + 255) & ~size_t(255));
        double *part = reinterpret_cast<double *>(base);
        base += (partb[k] + 255) & ~size_t(255);
        ent.push_back(BatchEntry{p, vin, nullptr, agg, part});  // no sum buffer: the output step sums the slabs
        descs.push_back(MvmDesc{static_cast<const int32_t *>(p->perm.ptr), static_cast<const int32_t *>(p->iperm.ptr),
                                vin, part, p->n, b->W, b->nrhs,
                                (int)p->passes.size(), p->kernel.outputscale2});
        const int64_t nin = (p->n * b->W + CHUNK - 1) / CHUNK;
        for (int64_t c = 0; c < nin; ++c) ii.push_back(make_int2((int)k, (int)c));
        for (int64_t c = 0; c < nin; ++c) io.push_back(make_int2((int)k, (int)c));
    }
    MM_TRY(sweep_batch_build(ent, b->W, b->WB, b->sweep));
    b->sweep.skip_accum = true;  // the output step sums the per-pass partials itself
    MM_TRY(upload_tab(b->desc, descs));
    MM_TRY(upload_tab(b->items_in, ii));
    MM_TRY(upload_tab(b->items_out, io));
    b->n_in = (int)ii.size();
    b->n_out = (int)io.size();
    MM_TRY(dev_alloc(b->io_dev, count * sizeof(MvmIo)));
    MM_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&b->io_host), count * sizeof(MvmIo), hipHostMallocDefault));
    MM_HIP_TRY(hipEventCreateWithFlags(&b->io_done, hipEventDisableTiming));
    return MM_OK;
}

}  // namespace

extern "C" {

mm_status mm_mvm_batch_create(const mm_plan *plans, int32_t count, int32_t nrhs, int32_t use_graph,
                              mm_mvm_batch *out) {
    clear_error();
    if (!out || !plans || count < 1) {
        set_error("plans, count >= 1 and out are required");
        return MM_ERR_ARG;
    }
    *out = nullptr;
    if (nrhs < 1 || nrhs > 256) {
        set_error("nrhs must be in [1, 256] (got %d)", nrhs);
        return MM_ERR_ARG;
    }
    for (int k = 0; k < count; ++k)
        if (!plans[k]) {
            set_error("plan %d is NULL", k);
            return MM_ERR_ARG;
        }
    mm_mvm_batch b = new (std::nothrow) mm_mvm_batch_s();
    if (!b) {
        set_error("host allocation failed");
        return MM_ERR_NOMEM;
    }
    b->nrhs = nrhs;
    // the width rule of matern_mvm (each problem's own kernel gives the same block)
    b->WB = rhs_block(plans[0]->kernel, plans[0]->d, nrhs);
    b->W = (nrhs + b->WB - 1) / b->WB * b->WB;
    b->use_graph = use_graph ? 1 : 0;
    for (int k = 0; k < count; ++k) {
        b->plans.push_back(plans[k]);
        plans[k]->npins++;  // the batch pins the plan's kernel and storage
    }
    mm_status st = mvm_batch_build(b);
    if (st != MM_OK) {
        mvm_batch_release(b);
        delete b;
        return st;
    }
    *out = b;
    return MM_OK;
}

mm_status mm_mvm_batch_set_schedule(mm_mvm_batch batch, int32_t sweep_wg_per_cu, int32_t grid) {
    clear_error();
    if (!batch || sweep_wg_per_cu < 1 || grid < 1) {
        set_error("batch is NULL or schedule out of range");
        return MM_ERR_ARG;
    }
    batch->sweep.grid_per_cu = sweep_wg_per_cu;
    batch->grid_cap = grid;
    drop_graph(batch);
    return MM_OK;
}

mm_status mm_mvm_batch_run(mm_mvm_batch b, const double *const *v, const int64_t *ldv, double *const *y,
                           const int64_t *ldy, double diag_shift, void *stream) {
    clear_error();
    if (!b || !v || !y || !ldv || !ldy) {
        set_error("batch, v, ldv, y and ldy are required");
        return MM_ERR_ARG;
    }
    if (!std::isfinite(diag_shift)) {
        set_error("diag_shift must be finite");
        return MM_ERR_ARG;
    }
    const size_t count = b->plans.size();
    for (size_t k = 0; k < count; ++k) {
        if (!v[k] || !y[k] || ldv[k] < b->plans[k]->n || ldy[k] < b->plans[k]->n) {
            set_error("problem %zu: v and y must be non-NULL with leading dimensions >= n", k);
            return MM_ERR_ARG;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the previous call's pointer upload must have completed before the staging is rewritten
    MM_HIP_TRY(hipEventSynchronize(b->io_done));
    for (size_t k = 0; k < count; ++k) b->io_host[k] = MvmIo{v[k], y[k], ldv[k], ldy[k]};
    MM_HIP_TRY(hipMemcpyAsync(b->io_dev.ptr, b->io_host, count * sizeof(MvmIo), hipMemcpyHostToDevice, s));
    MM_HIP_TRY(hipEventRecord(b->io_done, s));
    if (diag_shift != b->shift) drop_graph(b);
    b->shift = diag_shift;
    if (!b->use_graph) return mvm_batch_enqueue(b, s);
    if (!b->bs) {
        MM_HIP_TRY(hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking));
        MM_HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        MM_HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    }
    if (!b->graph) {
        hipGraph_t g = nullptr;
        MM_HIP_TRY(hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal));
        mm_status st = mvm_batch_enqueue(b, b->bs);
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
            b->graph = nullptr;
            set_error("graph instantiation failed: %s", hipGetErrorString(e));
            return MM_ERR_HIP;
        }
    }
    MM_HIP_TRY(hipEventRecord(b->ev_in, s));
    MM_HIP_TRY(hipStreamWaitEvent(b->bs, b->ev_in, 0));
    MM_HIP_TRY(hipGraphLaunch(b->graph, b->bs));
    MM_HIP_TRY(hipEventRecord(b->ev_out, b->bs));
    MM_HIP_TRY(hipStreamWaitEvent(s, b->ev_out, 0));
    return MM_OK;
}

mm_status mm_mvm_batch_destroy(mm_mvm_batch batch) {
    if (!batch) return MM_OK;
    (void)hipDeviceSynchronize();
    mvm_batch_release(batch);
    delete batch;
    return MM_OK;
}

}  // extern "C"
