// The kernel product without device allocation (matern_mvm_noalloc), for
// callers that cannot allocate device memory: code under HIP graph capture,
// tight serving loops, hosts that forbid allocation.  Its work buffers (the
// canonical input and sum, the tile aggregates and carries, the per-pass
// partial slabs) live in one file-scope device array of fixed size instead of
// the plan's lazily allocated buffers; the plan itself is built beforehand by
// mm_plan_create.  The arithmetic is matern_mvm's, kernel for kernel, so the
// results are bitwise the same.
#include "mm_internal.h"

#include <cmath>
#include <mutex>

namespace mm {
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)MM_NOALLOC_SCRATCH_MIB << 20;

// Each device holds its own copy for the life of the process.  Host code never
// passes this name to a kernel: it uses the device address looked up below.
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

// Device address of the current device's scratch, looked up once per device
// (with that device current) at its first call.
mm_status scratch_address(void **out) {
    int dev = 0;
    MM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device %d is beyond the %d devices the scratch table covers", dev, MAX_DEVICES);
        return MM_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
            (void)hipGetLastError();
            return MM_ERR_HIP;
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return MM_OK;
}

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace
}  // namespace mm

using namespace mm;

extern "C" {

mm_status matern_mvm_noalloc(mm_plan plan, const double *v, int64_t ldv, double *y, int64_t ldy, int32_t nrhs,
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
    const int R = rhs_block(plan->kernel, plan->d, nrhs);
    const int W = (nrhs + R - 1) / R * R;
    const size_t vb = round256((size_t)plan->n * W * sizeof(double));
    const size_t ab = round256(sweep_agg_bytes(plan->n, plan->d, W, plan->kernel));
    const size_t pb = round256(sweep_part_bytes(plan->n, (int)plan->passes.size(), W));
    const size_t need = 2 * vb + ab + pb;
    if (need > SCRATCH_BYTES) {
        set_error("matern_mvm_noalloc: n = %lld, d = %d with %d right-hand sides needs %zu bytes of work "
                  "memory, more than its fixed %zu-byte scratch; use matern_mvm",
                  (long long)plan->n, plan->d, nrhs, need, SCRATCH_BYTES);
        return MM_ERR_ARG;
    }
    void *base = nullptr;
    MM_TRY(scratch_address(&base));
    char *b = static_cast<char *>(base);
    double *vin = reinterpret_cast<double *>(b);
    double *yacc = reinterpret_cast<double *>(b + vb);
    SweepWs ws{reinterpret_cast<double *>(b + 2 * vb), reinterpret_cast<double *>(b + 2 * vb + ab)};
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    launch_gather_caller(plan, v, ldv, nrhs, vin, W, s);
    int tail[2] = {0, 1};
    MM_TRY(sweep_all(plan, vin, yacc, W, R, s, tail, &ws));
    launch_finish_out(plan, vin, ws.part, tail[0], tail[1], yacc, W, nrhs, plan->kernel.outputscale2, diag_shift, y,
                      ldy, s);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

}  // extern "C"
