// Plan construction: the stored sorting outputs of the divide-and-conquer.
//
// Section 2.2 of the paper stores, once per point set, the sorted subsets
// each coordinate needs, so that every later product replaces its sorts by
// lookups.  Here that structure is:
//   * a stable LSD radix sort of order-preserving 64-bit keys of x_1 (ties
//     broken by index, giving a strict total order); the points are then
//     renumbered in x_1 order ("canonical" indices) and their coordinates
//     stored column by column in that order;
//   * d >= 2: for every level l of the x_1-rank tree, the canonical indices
//     of each node (2^(l+1) consecutive ranks) listed in x_2 order.  The top
//     level is one radix sort by x_2; each lower level is a stable partition
//     of the level above by one bit of the canonical index (a segmented
//     split), so no further sort is needed;
//   * d = 3: for every x_1 level l1 and every x_2 level l2 <= l1 inside it,
//     the positions of the level-l1 (x_1, x_2) order listed by x_2 sub-node
//     and, inside each sub-node, in x_3 order; built the same way from one
//     radix sort by x_3.
#include "mm_internal.h"

#include <cstdarg>
#include <cstring>

namespace mm {

// ---------------------------------------------------------------------------
// errors and device buffers
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }
const char *last_error_str() { return g_err.c_str(); }

// Caller allocator (mm_set_allocator); NULL: hipMalloc / hipFree.
static mm_alloc_fn g_alloc = nullptr;
static mm_free_fn g_free = nullptr;
static void *g_alloc_ctx = nullptr;

void set_allocator(mm_alloc_fn alloc, mm_free_fn free, void *ctx) {
    g_alloc = alloc;
    g_free = free;
    g_alloc_ctx = alloc ? ctx : nullptr;
}

mm_status dev_alloc(DevBuf &b, size_t bytes) {
    dev_free(b);
    if (bytes == 0) return MM_OK;
    void *ptr = nullptr;
    if (g_alloc) {
        ptr = g_alloc(bytes, nullptr, g_alloc_ctx);
        if (!ptr) {
            set_error("the caller allocator returned NULL for %zu bytes", bytes);
            return MM_ERR_NOMEM;
        }
        b.freefn = g_free;
        b.ctx = g_alloc_ctx;
    } else {
        hipError_t e = hipMalloc(&ptr, bytes);
        if (e != hipSuccess) {
            set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? MM_ERR_NOMEM : MM_ERR_HIP;
        }
        b.freefn = nullptr;
        b.ctx = nullptr;
    }
    b.ptr = ptr;
    b.bytes = bytes;
    return MM_OK;
}

mm_status dev_reserve(DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes && b.ptr) return MM_OK;
    return dev_alloc(b, bytes);
}

void dev_free(DevBuf &b) {
    if (b.ptr) {
        if (b.freefn) {
            // hipFree waits for the device; keep that guarantee for the caller's allocator
            (void)hipDeviceSynchronize();
            b.freefn(b.ptr, nullptr, b.ctx);
        } else {
            (void)hipFree(b.ptr);
        }
    }
    b.ptr = nullptr;
    b.bytes = 0;
    b.freefn = nullptr;
    b.ctx = nullptr;
}

KParams kparams(const mm_kernel &k, int d) {
    KParams kp;
    kp.P = (k.two_nu + 1) / 2;
    kp.prod = (k.form == MM_FORM_PRODUCT) || d == 1 || kp.P == 1;
    kp.a = sqrt((double)k.two_nu) / k.lengthscale;
    kp.s2 = k.outputscale2;
    return kp;
}

namespace {

constexpr int BS = 256;            // threads per block of the build kernels
constexpr int ITEMS = 8;
constexpr int TILE = BS * ITEMS;   // 2048 elements per block
constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------

// Order-preserving map of an IEEE double to an unsigned 64-bit key (-0 and +0
// map to the same key); non-finite inputs raise `bad`.
__device__ __forceinline__ uint64_t f64_key(double x) {
    if (x == 0.0) x = 0.0;
    uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void keys_kernel(const double *x, int64_t n, uint64_t *keys, int32_t *vals,
                            unsigned long long *orand, int *bad) {
    uint64_t lo = ~0ull, hi = 0ull;
    int badl = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double xi = x[i];
        if (!isfinite(xi)) badl = 1;
        const uint64_t k = f64_key(xi);
        keys[i] = k;
        vals[i] = (int32_t)i;
        lo &= k;
        hi |= k;
    }
    atomicAnd(&orand[0], (unsigned long long)lo);
    atomicOr(&orand[1], (unsigned long long)hi);
    if (badl) atomicOr(bad, 1);
}

// raise `bad` if any of the d coordinate columns holds a NaN or an infinity
__global__ void finite_kernel(const double *x, int64_t ldx, int64_t n, int d, int *bad) {
    int badl = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < d; ++k)
            if (!isfinite(x[k * ldx + i])) badl = 1;
    if (badl) atomicOr(bad, 1);
}

// ---------------------------------------------------------------------------
// block-wide exclusive scan of one unsigned per thread (BS threads)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += y;
    }
    if (lane == WAVE - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < BS / WAVE; ++w) {
        if (w < wave) before += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    total = tot;
    return before + incl - v;
}

// exclusive scan of m unsigned values in place, one block of 1024 threads
__global__ void scan_single(uint32_t *data, int64_t m) {
    constexpr int NT = 1024;
    __shared__ uint32_t part[NT];
    const int t = threadIdx.x;
    const int64_t chunk = (m + NT - 1) / NT;
    const int64_t lo = t * chunk;
    const int64_t hi = lo + chunk < m ? lo + chunk : m;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += data[i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele over the 1024 partial sums
    for (int o = 1; o < NT; o <<= 1) {
        uint32_t y = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 4-bit digits
// ---------------------------------------------------------------------------
constexpr int RADIX = 16;

__global__ void radix_count(const uint64_t *keys, int64_t n, int shift, uint32_t *counts,
                            int64_t nblocks) {
    __shared__ uint32_t h[RADIX];
    if (threadIdx.x < RADIX) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE;
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t e = base + i * BS + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < RADIX) counts[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements are taken in increasing index order (round i,
// then wave, then lane), and each lane's rank among equal digits of its wave
// comes from ballots, so equal keys keep their input order.
__global__ void radix_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                              int32_t *vout, int64_t n, int shift, const uint32_t *offs,
                              int64_t nblocks) {
    __shared__ uint32_t base[RADIX];
    __shared__ uint32_t wcnt[BS / WAVE][RADIX];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    if (threadIdx.x < RADIX) base[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t ltmask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t b0 = (int64_t)blockIdx.x * TILE;
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t e = b0 + i * BS + threadIdx.x;
        const bool valid = e < n;
        const uint64_t key = valid ? kin[e] : 0ull;
        const int dg = valid ? (int)((key >> shift) & (RADIX - 1)) : RADIX;
        uint32_t rank = 0;
        for (int dv = 0; dv < RADIX; ++dv) {
            const uint64_t m = __ballot(dg == dv);
            if (dg == dv) rank = (uint32_t)__popcll(m & ltmask);
            if (lane == 0) wcnt[wave][dv] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        if (threadIdx.x < RADIX) {
            uint32_t run = base[threadIdx.x];
            for (int w = 0; w < BS / WAVE; ++w) {
                const uint32_t c = wcnt[w][threadIdx.x];
                wcnt[w][threadIdx.x] = run;
                run += c;
            }
            base[threadIdx.x] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = wcnt[wave][dg] + rank;
            if ((int64_t)dst < n) {  // always true for consistent counts; guards the write
                kout[dst] = key;
                vout[dst] = vin[e];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// stable partition of aligned segments by one bit of the stored value
// ---------------------------------------------------------------------------
__global__ void part_count(const int32_t *src, int64_t n, int bit, uint32_t *bsum) {
    __shared__ uint32_t wsum[BS / WAVE];
    const int64_t b0 = (int64_t)blockIdx.x * TILE + threadIdx.x * ITEMS;
    uint32_t c = 0;
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t p = b0 + i;
        if (p < n) c += (uint32_t)((src[p] >> bit) & 1);
    }
    uint32_t tot;
    (void)block_excl_scan(c, wsum, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// new position of p in its segment [s0, s0 + 2^seglog2): values whose bit is
// 0 first, then those whose bit is 1, each group in input order.  The zeros of
// a segment are exactly the values of its lower half, min(2^(seglog2-1), n - s0).
__global__ void part_scatter(const int32_t *src, int32_t *dst, int64_t n, int bit, int seglog2,
                             const uint32_t *boff) {
    __shared__ uint32_t lpre[TILE];
    __shared__ uint32_t wsum[BS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int64_t b0 = base + threadIdx.x * ITEMS;
    int32_t val[ITEMS];
    uint32_t f[ITEMS];
    uint32_t c = 0;
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t p = b0 + i;
        val[i] = p < n ? src[p] : 0;
        f[i] = p < n ? (uint32_t)((val[i] >> bit) & 1) : 0u;
        c += f[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(c, wsum, tot);
    for (int i = 0; i < ITEMS; ++i) {
        lpre[threadIdx.x * ITEMS + i] = run;
        run += f[i];
    }
    __syncthreads();
    const int64_t seg = int64_t(1) << seglog2;
    const uint32_t bo = boff[blockIdx.x];
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t p = b0 + i;
        if (p >= n) break;
        const int64_t s0 = p & ~(seg - 1);
        const uint32_t pre_p = bo + lpre[p - base];
        const uint32_t pre_s0 = (seg >= TILE) ? boff[s0 / TILE] : bo + lpre[s0 - base];
        const int64_t ones_before = (int64_t)(pre_p - pre_s0);
        const int64_t half = seg >> 1;
        const int64_t nz = half < n - s0 ? half : n - s0;
        const int64_t d = f[i] ? s0 + nz + ones_before : p - ones_before;
        const int64_t send = s0 + seg < n ? s0 + seg : n;
        if (d >= s0 && d < send) dst[d] = val[i];  // stays inside its segment
    }
}

// d = 3: the orthant group of position p of pass (l1, l2): the x1 half of the
// point xor its x2 half.  Sources of one group only meet targets of the same
// group (their halves differ in both coordinates), so each segment is split
// into its group-0 run and its group-1 run, each still in x3 order.
__device__ __forceinline__ uint32_t pass_group(const int32_t *ord, const int32_t *ord2, int64_t p, int l1, int l2) {
    const int64_t q = ord[p];
    const int64_t c = ord2[q];
    return (uint32_t)(((c >> l1) ^ (q >> l2)) & 1);
}

// per TILE block: the number of group-1 positions
__global__ void group_count(const int32_t *ord, const int32_t *ord2, int64_t n, int l1, int l2, uint32_t *bsum) {
    __shared__ uint32_t wsum[BS / WAVE];
    const int64_t b0 = (int64_t)blockIdx.x * TILE + threadIdx.x * ITEMS;
    uint32_t c = 0;
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t p = b0 + i;
        if (p < n) c += pass_group(ord, ord2, p, l1, l2);
    }
    uint32_t tot;
    (void)block_excl_scan(c, wsum, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// pre[p] = group-1 positions before p (exclusive prefix over the whole pass;
// pre[n] = the total), from the scanned block counts
__global__ void group_prefix(const int32_t *ord, const int32_t *ord2, int64_t n, int l1, int l2,
                             const uint32_t *boff, uint32_t *pre) {
    __shared__ uint32_t wsum[BS / WAVE];
    const int64_t b0 = (int64_t)blockIdx.x * TILE + threadIdx.x * ITEMS;
    uint32_t f[ITEMS];
    uint32_t c = 0;
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t p = b0 + i;
        f[i] = p < n ? pass_group(ord, ord2, p, l1, l2) : 0u;
        c += f[i];
    }
    uint32_t tot;
    uint32_t run = boff[blockIdx.x] + block_excl_scan(c, wsum, tot);
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t p = b0 + i;
        if (p < n) pre[p] = run;
        if (p == n - 1) pre[n] = run + f[i];
        run += f[i];
    }
}

// dst: each aligned segment of 2^seglog2 positions as its group-0 positions
// followed by its group-1 positions, both in input order (stable)
__global__ void group_scatter(const int32_t *ord, const int32_t *ord2, int64_t n, int l1, int l2, int seglog2,
                              const uint32_t *pre, int32_t *dst) {
    const int64_t seg = int64_t(1) << seglog2;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s0 = p & ~(seg - 1);
        const int64_t send = s0 + seg < n ? s0 + seg : n;
        const int64_t ones_before = (int64_t)(pre[p] - pre[s0]);
        const int64_t ones = (int64_t)(pre[send] - pre[s0]);
        const int64_t zeros = (send - s0) - ones;
        const int64_t d = pass_group(ord, ord2, p, l1, l2) ? s0 + zeros + ones_before : p - ones_before;
        dst[d] = ord[p];
    }
}

// iperm[perm[c]] = c: caller index -> canonical index
__global__ void invert_perm(const int32_t *perm, int64_t n, int32_t *iperm) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        iperm[perm[c]] = (int32_t)c;
}

__global__ void gather_coords(const double *x, int64_t ldx, int64_t n, int d, const int32_t *perm,
                              double *xc) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[c];
        for (int k = 0; k < d; ++k) xc[k * n + c] = x[k * ldx + i];
    }
}

// Geometry of one pass in pass order.  d = 2 (pass = x1 level l1): the
// point's x1 half within its node, its x1 offset from the node's split point
// (the first point of the right half) and its x2.  d = 3 (pass = (l1, l2)):
// also the x2 half within the x2 node and the x2 offset from that node's split.
template <int D>
__global__ void pass_geo_kernel(const int32_t *ord, const int32_t *ord2, int l1, int l2, const double *xc,
                                int64_t n, uint32_t *cf, double *xs, double *w1, double *w2) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        if constexpr (D == 2) {
            const int64_t c = ord[p];
            const uint32_t side1 = (uint32_t)((c >> l1) & 1);
            int64_t sp = ((c >> (l1 + 1)) << (l1 + 1)) + (int64_t(1) << l1);
            if (sp > n - 1) sp = n - 1;
            w1[p] = fabs(xc[c] - xc[sp]);
            xs[p] = xc[n + c];
            cf[p] = (uint32_t)c | (side1 << 30);
        } else {
            const int64_t q = ord[p];
            const int64_t c = ord2[q];
            const uint32_t side1 = (uint32_t)((c >> l1) & 1);
            const uint32_t side2 = (uint32_t)((q >> l2) & 1);
            int64_t sp1 = ((c >> (l1 + 1)) << (l1 + 1)) + (int64_t(1) << l1);
            if (sp1 > n - 1) sp1 = n - 1;
            int64_t sq2 = ((q >> (l2 + 1)) << (l2 + 1)) + (int64_t(1) << l2);
            if (sq2 > n - 1) sq2 = n - 1;
            w1[p] = fabs(xc[c] - xc[sp1]);
            w2[p] = fabs(xc[n + c] - xc[n + ord2[sq2]]);
            xs[p] = xc[2 * n + c];
            cf[p] = (uint32_t)c | (side1 << 30) | (side2 << 31);
        }
    }
}

__global__ void invert_kernel(const int32_t *ord, int64_t n, int32_t *inv) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        inv[ord[q]] = (int32_t)q;
}

__global__ void compose_kernel(const int32_t *inv, const int32_t *ord, int64_t n, int32_t *out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        out[p] = inv[ord[p]];
}

inline unsigned grid_for(int64_t n, int bs = BS) {
    int64_t g = (n + bs - 1) / bs;
    if (g > 65535 * 4) g = 65535 * 4;
    return (unsigned)(g < 1 ? 1 : g);
}

// Scratch used while building a plan.
struct BuildTmp {
    DevBuf k0, k1, v0, v1, counts, orand, bad;
};

// Sort `vals` (n int32) by `keys` (n u64) stably; the result ends in tmp.v0/k0.
mm_status radix_sort(BuildTmp &tmp, int64_t n, hipStream_t s) {
    const int64_t nb = (n + TILE - 1) / TILE;
    unsigned long long h_orand[2];
    MM_HIP_TRY(hipMemcpyAsync(h_orand, tmp.orand.ptr, sizeof h_orand, hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    const uint64_t diff = (uint64_t)(h_orand[0] ^ h_orand[1]);
    uint64_t *ka = static_cast<uint64_t *>(tmp.k0.ptr), *kb = static_cast<uint64_t *>(tmp.k1.ptr);
    int32_t *va = static_cast<int32_t *>(tmp.v0.ptr), *vb = static_cast<int32_t *>(tmp.v1.ptr);
    uint32_t *counts = static_cast<uint32_t *>(tmp.counts.ptr);
    int swaps = 0;
    for (int dpos = 0; dpos < 16; ++dpos) {
        const int shift = 4 * dpos;
        if (((diff >> shift) & 0xF) == 0) continue;  // digit equal in every key
        hipLaunchKernelGGL(radix_count, dim3((unsigned)nb), dim3(BS), 0, s, ka, n, shift, counts, nb);
        hipLaunchKernelGGL(scan_single, dim3(1), dim3(1024), 0, s, counts, (int64_t)RADIX * nb);
        hipLaunchKernelGGL(radix_scatter, dim3((unsigned)nb), dim3(BS), 0, s, ka, va, kb, vb, n, shift,
                           counts, nb);
        std::swap(ka, kb);
        std::swap(va, vb);
        ++swaps;
    }
    MM_HIP_TRY(hipGetLastError());
    if (swaps & 1) {
        MM_HIP_TRY(hipMemcpyAsync(tmp.k0.ptr, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        MM_HIP_TRY(hipMemcpyAsync(tmp.v0.ptr, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    return MM_OK;
}

// keys of column x (n doubles) with values 0..n-1, then a stable sort: tmp.v0 = order.
mm_status sort_column(BuildTmp &tmp, const double *x, int64_t n, hipStream_t s, bool check_bad) {
    unsigned long long init[2] = {~0ull, 0ull};
    MM_HIP_TRY(hipMemcpyAsync(tmp.orand.ptr, init, sizeof init, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(keys_kernel, dim3(grid_for(n)), dim3(BS), 0, s, x, n,
                       static_cast<uint64_t *>(tmp.k0.ptr), static_cast<int32_t *>(tmp.v0.ptr),
                       static_cast<unsigned long long *>(tmp.orand.ptr),
                       static_cast<int *>(tmp.bad.ptr));
    MM_HIP_TRY(hipGetLastError());
    (void)check_bad;
    return radix_sort(tmp, n, s);
}

// stable partition of src into dst by `bit` inside aligned segments of 2^seglog2
mm_status partition(BuildTmp &tmp, const int32_t *src, int32_t *dst, int64_t n, int bit, int seglog2,
                    hipStream_t s) {
    const int64_t nb = (n + TILE - 1) / TILE;
    uint32_t *bs = static_cast<uint32_t *>(tmp.counts.ptr);
    hipLaunchKernelGGL(part_count, dim3((unsigned)nb), dim3(BS), 0, s, src, n, bit, bs);
    hipLaunchKernelGGL(scan_single, dim3(1), dim3(1024), 0, s, bs, nb);
    hipLaunchKernelGGL(part_scatter, dim3((unsigned)nb), dim3(BS), 0, s, src, dst, n, bit, seglog2, bs);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

// d = 3: split every segment of pass (l1, l2) by orthant group (see
// pass_group) into dst; pre (n + 1 uint32) and the block counts are scratch.
mm_status group_split(BuildTmp &tmp, const int32_t *ord, const int32_t *ord2, int64_t n, int l1, int l2,
                      int seglog2, uint32_t *pre, int32_t *dst, hipStream_t s) {
    const int64_t nb = (n + TILE - 1) / TILE;
    uint32_t *bs = static_cast<uint32_t *>(tmp.counts.ptr);
    hipLaunchKernelGGL(group_count, dim3((unsigned)nb), dim3(BS), 0, s, ord, ord2, n, l1, l2, bs);
    hipLaunchKernelGGL(scan_single, dim3(1), dim3(1024), 0, s, bs, nb);
    hipLaunchKernelGGL(group_prefix, dim3((unsigned)nb), dim3(BS), 0, s, ord, ord2, n, l1, l2, bs, pre);
    hipLaunchKernelGGL(group_scatter, dim3(grid_for(n)), dim3(BS), 0, s, ord, ord2, n, l1, l2, seglog2, pre, dst);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

// Levels of the (x1, xk) structure: lev[l] lists, for every x1-rank node of
// 2^(l+1) canonical indices, its members in xk order.  `sorted` holds all
// canonical indices in xk order (the top level).
mm_status build_levels(BuildTmp &tmp, const int32_t *sorted, int32_t *lev, int64_t n, int L,
                       hipStream_t s) {
    if (L == 0) return MM_OK;
    MM_HIP_TRY(hipMemcpyAsync(lev + (int64_t)(L - 1) * n, sorted, n * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
    for (int l = L - 2; l >= 0; --l)
        MM_TRY(partition(tmp, lev + (int64_t)(l + 1) * n, lev + (int64_t)l * n, n, l + 1, l + 2, s));
    return MM_OK;
}

int ceil_log2(int64_t n) {
    int L = 0;
    while ((int64_t(1) << L) < n) ++L;
    return L;
}

}  // namespace

mm_status validate_kernel(const mm_kernel *k) {
    if (!k) {
        set_error("kernel is NULL");
        return MM_ERR_ARG;
    }
    if (k->two_nu != 1 && k->two_nu != 3 && k->two_nu != 5) {
        set_error("two_nu must be 1, 3 or 5 (got %d)", k->two_nu);
        return MM_ERR_ARG;
    }
    if (k->form != MM_FORM_L1 && k->form != MM_FORM_PRODUCT) {
        set_error("form must be MM_FORM_L1 or MM_FORM_PRODUCT (got %d)", k->form);
        return MM_ERR_ARG;
    }
    if (!(k->lengthscale > 0.0) || !std::isfinite(k->lengthscale)) {
        set_error("lengthscale must be positive and finite");
        return MM_ERR_ARG;
    }
    if (!(k->outputscale2 > 0.0) || !std::isfinite(k->outputscale2)) {
        set_error("outputscale2 must be positive and finite");
        return MM_ERR_ARG;
    }
    return MM_OK;
}

size_t structure_ints(int64_t n, int d) {
    const int L = ceil_log2(n);
    if (d == 1) return 0;
    if (d == 2) return (size_t)L * n;
    return (size_t)L * n + (size_t)L * (L + 1) / 2 * n;
}

// Bytes of the per-pass geometry: 4 (index and halves) + 8 (scan coordinate)
// + 8 per offset coordinate, per point and pass.
size_t geo_bytes(int64_t n, int d) {
    if (d == 1 || n < 2) return 0;
    const int L = ceil_log2(n);
    const size_t npass = d == 2 ? (size_t)L : (size_t)L * (L + 1) / 2;
    return npass * (size_t)n * (4 + 8 * (size_t)d);
}

size_t plan_footprint(int64_t n, int d, int nrhs, const mm_kernel &k) {
    const int R = rhs_block(k, d, nrhs);
    const int64_t W = (nrhs + R - 1) / R * R;
    // the stored orders and the geometry coexist while the plan is built
    size_t b = (size_t)d * n * 8 + (size_t)n * 8 + structure_ints(n, d) * 4 + geo_bytes(n, d);
    b += 2 * (size_t)n * W * 8;                       // product buffers
    b += sweep_agg_bytes(n, d, (int)W, k);
    {
        int L = ceil_log2(n);
        const int npass = n < 2 ? 0 : (d == 1 ? 1 : (d == 2 ? L : L * (L + 1) / 2));
        b += sweep_part_bytes(n, npass, (int)W);        // per-pass partial results
    }
    b += (size_t)n * 8 * 8 * (size_t)(d + 2);          // CG vectors for the fixed-effects solve
    return b;
}

mm_status plan_build(mm_plan p, const double *x, int64_t ldx, hipStream_t s) {
    const int64_t n = p->n;
    const int d = p->d;
    const int L = ceil_log2(n);
    p->L = L;
    BuildTmp tmp;
    const int64_t nb = (n + TILE - 1) / TILE;
    auto cleanup = [&]() {
        dev_free(tmp.k0); dev_free(tmp.k1); dev_free(tmp.v0); dev_free(tmp.v1);
        dev_free(tmp.counts); dev_free(tmp.orand); dev_free(tmp.bad);
    };
    mm_status st = MM_OK;
#define BUILD_TRY(expr)              \
    do {                             \
        st = (expr);                 \
        if (st != MM_OK) {           \
            cleanup();               \
            return st;               \
        }                            \
    } while (0)
    BUILD_TRY(dev_alloc(tmp.k0, n * 8));
    BUILD_TRY(dev_alloc(tmp.k1, n * 8));
    BUILD_TRY(dev_alloc(tmp.v0, n * 4));
    BUILD_TRY(dev_alloc(tmp.v1, n * 4));
    BUILD_TRY(dev_alloc(tmp.counts, (size_t)(RADIX * nb + 16) * 4));
    BUILD_TRY(dev_alloc(tmp.orand, 16));
    BUILD_TRY(dev_alloc(tmp.bad, 16));
    BUILD_TRY(dev_alloc(p->xc, (size_t)d * n * 8));
    BUILD_TRY(dev_alloc(p->perm, (size_t)n * 4));
    BUILD_TRY(dev_alloc(p->iperm, (size_t)n * 4));

    // finiteness of every coordinate
    if (hipMemsetAsync(tmp.bad.ptr, 0, 16, s) != hipSuccess) { cleanup(); set_error("memset"); return MM_ERR_HIP; }
    hipLaunchKernelGGL(finite_kernel, dim3(grid_for(n)), dim3(BS), 0, s, x, ldx, n, d,
                       static_cast<int *>(tmp.bad.ptr));
    int hbad = 0;
    if (hipMemcpyAsync(&hbad, tmp.bad.ptr, sizeof hbad, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        set_error("HIP error while checking the coordinates: %s", hipGetErrorString(hipGetLastError()));
        return MM_ERR_HIP;
    }
    if (hbad) {
        cleanup();
        set_error("x contains NaN or infinite coordinates");
        return MM_ERR_ARG;
    }

    // canonical order: stable sort by x1
    BUILD_TRY(sort_column(tmp, x, n, s, true));
    if (hipMemcpyAsync(p->perm.ptr, tmp.v0.ptr, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        cleanup(); set_error("copy"); return MM_ERR_HIP;
    }
    hipLaunchKernelGGL(gather_coords, dim3(grid_for(n)), dim3(BS), 0, s, x, ldx, n, d,
                       static_cast<const int32_t *>(p->perm.ptr), static_cast<double *>(p->xc.ptr));
    hipLaunchKernelGGL(invert_perm, dim3(grid_for(n)), dim3(BS), 0, s, static_cast<const int32_t *>(p->perm.ptr),
                       n, static_cast<int32_t *>(p->iperm.ptr));
    const double *xc = static_cast<const double *>(p->xc.ptr);

    p->passes.clear();
    if (n >= 2) {
        if (d == 1) {
            Pass ps;
            ps.seg_log2 = L;
            p->passes.push_back(ps);
        } else {
            BUILD_TRY(dev_alloc(p->structure, structure_ints(n, d) * 4));
            int32_t *ord2 = static_cast<int32_t *>(p->structure.ptr);
            // (x1, x2) levels from one sort by x2 of the canonical points
            BUILD_TRY(sort_column(tmp, xc + n, n, s, false));
            BUILD_TRY(build_levels(tmp, static_cast<const int32_t *>(tmp.v0.ptr), ord2, n, L, s));
            if (d == 2) {
                for (int l = 0; l < L; ++l) {
                    Pass ps;
                    ps.ord = ord2 + (int64_t)l * n;
                    ps.l1 = l;
                    ps.seg_log2 = l + 1;
                    p->passes.push_back(ps);
                }
            } else {
                // (x1, x3) levels (temporary), then per x1 level the x3-ordered
                // positions of the (x1, x2) order, split down the x2 levels.
                DevBuf lev3, inv;
                st = dev_alloc(lev3, (size_t)L * n * 4);
                if (st == MM_OK) st = dev_alloc(inv, (size_t)n * 4);
                if (st != MM_OK) { dev_free(lev3); dev_free(inv); cleanup(); return st; }
                int32_t *o3 = static_cast<int32_t *>(lev3.ptr);
                int32_t *iv = static_cast<int32_t *>(inv.ptr);
                st = sort_column(tmp, xc + 2 * n, n, s, false);
                if (st == MM_OK) st = build_levels(tmp, static_cast<const int32_t *>(tmp.v0.ptr), o3, n, L, s);
                int32_t *pass_base = ord2 + (int64_t)L * n;
                int64_t slot = 0;
                for (int l1 = 0; l1 < L && st == MM_OK; ++l1) {
                    const int32_t *o2l = ord2 + (int64_t)l1 * n;
                    hipLaunchKernelGGL(invert_kernel, dim3(grid_for(n)), dim3(BS), 0, s, o2l, n, iv);
                    int32_t *top = pass_base + (slot + l1) * n;  // pass (l1, l1)
                    hipLaunchKernelGGL(compose_kernel, dim3(grid_for(n)), dim3(BS), 0, s, iv,
                                       o3 + (int64_t)l1 * n, n, top);
                    for (int l2 = l1 - 1; l2 >= 0 && st == MM_OK; --l2)
                        st = partition(tmp, pass_base + (slot + l2 + 1) * n, pass_base + (slot + l2) * n, n,
                                       l2 + 1, l2 + 2, s);
                    for (int l2 = 0; l2 <= l1; ++l2) {
                        Pass ps;
                        ps.ord = pass_base + (slot + l2) * n;
                        ps.ord2 = o2l;
                        ps.l1 = l1;
                        ps.l2 = l2;
                        ps.seg_log2 = l2 + 1;
                        p->passes.push_back(ps);
                    }
                    slot += l1 + 1;
                }
                if (st == MM_OK && hipStreamSynchronize(s) != hipSuccess) {
                    set_error("HIP error while building the structure: %s", hipGetErrorString(hipGetLastError()));
                    st = MM_ERR_HIP;
                }
                dev_free(lev3);
                dev_free(inv);
                if (st != MM_OK) { cleanup(); return st; }
            }
        }
    }
    // geometry of every pass in pass order; the orders are not needed afterwards
    if (d >= 2 && n >= 2) {
        BUILD_TRY(dev_alloc(p->geo, geo_bytes(n, d)));
        const size_t np = p->passes.size();
        double *g = static_cast<double *>(p->geo.ptr);
        double *gxs = g;
        double *gw1 = g + np * n;
        double *gw2 = d == 3 ? g + 2 * np * n : nullptr;
        uint32_t *gcf = reinterpret_cast<uint32_t *>(g + (size_t)d * np * n);
        for (size_t i = 0; i < np; ++i) {
            Pass &ps = p->passes[i];
            ps.xs = gxs + i * n;
            ps.w1 = gw1 + i * n;
            ps.w2 = d == 3 ? gw2 + i * n : nullptr;
            ps.cf = gcf + i * n;
            if (d == 2)
                hipLaunchKernelGGL(pass_geo_kernel<2>, dim3(grid_for(n)), dim3(BS), 0, s, ps.ord, ps.ord2, ps.l1,
                                   ps.l2, xc, n, const_cast<uint32_t *>(ps.cf), const_cast<double *>(ps.xs),
                                   const_cast<double *>(ps.w1), nullptr);
            else {
                // the segments split by orthant group first (tmp.k0 holds the prefix counts)
                int32_t *split = static_cast<int32_t *>(tmp.v1.ptr);
                BUILD_TRY(group_split(tmp, ps.ord, ps.ord2, n, ps.l1, ps.l2, ps.seg_log2,
                                      static_cast<uint32_t *>(tmp.k0.ptr), split, s));
                hipLaunchKernelGGL(pass_geo_kernel<3>, dim3(grid_for(n)), dim3(BS), 0, s, split, ps.ord2, ps.l1,
                                   ps.l2, xc, n, const_cast<uint32_t *>(ps.cf), const_cast<double *>(ps.xs),
                                   const_cast<double *>(ps.w1), const_cast<double *>(ps.w2));
            }
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) {
        set_error("HIP error while building the plan: %s", hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    dev_free(p->structure);
    for (Pass &ps : p->passes) {
        ps.ord = nullptr;
        ps.ord2 = nullptr;
    }
    MM_TRY(upload_pass_tables(p));
#undef BUILD_TRY
    return MM_OK;
}

}  // namespace mm
