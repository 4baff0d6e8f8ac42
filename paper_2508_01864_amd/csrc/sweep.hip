// Host side of the sweeps: workspace sizing, pass tables, the per-product
// launch sequence and the batched launches.  The kernels and their
// configurations are in sweep_core.h.

#include "sweep_core.h"

#include <algorithm>

namespace mm {

// Columns per wave (the padding unit of the number of right-hand sides):
// 32 from 32 columns up, 4 from 4, else 2 or 1.
int rhs_block(const mm_kernel &k, int d, int nrhs) {
    (void)k;
    (void)d;
    return nrhs >= 32 ? 32 : (nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1));
}

// Passes per group: the partial slabs of one group stay within 1 GiB.
constexpr size_t PART_BUDGET = size_t(1) << 30;

static int group_size(int64_t n, int npass, int W) {
    const size_t slabb = (size_t)n * W * sizeof(double);
    int64_t g = (int64_t)(PART_BUDGET / (slabb > 0 ? slabb : 1));
    if (g < 1) g = 1;
    if (g > npass) g = npass;
    return (int)(g < 1 ? 1 : g);
}

int group_passes(mm_plan p, int W) { return group_size(p->n, (int)p->passes.size(), W); }

size_t sweep_part_bytes(int64_t n, int npass, int W) {
    if (npass == 0) return 0;
    return (size_t)group_size(n, npass, W) * n * W * sizeof(double);
}

// Doubles of one tile aggregate per right-hand side: classes x channel rows
// x scan channels (the configuration's FULLSLOT), for the kernel and, with
// der, also for its lengthscale-derivative sweeps (one more channel in one
// factor).  At most 2 x 9 x 3 = 54 for the kernel and 72 with der (d = 3,
// product form, nu = 5/2).
int agg_per_rhs(int d, const mm_kernel &k, bool der) {
    const KParams kp = kparams(k, d);
    const int ncls = d == 1 ? 1 : 2;  // two classes (the x1 half) in d = 2 and, per orthant group, in d = 3
    int best = 0;
    for (int gj = -1; gj < (der ? d : 0); ++gj) {
        if (!kp.prod && gj >= 0 && gj != d - 1) continue;
        int nth = 1;
        if (kp.prod)
            for (int c = 0; c < d - 1; ++c) nth *= kp.P + (gj == c ? 1 : 0);
        const int ps = kp.P + (gj == d - 1 ? 1 : 0);
        best = std::max(best, ncls * nth * ps);
    }
    return best;
}

// Aggregates and carries: agg_per_rhs doubles per tile and right-hand side,
// two directions, per pass of a group; anchors and decays 2 each per tile and
// pass.  The smallest tile (128 positions) gives the most tiles.  For d <= 2,
// also the runs' within-tile carries of the cross-tile passes: agg_per_rhs
// doubles per lane, two directions, per run of at least 8 positions -- at most
// 32 lanes per column per 256 positions.  (The slab budget caps G n W, so this
// stays below agg_per_rhs / 4 GiB at any width.)
static size_t agg_bytes_for(int64_t n, int d, int W, int64_t G, int per_rhs) {
    const int64_t ntile = (n + 127) / 128;
    size_t dbl = (size_t)(2 * (2 * G * ntile * (int64_t)W * per_rhs) + 4 * G * ntile + 16);
    if (d <= 2) dbl += (size_t)2 * G * ((n + 255) / 256) * 32 * W * per_rhs;
    return dbl * sizeof(double);
}

size_t sweep_agg_bytes(int64_t n, int d, int W, const mm_kernel &k, bool der) {
    int L = 0;
    while ((int64_t(1) << L) < n) ++L;
    const int npass = n < 2 ? 0 : (d == 1 ? 1 : (d == 2 ? L : L * (L + 1) / 2));
    const int64_t G = npass == 0 ? 1 : group_size(n, npass, W);
    return agg_bytes_for(n, d, W, G, agg_per_rhs(d, k, der));
}

// A batched problem runs all its passes as one group, its partial slabs in a
// workspace of its own; up to 16 GiB of them per problem.
constexpr size_t BATCH_PART_BUDGET = size_t(16) << 30;

bool sweep_batch_bytes_n(int64_t n, int d, const mm_kernel &k, int npass, int W, size_t *agg_bytes,
                         size_t *part_bytes) {
    const size_t slab = (size_t)n * W * sizeof(double);
    if (npass > 0 && (size_t)npass * slab > BATCH_PART_BUDGET) return false;
    const int64_t G = npass > 0 ? npass : 1;
    *part_bytes = (size_t)G * slab;
    *agg_bytes = agg_bytes_for(n, d, W, G, agg_per_rhs(d, k, false));
    return true;
}

bool sweep_batch_bytes(mm_plan p, int W, size_t *agg_bytes, size_t *part_bytes) {
    return sweep_batch_bytes_n(p->n, p->d, p->kernel, (int)p->passes.size(), W, agg_bytes, part_bytes);
}

mm_status upload_pass_tables(mm_plan p) {
    std::vector<PassDev> tab;
    for (int ti = 0; ti < mm_plan_s::NTS; ++ti) p->xt_host[ti].clear();
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const Pass &q = p->passes[i];
        PassDev dv{q.cf, q.xs, q.w1, q.w2, q.l1, q.l2, q.seg_log2, 0};
        tab.push_back(dv);
        for (int ti = 0; ti < mm_plan_s::NTS; ++ti)
            if (q.seg_log2 > 7 + ti) p->xt_host[ti].push_back((int)i);
    }
    if (tab.empty()) return MM_OK;
    MM_TRY(dev_alloc(p->pass_dev, tab.size() * sizeof(PassDev)));
    MM_HIP_TRY(hipMemcpy(p->pass_dev.ptr, tab.data(), tab.size() * sizeof(PassDev), hipMemcpyHostToDevice));
    for (int ti = 0; ti < mm_plan_s::NTS; ++ti) {
        if (p->xt_host[ti].empty()) continue;
        std::vector<int32_t> pos(p->passes.size(), -1);
        for (size_t k = 0; k < p->xt_host[ti].size(); ++k) pos[p->xt_host[ti][k]] = (int32_t)k;
        MM_TRY(dev_alloc(p->pass_xtpos[ti], pos.size() * sizeof(int32_t)));
        MM_HIP_TRY(hipMemcpy(p->pass_xtpos[ti].ptr, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        MM_TRY(dev_alloc(p->pass_xt[ti], p->xt_host[ti].size() * sizeof(int32_t)));
        MM_HIP_TRY(hipMemcpy(p->pass_xt[ti].ptr, p->xt_host[ti].data(), p->xt_host[ti].size() * sizeof(int32_t),
                             hipMemcpyHostToDevice));
        // segments (pass, first tile, end tile) of the cross-tile passes, and the
        // offset of each pass's first segment (seg_off[k] for xt entry k)
        const int64_t T = int64_t(128) << ti;
        const int64_t ntile = (p->n + T - 1) / T;
        std::vector<int4> tab4;
        p->seg_off[ti].clear();
        for (int pi : p->xt_host[ti]) {
            p->seg_off[ti].push_back((int)tab4.size());
            const int64_t tps = (int64_t(1) << p->passes[pi].seg_log2) / T;
            for (int64_t t0 = 0; t0 < ntile; t0 += tps) {
                const int64_t t1 = t0 + tps < ntile ? t0 + tps : ntile;
                if (t1 - t0 >= 2) tab4.push_back(make_int4(pi, (int)t0, (int)t1, 0));
            }
        }
        p->seg_off[ti].push_back((int)tab4.size());
        p->seg_host[ti] = tab4;
        if (!tab4.empty()) {
            MM_TRY(dev_alloc(p->seg_tab[ti], tab4.size() * sizeof(int4)));
            MM_HIP_TRY(hipMemcpy(p->seg_tab[ti].ptr, tab4.data(), tab4.size() * sizeof(int4), hipMemcpyHostToDevice));
        }
        // the segments the carry scan gives a wave per slice (more than CARRY_SMALL
        // tiles), listed apart so that a product's carry launch sizes each kind's blocks
        std::vector<int32_t> big;
        p->big_off[ti].clear();
        for (size_t k = 0; k + 1 < p->seg_off[ti].size(); ++k) {
            p->big_off[ti].push_back((int)big.size());
            for (int sg = p->seg_off[ti][k]; sg < p->seg_off[ti][k + 1]; ++sg)
                if (tab4[sg].z - tab4[sg].y > CARRY_SMALL) big.push_back(sg);
        }
        p->big_off[ti].push_back((int)big.size());
        if (!big.empty()) {
            MM_TRY(dev_alloc(p->seg_big[ti], big.size() * sizeof(int32_t)));
            MM_HIP_TRY(hipMemcpy(p->seg_big[ti].ptr, big.data(), big.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        }
    }
    return MM_OK;
}

Sched plan_sched(mm_plan p, int W, int WB) {
    for (const auto &e : p->sched)
        if (e.first == W) return e.second;
    return Sched{WB, 0, 1};
}

bool sched_available(int d, const KParams &kp, const Sched &sc, int W) { return sched_compiled(d, kp, sc, W); }

// WB: the default column block (1, 2, 4 or 32); W a multiple of WB.  The plan's
// schedule for W, if one was set, replaces the default.
mm_status sweep_all(mm_plan p, const double *vin, double *yacc, int W, int WB, hipStream_t s, int *tail,
                    const SweepWs *ws) {
    const KParams kp = kparams(p->kernel, p->d);
    if ((WB != 1 && WB != 2 && WB != 4 && WB != 32) || W % WB != 0) {
        set_error("internal: width %d does not match the block %d", W, WB);
        return MM_ERR_ARG;
    }
    const Sched sc = plan_sched(p, W, WB);
    return with_cfg(p->d, kp, sc, W, [&](auto t) {
        using C = typename decltype(t)::type;
        return run_passes<C>(p, vin, yacc, W, s, false, tail, ws, sc.runex);
    });
}

// ---------------------------------------------------------------------------
// Batched sweeps: several problems (each with its own plan) of the same width
// W in one launch per kernel configuration and phase.  The tables list work
// items (problem, block x, block y); a fixed grid walks them.
// ---------------------------------------------------------------------------
namespace {
__global__ void accum_batch_kernel(const AccumDesc *descs, const int2 *items, int nitems) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const AccumDesc d = descs[it.x];
        const int64_t lo = (int64_t)it.y * ACC_CHUNK;
        const int64_t hi = lo + ACC_CHUNK < d.len ? lo + ACC_CHUNK : d.len;
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            double sum = 0.0;
            for (int g = 0; g < d.G; ++g) sum += d.ypart[(int64_t)g * d.len + e];
            d.yacc[e] = sum;
        }
    }
}

template <class T>
mm_status upload(DevBuf &b, const std::vector<T> &v) {
    if (v.empty()) return MM_OK;
    MM_TRY(dev_alloc(b, v.size() * sizeof(T)));
    MM_HIP_TRY(hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return MM_OK;
}

inline unsigned persist_grid(int nitems, int per_cu) {
    int64_t g = (int64_t)256 * per_cu;
    if (g > nitems) g = nitems;
    return (unsigned)(g < 1 ? 1 : g);
}
}  // namespace

mm_status sweep_batch_build(const std::vector<BatchEntry> &probs, int W, int WB, SweepBatch &out) {
    sweep_batch_free(out);
    out.W = W;
    out.WB = WB;
    for (const BatchEntry &e : probs) out.plans.push_back(e.p);
    // group the problems by kernel configuration
    std::vector<int> keys;
    for (size_t k = 0; k < probs.size(); ++k) {
        mm_plan p = probs[k].p;
        const KParams kp = kparams(p->kernel, p->d);
        const Sched sc = plan_sched(p, W, WB);
        // one class per kernel configuration and schedule
        const int key = ((((p->d * 4 + kp.P) * 2 + (kp.prod ? 1 : 0)) * 64 + sc.wb) * 256 + sc.e) * 2 + sc.runex;
        size_t c = 0;
        while (c < keys.size() && keys[c] != key) ++c;
        if (c == keys.size()) {
            keys.push_back(key);
            out.classes.emplace_back();
            out.classes.back().key = key;
            out.classes.back().d = p->d;
            out.classes.back().kp = kp;
            out.classes.back().sc = sc;
        }
        out.classes[c].members.push_back((int)k);
        size_t ab = 0, pb = 0;
        if (!sweep_batch_bytes(p, W, &ab, &pb)) {
            set_error("batched product: problem %zu needs several pass groups at width %d", k, W);
            return MM_ERR_ARG;
        }
    }
    std::vector<AccumDesc> ad;
    std::vector<int2> ai;
    for (size_t k = 0; k < probs.size(); ++k) {
        mm_plan p = probs[k].p;
        AccumDesc d{probs[k].part, probs[k].yacc, (int64_t)p->n * W, (int)p->passes.size()};
        ad.push_back(d);
        const int64_t nch = (d.len + ACC_CHUNK - 1) / ACC_CHUNK;
        for (int64_t c = 0; c < nch; ++c) ai.push_back(make_int2((int)k, (int)c));
    }
    MM_TRY(upload(out.acc_desc, ad));
    MM_TRY(upload(out.acc_items, ai));
    out.n_acc = (int)ai.size();
    for (auto &cl : out.classes) {
        MM_TRY(with_cfg(cl.d, cl.kp, cl.sc, W, [&](auto t) {
            using C = typename decltype(t)::type;
            const int ti = tile_index(C::T);
            std::vector<SweepArgs> descs;
            std::vector<int4> ia, ic, im;
            for (size_t m = 0; m < cl.members.size(); ++m) {
                const BatchEntry &e = probs[cl.members[m]];
                mm_plan p = e.p;
                const int npass = (int)p->passes.size();
                SweepArgs A = make_args<C>(p, e.vin, e.agg, e.part, W, npass > 0 ? npass : 1, cl.sc.runex);
                descs.push_back(A);
                if (npass == 0) continue;
                const int ncb = W / C::WCOL;
                const int64_t nxt = (int64_t)p->xt_host[ti].size();
                if (A.ntile > 1)
                    for (int64_t bx = 0; bx < nxt * A.ntile; ++bx)
                        for (int by = 0; by < ncb; ++by) ia.push_back(make_int4((int)m, (int)bx, by, 0));
                const int nseg = p->seg_off[ti].empty() ? 0 : p->seg_off[ti].back();
                if (A.ntile > 1)
                    for (int sg = 0; sg < nseg; ++sg) {
                        const int4 g = p->seg_host[ti][sg];
                        // (direction, slice) pairs: threads of one block, or one wave each
                        const int nby = (g.z - g.y <= CARRY_SMALL) ? (2 * A.nslice + 255) / 256 : (2 * A.nslice + 3) / 4;
                        for (int by = 0; by < nby; ++by) ic.push_back(make_int4((int)m, sg, by, 0));
                    }
                for (int64_t bx = 0; bx < (int64_t)npass * A.ntile; ++bx)
                    for (int by = 0; by < ncb; ++by) im.push_back(make_int4((int)m, (int)bx, by, 0));
            }
            if (ia.size() > (size_t)INT32_MAX || ic.size() > (size_t)INT32_MAX || im.size() > (size_t)INT32_MAX) {
                set_error("batched product: more than 2^31-1 work items in one kernel class");
                return MM_ERR_ARG;
            }
            MM_TRY(upload(cl.descs, descs));
            MM_TRY(upload(cl.items_agg, ia));
            MM_TRY(upload(cl.items_carry, ic));
            MM_TRY(upload(cl.items_main, im));
            cl.n_agg = (int)ia.size();
            cl.n_carry = (int)ic.size();
            cl.n_main = (int)im.size();
            return MM_OK;
        }));
    }
    return MM_OK;
}

mm_status sweep_batch_run(SweepBatch &b, hipStream_t s) {
    for (auto &cl : b.classes) {
        MM_TRY(with_cfg(cl.d, cl.kp, cl.sc, b.W, [&](auto t) {
            using C = typename decltype(t)::type;
            const SweepArgs *descs = static_cast<const SweepArgs *>(cl.descs.ptr);
            if (cl.n_agg > 0)
                hipLaunchKernelGGL((sweep_batch_kernel<C, 1>), dim3(cl.n_agg), dim3(C::BLOCK), 0,
                                   s, descs, static_cast<const int4 *>(cl.items_agg.ptr), cl.n_agg);
            if (cl.n_carry > 0)
                hipLaunchKernelGGL((carry_batch_kernel<C>), dim3(persist_grid(cl.n_carry, b.grid_per_cu)), dim3(256),
                                   0, s, descs, static_cast<const int4 *>(cl.items_carry.ptr), cl.n_carry);
            if (cl.n_main > 0) {
                hipEvent_t ev1 = nullptr;
                if (b.plans.size() == 1) MM_TRY(profile_begin(b.plans[0], (int)b.plans[0]->passes.size(), s, &ev1));
                hipLaunchKernelGGL((sweep_batch_kernel<C, 0>), dim3(cl.n_main), dim3(C::BLOCK),
                                   0, s, descs, static_cast<const int4 *>(cl.items_main.ptr), cl.n_main);
                if (ev1) MM_HIP_TRY(hipEventRecord(ev1, s));
            }
            return MM_OK;
        }));
    }
    if (b.n_acc > 0 && !b.skip_accum)
        hipLaunchKernelGGL(accum_batch_kernel, dim3(persist_grid(b.n_acc, 16)), dim3(256), 0, s,
                           static_cast<const AccumDesc *>(b.acc_desc.ptr), static_cast<const int2 *>(b.acc_items.ptr),
                           b.n_acc);
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

void sweep_batch_free(SweepBatch &b) {
    for (auto &cl : b.classes) {
        dev_free(cl.descs);
        dev_free(cl.items_agg);
        dev_free(cl.items_carry);
        dev_free(cl.items_main);
    }
    b.classes.clear();
    b.plans.clear();
    dev_free(b.acc_desc);
    dev_free(b.acc_items);
    b.n_acc = 0;
}

}  // namespace mm
