// Divide-and-conquer weighted-ECDF sweeps: the hot loop of the exact Matern
// kernel product.
//
// The paper writes the kernel sum over the 2^d sign orthants as weighted
// empirical CDFs (eq. ECDFdelta; Prop. 1 for the L1 kernel, Prop. 2 for the
// product kernel; the Matern instances in Section 2.3) and evaluates all of
// them with a divide-and-conquer over presorted coordinates (Section 2.2).
// Here every pair of distinct points meets in exactly one "pass": the level
// of the x1-rank tree where they fall into different halves (and, in d = 3,
// the level of the x2-rank tree inside that node).  Within a pass the points
// of each node are listed in the order of the last coordinate, and the
// orthant sums become bidirectional segmented scans:
//   forward scan (<=)  gives the orthants with delta_last = +1,
//   backward scan (>)  gives delta_last = -1,
//   the source/target classes (which half of the x1 node, and in d = 3 of
//   the x2 node) give the remaining signs.
//
// Numerics.  The paper's weights exp(+a delta.x) (eq. matern_weights) grow
// without bound and their polynomial companions cancel.  Instead the scan
// carries, per orthant class, the vector
//     S_m = sum_i v_i (a r_i)^m / m! exp(-a r_i),   m = 0..P-1,
// where r_i is the distance from source i to the current scan position.
// Moving the position by Delta >= 0 is the linear map
//     S_m <- exp(-a Delta) sum_{q<=m} (a Delta)^(m-q)/(m-q)! S_q,
// whose coefficients lie in [0, 1]; the offsets of the other coordinates are
// measured from the node's split point, so every factor is a bounded,
// non-negative number and no sign cancellation occurs apart from v's own
// signs.  The profile is recovered with the coefficients
//     k(a r) = sum_m c_m (a r)^m / m! exp(-a r),
//     c = [1] (nu=1/2), [1, 1] (nu=3/2), [1, 1, 2/3] (nu=5/2),
// which restate Appendix C eq. matern_1_2 / 3_2 / 5_2 in this basis.

#include "mm_internal.h"

namespace mm {
namespace {

constexpr int WG = 256;
constexpr int WAVE = 64;
constexpr int NWAVE = WG / WAVE;

template <int B, int E>
struct IPow { static constexpr int v = B * IPow<B, E - 1>::v; };
template <int B>
struct IPow<B, 0> { static constexpr int v = 1; };

// c_m coefficients of the profile in the scaled-power basis.
template <int P>
__device__ __forceinline__ double coef(int m) {
    if constexpr (P == 3) return m == 2 ? (2.0 / 3.0) : 1.0;
    return 1.0;
}

// Source factor s_m(E, t) = E t^m / m!  (t = a w, E = exp(-t)).
template <int P>
__device__ __forceinline__ void src_vec(double E, double t, double (&sv)[P]) {
    sv[0] = E;
    if constexpr (P > 1) sv[1] = E * t;
    if constexpr (P > 2) sv[2] = E * t * t * 0.5;
}

// Target factor g_q(E, t) = E sum_{m>=q} c_m t^(m-q)/(m-q)!: the profile
// coefficients moved across an offset t (k(a(u+w)) = sum_q g_q(u) s_q(w)).
template <int P>
__device__ __forceinline__ void tgt_vec(double E, double t, double (&gv)[P]) {
    if constexpr (P == 1) {
        gv[0] = E;
    } else if constexpr (P == 2) {
        gv[0] = E * (1.0 + t);
        gv[1] = E;
    } else {
        gv[0] = E * (1.0 + t + t * t * (1.0 / 3.0));
        gv[1] = E * (1.0 + t * (2.0 / 3.0));
        gv[2] = E * (2.0 / 3.0);
    }
}

// Flags stored with each staged element.
constexpr int F_SIDE1 = 1;     // x1 half (d >= 2)
constexpr int F_SIDE2 = 2;     // x2 half (d = 3)
constexpr int F_SEGSTART = 4;  // first position of a segment
constexpr int F_SEGEND = 8;    // last position of a segment (or of the array)
constexpr int F_VALID = 16;    // position < n

// One divide-and-conquer pass as the kernels see it (device table).
struct PassDev {
    const int32_t *ord;   // position -> canonical index (d = 2) or q (d = 3)
    const int32_t *ord2;  // d = 3: q -> canonical index at level l1
    int l1, l2;
    int seg_log2;         // segments of 2^seg_log2 positions
    int pad;
};

// Kernel arguments for one group of passes.
struct SweepArgs {
    const double *xc;      // d x n canonical coordinates
    const PassDev *passes; // every pass of the plan
    const int32_t *xt;     // indices of the passes whose segments span several tiles
    const double *vin;     // n x W point-major canonical input
    double *ypart;         // G slabs of n x W: one partial result per pass of the group
    double *agg;           // tile aggregates [2 dirs][G][ntile][nrb][NHALF][NSLOT]
    double *anc;           // tile anchors [2 dirs][G][ntile]
    int64_t n;
    int64_t ntile;
    int W;                 // leading width of vin / ypart (columns)
    int g0;                // first pass of the group
    int k0;                // first entry of xt inside the group
    int G;                 // passes in the group
    double a;
};

// Static configuration of a sweep instance.
template <int D_, int P_, bool PROD_, int R_, int E_>
struct Cfg {
    static constexpr int D = D_;
    static constexpr int P = P_;
    static constexpr bool PROD = PROD_;
    static constexpr int R = R_;
    static constexpr int E = E_;
    static constexpr int T = WG * E;                       // tile positions
    static constexpr int NTH = PROD ? IPow<P, D - 1>::v : 1; // non-scan channel rows
    // source classes (orthants of the non-scan coordinates) and how many
    // sub-sweeps they are split over so that one state fits the register file
    static constexpr int NCLS_ALL = (D == 1) ? 1 : (D == 2 ? 2 : 4);
    static constexpr int FULLSLOT = NCLS_ALL * NTH * P;
    static constexpr int NHALF = (D == 3) ? (FULLSLOT <= 16 ? 1 : (FULLSLOT <= 32 ? 2 : 4)) : 1;
    static constexpr int NCLS = NCLS_ALL / NHALF;
    static constexpr int NSLOT = NCLS * NTH * P * R;       // doubles per state
    static constexpr int G = 2 * (D - 1);                  // staged geometry doubles
};

template <class C>
struct State {
    double s[C::NCLS][C::NTH][C::P][C::R];

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
            for (int h = 0; h < C::NTH; ++h)
#pragma unroll
                for (int m = 0; m < C::P; ++m)
#pragma unroll
                    for (int r = 0; r < C::R; ++r) s[c][h][m][r] = 0.0;
    }

    // this <- M(E, t) this
    __device__ __forceinline__ void shift(double E, double t) {
        const double t2 = 0.5 * t * t;
#pragma unroll
        for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
            for (int h = 0; h < C::NTH; ++h)
#pragma unroll
                for (int r = 0; r < C::R; ++r) {
                    if constexpr (C::P == 3) s[c][h][2][r] = E * (s[c][h][2][r] + t * s[c][h][1][r] + t2 * s[c][h][0][r]);
                    if constexpr (C::P >= 2) s[c][h][1][r] = E * (s[c][h][1][r] + t * s[c][h][0][r]);
                    s[c][h][0][r] = E * s[c][h][0][r];
                }
    }

    // this <- this + M(E, t) o
    __device__ __forceinline__ void add_shifted(const State &o, double E, double t) {
        const double t2 = 0.5 * t * t;
#pragma unroll
        for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
            for (int h = 0; h < C::NTH; ++h)
#pragma unroll
                for (int r = 0; r < C::R; ++r) {
                    if constexpr (C::P == 3) s[c][h][2][r] += E * (o.s[c][h][2][r] + t * o.s[c][h][1][r] + t2 * o.s[c][h][0][r]);
                    if constexpr (C::P >= 2) s[c][h][1][r] += E * (o.s[c][h][1][r] + t * o.s[c][h][0][r]);
                    s[c][h][0][r] += E * o.s[c][h][0][r];
                }
    }

    __device__ __forceinline__ double *flat() { return &s[0][0][0][0]; }
    __device__ __forceinline__ const double *flat() const { return &s[0][0][0][0]; }
};

// Geometry of one element (source and target vectors) derived from its staged offsets.
//   product form: f[th] = prod_k s_{th_k}(w_k) (source, enters the m = 0 slot),
//                 g[th] = prod_k g_{th_k}(w_k) (target, times the profile coefficients c_m);
//   L1 form:      f[m] = s_m(W), g[m] = g_m(W) with W the summed offset.
template <class C>
struct ElemVec {
    double f[C::NTH][C::PROD ? 1 : C::P];
    double g[C::PROD ? C::NTH : C::P];
};

template <class C>
__device__ __forceinline__ void elem_vectors(const double *geo, ElemVec<C> &ev) {
    constexpr int P = C::P;
    if constexpr (C::D == 1) {  // no other coordinate: unit source and target
        static_assert(C::D != 1 || C::PROD, "d = 1 uses the product path");
        ev.f[0][0] = 1.0;
        ev.g[0] = 1.0;
        return;
    } else if constexpr (C::PROD) {
        double sv[C::D - 1][P];
        double gv[C::D - 1][P];
#pragma unroll
        for (int k = 0; k < C::D - 1; ++k) {
            src_vec<P>(geo[2 * k], geo[2 * k + 1], sv[k]);
            tgt_vec<P>(geo[2 * k], geo[2 * k + 1], gv[k]);
        }
#pragma unroll
        for (int th = 0; th < C::NTH; ++th) {
            double fs = 1.0, gs = 1.0;
            int rem = th;
#pragma unroll
            for (int k = 0; k < C::D - 1; ++k) {
                const int idx = rem % P;
                rem /= P;
                fs *= sv[k][idx];
                gs *= gv[k][idx];
            }
            ev.f[th][0] = fs;
            ev.g[th] = gs;
        }
    } else {
        // L1: offsets add up; exp of the sum is the product of the exps.
        double E = 1.0, t = 0.0;
#pragma unroll
        for (int k = 0; k < C::D - 1; ++k) {
            E *= geo[2 * k];
            t += geo[2 * k + 1];
        }
        double sv[P], gv[P];
        src_vec<P>(E, t, sv);
        tgt_vec<P>(E, t, gv);
#pragma unroll
        for (int m = 0; m < P; ++m) {
            ev.f[0][m] = sv[m];
            ev.g[m] = gv[m];
        }
    }
}

// S[cls] += v * source vector.  The class is selected through the value
// (v or 0) rather than a branch so the state stays in registers.
template <class C>
__device__ __forceinline__ void add_source(State<C> &S, int cls, const ElemVec<C> &ev,
                                           const double (&v)[C::R]) {
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c) {
#pragma unroll
        for (int r = 0; r < C::R; ++r) {
            const double vc = (c == cls) ? v[r] : 0.0;
#pragma unroll
            for (int h = 0; h < C::NTH; ++h) {
                if constexpr (C::PROD) {
                    S.s[c][h][0][r] += ev.f[h][0] * vc;
                } else {
#pragma unroll
                    for (int m = 0; m < C::P; ++m) S.s[c][h][m][r] += ev.f[h][m] * vc;
                }
            }
        }
    }
}

// out += target vector . S[cls]
template <class C>
__device__ __forceinline__ void read_target(const State<C> &S, int cls, const ElemVec<C> &ev,
                                            double (&out)[C::R]) {
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c) {
#pragma unroll
        for (int r = 0; r < C::R; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int h = 0; h < C::NTH; ++h) {
                if constexpr (C::PROD) {
                    double row = S.s[c][h][0][r];
#pragma unroll
                    for (int m = 1; m < C::P; ++m) row += coef<C::P>(m) * S.s[c][h][m][r];
                    acc += ev.g[h] * row;
                } else {
#pragma unroll
                    for (int m = 0; m < C::P; ++m) acc += ev.g[m] * S.s[c][h][m][r];
                }
            }
            out[r] += (c == cls) ? acc : 0.0;
        }
    }
}

// Source / target class of an element in sub-sweep `hh`.  d = 2: the x1 half
// (sources of one half feed targets of the other).  d = 3: the (x1, x2)
// halves; a source class feeds the targets in the opposite halves of both.
// With NHALF > 1 each sub-sweep carries only part of the classes.
template <class C>
__device__ __forceinline__ void classes(int flags, int hh, int &scls, int &tcls) {
    if constexpr (C::D == 1) {
        scls = 0;
        tcls = 0;
    } else if constexpr (C::D == 2) {
        const int s1 = flags & F_SIDE1;
        scls = s1;
        tcls = 1 - s1;
    } else {
        const int s1 = flags & F_SIDE1;
        const int s2 = (flags & F_SIDE2) ? 1 : 0;
        const int full = s1 * 2 + s2;
        if constexpr (C::NHALF == 1) {
            scls = full;
            tcls = 3 - full;
        } else if constexpr (C::NHALF == 2) {
            scls = (s1 == hh) ? s2 : -1;
            tcls = (s1 == 1 - hh) ? 1 - s2 : -1;
        } else {
            scls = (full == hh) ? 0 : -1;
            tcls = (3 - full == hh) ? 0 : -1;
        }
    }
    if (!(flags & F_VALID)) {
        scls = -1;
        tcls = -1;
    }
}

// Exchange a state with another lane (DS permute of the 64-bit halves).
template <class C>
__device__ __forceinline__ void shfl_up_state(const State<C> &in, State<C> &out, int delta) {
#pragma unroll
    for (int i = 0; i < C::NSLOT; ++i) out.flat()[i] = __shfl_up(in.flat()[i], delta, WAVE);
}
template <class C>
__device__ __forceinline__ void shfl_down_state(const State<C> &in, State<C> &out, int delta) {
#pragma unroll
    for (int i = 0; i < C::NSLOT; ++i) out.flat()[i] = __shfl_down(in.flat()[i], delta, WAVE);
}

template <class C>
struct Smem {
    int32_t c[C::T];
    int32_t flags[C::T];
    double xs[C::T];
    double est[C::T];
    double geo[C::G > 0 ? C::G : 1][C::T];
    double waveF[NWAVE][C::NSLOT];
    double waveFx[NWAVE];
    double car[2][C::NSLOT];   // carry from the other tiles of the segment, per direction
    double carx[2];            // its anchor
    int carhas[2];
};

// Stage the tile's positions: indices, flags, scan coordinate and offsets.
template <class C>
__device__ __forceinline__ void stage_tile(const SweepArgs &A, const PassDev &ps, Smem<C> &sm,
                                           int64_t p0) {
    const int64_t n = A.n;
    const int64_t segmask = (int64_t(1) << ps.seg_log2) - 1;
    for (int j = threadIdx.x; j < C::T; j += WG) {
        const int64_t p = p0 + j;
        const int64_t pc = p < n ? p : n - 1;
        int flags = p < n ? F_VALID : 0;
        if (p < n && (p & segmask) == 0) flags |= F_SEGSTART;
        if (p >= n - 1 || ((p + 1) & segmask) == 0) flags |= F_SEGEND;
        int64_t c;
        if constexpr (C::D == 1) {
            c = pc;
            sm.xs[j] = A.xc[c];
        } else if constexpr (C::D == 2) {
            c = ps.ord[pc];
            const int l = ps.l1;
            flags |= (int)((c >> l) & 1) ? F_SIDE1 : 0;
            int64_t sp = ((c >> (l + 1)) << (l + 1)) + (int64_t(1) << l);
            if (sp > n - 1) sp = n - 1;
            const double w = fabs(A.xc[c] - A.xc[sp]);
            const double t = A.a * w;
            sm.geo[0][j] = exp(-t);
            sm.geo[1][j] = t;
            sm.xs[j] = A.xc[n + c];
        } else {
            const int64_t q = ps.ord[pc];
            c = ps.ord2[q];
            const int l1 = ps.l1, l2 = ps.l2;
            flags |= (int)((c >> l1) & 1) ? F_SIDE1 : 0;
            flags |= (int)((q >> l2) & 1) ? F_SIDE2 : 0;
            int64_t sp1 = ((c >> (l1 + 1)) << (l1 + 1)) + (int64_t(1) << l1);
            if (sp1 > n - 1) sp1 = n - 1;
            int64_t sq2 = ((q >> (l2 + 1)) << (l2 + 1)) + (int64_t(1) << l2);
            if (sq2 > n - 1) sq2 = n - 1;
            const double w1 = fabs(A.xc[c] - A.xc[sp1]);
            const double w2 = fabs(A.xc[n + c] - A.xc[n + ps.ord2[sq2]]);
            const double t1 = A.a * w1, t2 = A.a * w2;
            sm.geo[0][j] = exp(-t1);
            sm.geo[1][j] = t1;
            sm.geo[2][j] = exp(-t2);
            sm.geo[3][j] = t2;
            sm.xs[j] = A.xc[2 * n + c];
        }
        sm.c[j] = (int32_t)c;
        sm.flags[j] = flags;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < C::T; j += WG) {
        double e = 1.0;
        if (j > 0 && !(sm.flags[j] & F_SEGSTART)) e = exp(-A.a * (sm.xs[j] - sm.xs[j - 1]));
        sm.est[j] = e;
    }
    __syncthreads();
}

template <class C>
__device__ __forceinline__ void load_v(const SweepArgs &A, int c, int rb, double (&v)[C::R]) {
    const double *src = A.vin + (int64_t)c * A.W + rb * C::R;
#pragma unroll
    for (int r = 0; r < C::R; ++r) v[r] = src[r];
}

template <class C>
__device__ __forceinline__ void load_geo(const Smem<C> &sm, int j, double (&geo)[C::G > 0 ? C::G : 1]) {
#pragma unroll
    for (int k = 0; k < C::G; ++k) geo[k] = sm.geo[k][j];
}

template <class C>
__device__ __forceinline__ int64_t agg_index(const SweepArgs &A, int dir, int pl, int tile, int rb,
                                             int nrb, int hh) {
    return (((((int64_t)dir * A.G + pl) * A.ntile + tile) * nrb + rb) * C::NHALF + hh) * C::NSLOT;
}

// One scan direction over this thread's run of E positions, with every carry.
// DIR 0: forward (positions in increasing order, sources at or before the
//        target in the last coordinate: delta_last = +1);
// DIR 1: backward (decreasing order, sources strictly after: delta_last = -1).
// MODE 0 accumulates target values into outv; MODE 1 writes the tile's total.
template <class C, int MODE, int DIR>
__device__ __forceinline__ void run_direction(const SweepArgs &A, const PassDev &ps, Smem<C> &sm,
                                              int hh, int tile, int pl, int rb, int nrb,
                                              double (&outv)[C::E][C::R]) {
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = tid / WAVE;
    const int j0 = tid * C::E;
    const int seg = 1 << (ps.seg_log2 < 30 ? ps.seg_log2 : 30);
    const int G = seg <= C::E ? 1 : (seg >= C::T ? WG : seg / C::E);
    const int gw = G < WAVE ? G : WAVE;
    const int lig = lane & (gw - 1);
    const double a = A.a;
    constexpr int BOUND = DIR == 0 ? F_SEGSTART : F_SEGEND;
    // first / last processed element of the run
    const int jbeg = DIR == 0 ? j0 : j0 + C::E - 1;
    const int jend = DIR == 0 ? j0 + C::E - 1 : j0;
    const double xbeg = sm.xs[jbeg];
    const double xend = sm.xs[jend];

    State<C> Ex;  // carry entering the run, anchored at xex
    Ex.zero();
    double xex = xbeg;

    if (G > 1) {
        // ---- run aggregate (anchored at xend)
        State<C> F;
        F.zero();
#pragma unroll
        for (int i = 0; i < C::E; ++i) {
            const int e = DIR == 0 ? i : C::E - 1 - i;
            const int j = j0 + e;
            int sc, tc;
            classes<C>(sm.flags[j], hh, sc, tc);
            double geo[C::G > 0 ? C::G : 1];
            load_geo<C>(sm, j, geo);
            ElemVec<C> ev;
            elem_vectors<C>(geo, ev);
            double v[C::R];
            load_v<C>(A, sm.c[j], rb, v);
            if (i > 0) {
                const int js = DIR == 0 ? j : j + 1;  // decay between j and its predecessor
                const double t = a * (DIR == 0 ? sm.xs[j] - sm.xs[j - 1] : sm.xs[j + 1] - sm.xs[j]);
                F.shift(sm.est[js], t);
            }
            add_source<C>(F, sc, ev, v);
        }
        State<C> Frun = F;
        // ---- wave-level inclusive scan toward this direction
#pragma unroll 1
        for (int o = 1; o < gw; o <<= 1) {
            State<C> T2;
            double xp;
            if constexpr (DIR == 0) {
                xp = __shfl_up(xend, o, WAVE);
                shfl_up_state<C>(F, T2, o);
            } else {
                xp = __shfl_down(xend, o, WAVE);
                shfl_down_state<C>(F, T2, o);
            }
            const bool ok = DIR == 0 ? (lig >= o) : (lig + o < gw);
            if (ok) {
                const double t = a * (DIR == 0 ? xend - xp : xp - xend);
                F.add_shifted(T2, exp(-t), t);
            }
        }
        // exclusive value inside the wave group
        {
            double xp;
            if constexpr (DIR == 0) {
                xp = __shfl_up(xend, 1, WAVE);
                shfl_up_state<C>(F, Ex, 1);
            } else {
                xp = __shfl_down(xend, 1, WAVE);
                shfl_down_state<C>(F, Ex, 1);
            }
            const bool has = DIR == 0 ? (lig > 0) : (lig < gw - 1);
            if (has) {
                xex = xp;
            } else {
                Ex.zero();
            }
        }
        // ---- across the waves of a group (128 or 256 threads)
        if (G > WAVE) {
            const int edge = DIR == 0 ? WAVE - 1 : 0;
            if (lane == edge) {
#pragma unroll
                for (int i = 0; i < C::NSLOT; ++i) sm.waveF[wave][i] = F.flat()[i];
                sm.waveFx[wave] = xend;
            }
            __syncthreads();
            const int wpg = G / WAVE;
            const int gfirst = (wave / wpg) * wpg;
            const int glast = gfirst + wpg - 1;
            const bool has_prev_waves = DIR == 0 ? (wave > gfirst) : (wave < glast);
            if (has_prev_waves) {
                State<C> acc, tmp;
                acc.zero();
                const int wstart = DIR == 0 ? gfirst : glast;
                double ax = sm.waveFx[wstart];
                for (int w = wstart; w != wave; w += (DIR == 0 ? 1 : -1)) {
#pragma unroll
                    for (int i = 0; i < C::NSLOT; ++i) tmp.flat()[i] = sm.waveF[w][i];
                    const double t = a * (DIR == 0 ? sm.waveFx[w] - ax : ax - sm.waveFx[w]);
                    acc.shift(exp(-t), t);
                    acc.add_shifted(tmp, 1.0, 0.0);
                    ax = sm.waveFx[w];
                }
                if (lane == (DIR == 0 ? 0 : WAVE - 1)) xex = ax;
                const double t = a * (DIR == 0 ? xex - ax : ax - xex);
                Ex.add_shifted(acc, exp(-t), t);
            }
            __syncthreads();
        }
        if constexpr (MODE == 1) {
            // tile total: inclusive value of the run that ends the tile in this direction
            const int owner = DIR == 0 ? WG - 1 : 0;
            if (tid == owner) {
                State<C> tot = Ex;
                const double t = a * (DIR == 0 ? xend - xex : xex - xend);
                tot.shift(exp(-t), t);
                tot.add_shifted(Frun, 1.0, 0.0);
                double *dst = A.agg + agg_index<C>(A, DIR, pl, tile, rb, nrb, hh);
#pragma unroll
                for (int i = 0; i < C::NSLOT; ++i) dst[i] = tot.flat()[i];
                if (rb == 0 && hh == 0) A.anc[((int64_t)DIR * A.G + pl) * A.ntile + tile] = xend;
            }
            return;
        }
        // ---- carry from the other tiles of the same segment (reduced into LDS)
        if (sm.carhas[DIR]) {
            State<C> cf;
#pragma unroll
            for (int i = 0; i < C::NSLOT; ++i) cf.flat()[i] = sm.car[DIR][i];
            const double anc = sm.carx[DIR];
            if (tid == (DIR == 0 ? 0 : WG - 1)) xex = anc;
            const double t = a * (DIR == 0 ? xex - anc : anc - xex);
            Ex.add_shifted(cf, exp(-t), t);
        }
    }
    if constexpr (MODE == 0) {
        // ---- the scan proper: targets read the state, then sources enter it
        State<C> S = Ex;
        double prevx = xex;
#pragma unroll
        for (int i = 0; i < C::E; ++i) {
            const int e = DIR == 0 ? i : C::E - 1 - i;
            const int j = j0 + e;
            const int fl = sm.flags[j];
            int sc, tc;
            classes<C>(fl, hh, sc, tc);
            const double xj = sm.xs[j];
            if (fl & BOUND) {
                S.zero();
            } else {
                const double t = a * (DIR == 0 ? xj - prevx : prevx - xj);
                const double E = (i == 0) ? exp(-t) : sm.est[DIR == 0 ? j : j + 1];
                S.shift(E, t);
            }
            prevx = xj;
            double geo[C::G > 0 ? C::G : 1];
            load_geo<C>(sm, j, geo);
            ElemVec<C> ev;
            elem_vectors<C>(geo, ev);
            double v[C::R];
            load_v<C>(A, sm.c[j], rb, v);
            read_target<C>(S, tc, ev, outv[e]);
            add_source<C>(S, sc, ev, v);
        }
    }
}

// Sum over the tiles t' of a segment on one side of `tile` of the tile
// aggregates shifted to the anchor next to `tile`; every term is a product of
// bounded factors, so the tiles are combined in parallel (fixed order).
template <class C>
__device__ __forceinline__ void tile_carries(const SweepArgs &A, const PassDev &ps, Smem<C> &sm,
                                             int tile, int pl, int rb, int nrb, int hh) {
    const int seg = 1 << (ps.seg_log2 < 30 ? ps.seg_log2 : 30);
    if (threadIdx.x < 2) sm.carhas[threadIdx.x] = 0;
    if (seg <= C::T || A.ntile < 2) {
        __syncthreads();
        return;
    }
    const int64_t tps = seg / C::T;
    const int64_t ts0 = (tile / tps) * tps;
    const int64_t ts1 = ts0 + tps < A.ntile ? ts0 + tps : A.ntile;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
#pragma unroll 1
    for (int dir = 0; dir < 2; ++dir) {
        const bool has = dir == 0 ? tile > ts0 : tile + 1 < ts1;
        if (!has) continue;  // uniform over the block
        const double *ancd = A.anc + (int64_t)dir * A.G * A.ntile + (int64_t)pl * A.ntile;
        const double xref = dir == 0 ? ancd[tile - 1] : ancd[tile + 1];
        const int64_t lo = dir == 0 ? ts0 : tile + 1;
        const int64_t hi = dir == 0 ? tile : ts1;
        State<C> acc, tmp;
        acc.zero();
        for (int64_t t = lo + threadIdx.x; t < hi; t += WG) {
            const double *src = A.agg + agg_index<C>(A, dir, pl, (int)t, rb, nrb, hh);
#pragma unroll
            for (int i = 0; i < C::NSLOT; ++i) tmp.flat()[i] = src[i];
            const double sh = A.a * (dir == 0 ? xref - ancd[t] : ancd[t] - xref);
            acc.add_shifted(tmp, exp(-sh), sh);
        }
        // block reduction: butterfly inside each wave, then the waves in order
#pragma unroll
        for (int i = 0; i < C::NSLOT; ++i) {
            double v = acc.flat()[i];
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
            if (lane == 0) sm.waveF[wave][i] = v;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < C::NSLOT; i += WG) {
            double v = 0.0;
            for (int w = 0; w < NWAVE; ++w) v += sm.waveF[w][i];
            sm.car[dir][i] = v;
        }
        if (threadIdx.x == 0) {
            sm.carx[dir] = xref;
            sm.carhas[dir] = 1;
        }
        __syncthreads();
    }
    __syncthreads();
}

// MODE 0: one (pass, tile) of the group; the targets' sums go to the pass's slab.
// MODE 1: tile aggregates of the passes whose segments span tiles.
template <class C, int MODE>
__global__ __launch_bounds__(WG) void sweep_kernel(SweepArgs A) {
    __shared__ Smem<C> sm;
    int pass, tile;
    if constexpr (MODE == 0) {
        pass = A.g0 + (int)(blockIdx.x / A.ntile);
        tile = (int)(blockIdx.x % A.ntile);
    } else {
        pass = A.xt[A.k0 + (int)(blockIdx.x / A.ntile)];
        tile = (int)(blockIdx.x % A.ntile);
    }
    const int pl = pass - A.g0;
    const PassDev ps = A.passes[pass];
    const int rb = blockIdx.y;
    const int nrb = gridDim.y;
    const int64_t p0 = (int64_t)tile * C::T;
    stage_tile<C>(A, ps, sm, p0);

    double outv[C::E][C::R];
#pragma unroll
    for (int e = 0; e < C::E; ++e)
#pragma unroll
        for (int r = 0; r < C::R; ++r) outv[e][r] = 0.0;

#pragma unroll 1
    for (int hh = 0; hh < C::NHALF; ++hh) {
        if constexpr (MODE == 0) tile_carries<C>(A, ps, sm, tile, pl, rb, nrb, hh);
        run_direction<C, MODE, 0>(A, ps, sm, hh, tile, pl, rb, nrb, outv);
        run_direction<C, MODE, 1>(A, ps, sm, hh, tile, pl, rb, nrb, outv);
        __syncthreads();
    }

    if constexpr (MODE == 0) {
        const int j0 = threadIdx.x * C::E;
        double *slab = A.ypart + (int64_t)pl * A.n * A.W;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int j = j0 + e;
            if (sm.flags[j] & F_VALID) {
                double *dst = slab + (int64_t)sm.c[j] * A.W + rb * C::R;
#pragma unroll
                for (int r = 0; r < C::R; ++r) dst[r] = outv[e][r];
            }
        }
    }
}

// yacc = [yacc +] sum of the group's slabs, in pass order.
__global__ void accum_kernel(const double *ypart, int G, int64_t len, double *yacc, int first) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = first ? 0.0 : yacc[e];
        for (int g = 0; g < G; ++g) s += ypart[(int64_t)g * len + e];
        yacc[e] = s;
    }
}

__global__ void zero_kernel(double *p, int64_t len) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

// ---------------------------------------------------------------------------
// Host-side dispatch.
// ---------------------------------------------------------------------------
constexpr int E_RUN = 4;
constexpr int TILE = WG * E_RUN;

inline unsigned grid_1d(int64_t n) {
    int64_t g = (n + WG - 1) / WG;
    if (g > 65535 * 8) g = 65535 * 8;
    return (unsigned)(g < 1 ? 1 : g);
}

template <class C>
mm_status run_passes(mm_plan p, const double *vin, double *yacc, int W, hipStream_t s) {
    static_assert(C::T == TILE, "tile size");
    const KParams kp = kparams(p->kernel, p->d);
    const int64_t n = p->n;
    const int nrb = W / C::R;
    const int64_t ntile = (n + C::T - 1) / C::T;
    const int npass = (int)p->passes.size();
    const int64_t len = n * W;
    if (npass == 0) {
        hipLaunchKernelGGL(zero_kernel, dim3(grid_1d(len)), dim3(WG), 0, s, yacc, len);
        MM_HIP_TRY(hipGetLastError());
        return MM_OK;
    }
    const int gmax = group_passes(p, W);
    SweepArgs A{};
    A.xc = static_cast<const double *>(p->xc.ptr);
    A.passes = static_cast<const PassDev *>(p->pass_dev.ptr);
    A.xt = static_cast<const int32_t *>(p->pass_xt.ptr);
    A.vin = vin;
    A.ypart = static_cast<double *>(p->part.ptr);
    A.n = n;
    A.ntile = ntile;
    A.W = W;
    A.a = kp.a;
    const size_t aggslab = (size_t)2 * gmax * ntile * nrb * C::NHALF * C::NSLOT;
    A.agg = static_cast<double *>(p->agg.ptr);
    A.anc = A.agg + aggslab;
    for (int g0 = 0; g0 < npass; g0 += gmax) {
        const int G = npass - g0 < gmax ? npass - g0 : gmax;
        A.g0 = g0;
        A.G = G;
        // passes of the group whose segments span tiles: a contiguous range of xt
        int k0 = 0, k1 = 0;
        while (k0 < (int)p->xt_host.size() && p->xt_host[k0] < g0) ++k0;
        k1 = k0;
        while (k1 < (int)p->xt_host.size() && p->xt_host[k1] < g0 + G) ++k1;
        A.k0 = k0;
        if (k1 > k0 && ntile > 1)
            hipLaunchKernelGGL((sweep_kernel<C, 1>), dim3((unsigned)((k1 - k0) * ntile), (unsigned)nrb),
                               dim3(WG), 0, s, A);
        hipEvent_t ev1 = nullptr;
        if (p->profile) {
            // bracket the main sweep launch with events on its stream
            if (p->prof_used >= 4096) {
                double ms = 0.0;
                int64_t cnt = 0;
                MM_TRY(profile_flush(p, &ms, &cnt));
            }
            if (p->prof_used >= p->prof_events.size()) {
                hipEvent_t e0, e1;
                MM_HIP_TRY(hipEventCreate(&e0));
                MM_HIP_TRY(hipEventCreate(&e1));
                p->prof_events.push_back({e0, e1});
            }
            MM_HIP_TRY(hipEventRecord(p->prof_events[p->prof_used].first, s));
            ev1 = p->prof_events[p->prof_used].second;
            p->prof_used++;
            p->prof_units += (int64_t)G;
        }
        hipLaunchKernelGGL((sweep_kernel<C, 0>), dim3((unsigned)(G * ntile), (unsigned)nrb), dim3(WG), 0, s, A);
        if (ev1) MM_HIP_TRY(hipEventRecord(ev1, s));
        hipLaunchKernelGGL(accum_kernel, dim3(grid_1d(len)), dim3(WG), 0, s,
                           static_cast<const double *>(p->part.ptr), G, len, yacc, g0 == 0 ? 1 : 0);
    }
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

template <int D, int P, bool PROD>
mm_status dispatch_r(mm_plan p, const double *vin, double *yacc, int W, int R, hipStream_t s) {
    // only the blocks that max_r() can select are instantiated
    if constexpr (Cfg<D, P, PROD, 4, E_RUN>::NSLOT <= 16) {
        if (R == 4) return run_passes<Cfg<D, P, PROD, 4, E_RUN>>(p, vin, yacc, W, s);
    }
    if constexpr (Cfg<D, P, PROD, 2, E_RUN>::NSLOT <= 16) {
        if (R == 2) return run_passes<Cfg<D, P, PROD, 2, E_RUN>>(p, vin, yacc, W, s);
    }
    return run_passes<Cfg<D, P, PROD, 1, E_RUN>>(p, vin, yacc, W, s);
}

template <int D, int P, bool PROD>
int max_r() {
    // right-hand sides per thread such that a scan state stays within the register budget
    if (Cfg<D, P, PROD, 4, E_RUN>::NSLOT <= 16) return 4;
    if (Cfg<D, P, PROD, 2, E_RUN>::NSLOT <= 16) return 2;
    return 1;
}

template <int D>
int max_r_d(const KParams &kp) {
    if (kp.P == 1) return max_r<D, 1, true>();
    if constexpr (D == 1) {
        return kp.P == 2 ? max_r<D, 2, true>() : max_r<D, 3, true>();
    } else {
        if (kp.P == 2) return kp.prod ? max_r<D, 2, true>() : max_r<D, 2, false>();
        return kp.prod ? max_r<D, 3, true>() : max_r<D, 3, false>();
    }
}

template <int D>
mm_status dispatch_p(mm_plan p, const KParams &kp, const double *vin, double *yacc, int W, int R,
                     hipStream_t s) {
    if (kp.P == 1) return dispatch_r<D, 1, true>(p, vin, yacc, W, R, s);
    if constexpr (D == 1) {
        if (kp.P == 2) return dispatch_r<D, 2, true>(p, vin, yacc, W, R, s);
        return dispatch_r<D, 3, true>(p, vin, yacc, W, R, s);
    } else {
        if (kp.P == 2)
            return kp.prod ? dispatch_r<D, 2, true>(p, vin, yacc, W, R, s)
                           : dispatch_r<D, 2, false>(p, vin, yacc, W, R, s);
        return kp.prod ? dispatch_r<D, 3, true>(p, vin, yacc, W, R, s)
                       : dispatch_r<D, 3, false>(p, vin, yacc, W, R, s);
    }
}

}  // namespace

int rhs_block(const mm_kernel &k, int d, int nrhs) {
    const KParams kp = kparams(k, d);
    int rmax = d == 1 ? max_r_d<1>(kp) : (d == 2 ? max_r_d<2>(kp) : max_r_d<3>(kp));
    int R = 1;
    while (R * 2 <= rmax && R * 2 <= nrhs) R *= 2;
    return R;
}

// Passes per group: the partial slabs of one group stay within 1 GiB.
constexpr size_t PART_BUDGET = size_t(1) << 30;

static int group_size(int64_t n, int npass, int W) {
    const size_t slab = (size_t)n * W * sizeof(double);
    int64_t g = (int64_t)(PART_BUDGET / (slab > 0 ? slab : 1));
    if (g < 1) g = 1;
    if (g > npass) g = npass;
    return (int)(g < 1 ? 1 : g);
}

int group_passes(mm_plan p, int W) { return group_size(p->n, (int)p->passes.size(), W); }

size_t sweep_part_bytes(int64_t n, int npass, int W) {
    if (npass == 0) return 0;
    return (size_t)group_size(n, npass, W) * n * W * sizeof(double);
}

size_t sweep_agg_bytes(int64_t n, int d, int W, const mm_kernel &k) {
    (void)k;
    // per tile and right-hand side at most NHALF*NCLS*NTH*P <= 108 doubles
    // (d = 3, product form, nu = 5/2), two directions, per pass of a group
    int L = 0;
    while ((int64_t(1) << L) < n) ++L;
    const int npass = n < 2 ? 0 : (d == 1 ? 1 : (d == 2 ? L : L * (L + 1) / 2));
    const int64_t G = npass == 0 ? 1 : group_size(n, npass, W);
    const int64_t ntile = (n + TILE - 1) / TILE;
    const int64_t per_rhs = 128;
    return (size_t)(2 * G * ntile * (int64_t)W * per_rhs + 2 * G * ntile + 16) * sizeof(double);
}

mm_status upload_pass_tables(mm_plan p) {
    std::vector<PassDev> tab;
    p->xt_host.clear();
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const Pass &q = p->passes[i];
        PassDev d{q.ord, q.ord2, q.l1, q.l2, q.seg_log2, 0};
        tab.push_back(d);
        if ((int64_t(1) << (q.seg_log2 < 40 ? q.seg_log2 : 40)) > TILE) p->xt_host.push_back((int)i);
    }
    if (tab.empty()) return MM_OK;
    MM_TRY(dev_alloc(p->pass_dev, tab.size() * sizeof(PassDev)));
    MM_HIP_TRY(hipMemcpy(p->pass_dev.ptr, tab.data(), tab.size() * sizeof(PassDev), hipMemcpyHostToDevice));
    if (!p->xt_host.empty()) {
        MM_TRY(dev_alloc(p->pass_xt, p->xt_host.size() * sizeof(int32_t)));
        MM_HIP_TRY(hipMemcpy(p->pass_xt.ptr, p->xt_host.data(), p->xt_host.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice));
    }
    return MM_OK;
}

mm_status sweep_all(mm_plan p, const double *vin, double *yacc, int W, int R, hipStream_t s) {
    const KParams kp = kparams(p->kernel, p->d);
    if (W % R != 0) {
        set_error("internal: width %d is not a multiple of the block %d", W, R);
        return MM_ERR_ARG;
    }
    switch (p->d) {
        case 1: return dispatch_p<1>(p, kp, vin, yacc, W, R, s);
        case 2: return dispatch_p<2>(p, kp, vin, yacc, W, R, s);
        default: return dispatch_p<3>(p, kp, vin, yacc, W, R, s);
    }
}

}  // namespace mm
