#pragma once
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
//
// Lengthscale derivative.  With t = a r and a = sqrt(2 nu)/l,
//     l d/dl k(a r) = -t k'(t) = sum_m e_m t^m / m! exp(-t),
//     e_m = m (c_{m-1} - c_m)  (c_{-1} = c_P = 0, m = 0..P),
// i.e. e = [0, 1], [0, 0, 2], [0, 0, 2/3, 2]: one more channel in the same
// basis (the gradients of the Section 2.3 examples).  The L1 form's
// derivative is that profile of the summed offset; the product form's is
// the sum over coordinates j of the product with factor j differentiated,
// one sweep per j.

#include "mm_internal.h"

#include <cstdlib>

namespace mm {
namespace {

constexpr int WG = 256;
constexpr int WAVE = 64;
constexpr int NWAVE = WG / WAVE;

template <int B, int E>
struct IPow { static constexpr int v = B * IPow<B, E - 1>::v; };
template <int B>
struct IPow<B, 0> { static constexpr int v = 1; };

// c_m coefficients of the profile in the scaled-power basis; with DER the
// coefficients e_m of l dk/dl (P + 1 of them).
template <int P, bool DER = false>
__device__ __forceinline__ double coef(int m) {
    if constexpr (DER) {
        if constexpr (P == 1) return m == 1 ? 1.0 : 0.0;
        if constexpr (P == 2) return m == 2 ? 2.0 : 0.0;
        return m == 3 ? 2.0 : (m == 2 ? 2.0 / 3.0 : 0.0);
    }
    if constexpr (P == 3) return m == 2 ? (2.0 / 3.0) : 1.0;
    return 1.0;
}

// Source factor s_m(E, t) = E t^m / m!  (t = a w, E = exp(-t)).
template <int P>
__device__ __forceinline__ void src_vec(double E, double t, double (&sv)[P]) {
    sv[0] = E;
    if constexpr (P > 1) sv[1] = E * t;
    if constexpr (P > 2) sv[2] = E * t * t * 0.5;
    if constexpr (P > 3) sv[3] = sv[2] * t * (1.0 / 3.0);
}

// s <- M(E, t) s: s_m <- E sum_{q<=m} t^(m-q)/(m-q)! s_q (in place, top down).
template <int N>
__device__ __forceinline__ void mshift(double (&s)[N], double E, double t) {
    const double t2 = 0.5 * t * t;
    if constexpr (N == 4) s[3] = E * fma(t2 * t * (1.0 / 3.0), s[0], fma(t2, s[1], fma(t, s[2], s[3])));
    if constexpr (N >= 3) s[2] = E * fma(t2, s[0], fma(t, s[1], s[2]));
    if constexpr (N >= 2) s[1] = E * fma(t, s[0], s[1]);
    s[0] = E * s[0];
}

// acc <- acc + M(E, t) q.
template <int N>
__device__ __forceinline__ void madd(double (&acc)[N], const double (&q)[N], double E, double t) {
    const double t2 = 0.5 * t * t;
    if constexpr (N == 4) acc[3] = fma(E, fma(t2 * t * (1.0 / 3.0), q[0], fma(t2, q[1], fma(t, q[2], q[3]))), acc[3]);
    if constexpr (N >= 3) acc[2] = fma(E, fma(t2, q[0], fma(t, q[1], q[2])), acc[2]);
    if constexpr (N >= 2) acc[1] = fma(E, fma(t, q[0], q[1]), acc[1]);
    acc[0] = fma(E, q[0], acc[0]);
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
        gv[0] = E * fma(t * (1.0 / 3.0), t, 1.0 + t);
        gv[1] = E * fma(t, 2.0 / 3.0, 1.0);
        gv[2] = E * (2.0 / 3.0);
    }
}

// The same for the derivative profile e (P + 1 channels):
// g_q = E sum_{m>=q} e_m t^(m-q)/(m-q)!.
template <int P>
__device__ __forceinline__ void tgt_vec_der(double E, double t, double (&gv)[P + 1]) {
    if constexpr (P == 1) {
        gv[0] = E * t;
        gv[1] = E;
    } else if constexpr (P == 2) {
        gv[0] = E * t * t;
        gv[1] = 2.0 * E * t;
        gv[2] = 2.0 * E;
    } else {
        gv[0] = E * t * t * (1.0 + t) * (1.0 / 3.0);
        gv[1] = E * t * (2.0 / 3.0 + t);
        gv[2] = E * fma(2.0, t, 2.0 / 3.0);
        gv[3] = 2.0 * E;
    }
}

// Source and target vectors of one coordinate's factor: the kernel profile
// (N = P channels) or, for the differentiated coordinate, its derivative
// profile (N = P + 1).
template <int P, int N>
__device__ __forceinline__ void factor_vecs(double E, double t, double (&sv)[N], double (&gv)[N]) {
    src_vec<N>(E, t, sv);
    if constexpr (N == P) tgt_vec<P>(E, t, gv);
    else tgt_vec_der<P>(E, t, gv);
}

// Flags stored with each staged element.
constexpr int F_SIDE1 = 1;     // x1 half (d >= 2)
constexpr int F_SIDE2 = 2;     // x2 half (d = 3)
constexpr int F_VALID = 16;    // position < n

// Accesses through the global address space.  The kernels read their pointers
// from descriptors in memory, so the compiler cannot tell they are global and
// would issue flat accesses, which also count against the LDS wait counter:
// every wait for a staged LDS value would then wait for the gathers in flight.
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

// One divide-and-conquer pass as the kernels see it (device table).
struct PassDev {
    const uint32_t *cf;   // canonical index | x1 half << 30 | x2 half << 31, in pass order
    const double *xs;     // scan coordinate in pass order
    const double *w1;     // x1 offset from the node's split point
    const double *w2;     // d = 3: x2 offset from the x2 node's split point
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
    double *agg;           // tile aggregates [2 dirs][G][ntile][W][NSUB][NSLOT]
    double *car;           // tile carries, same layout as agg
    double *anc;           // tile anchors [2 dirs][G][ntile]
    double *dec;           // decay from the previous tile's anchor (scan order) to the tile's, same layout
    int64_t n;
    int64_t ntile;
    int W;                 // leading width of vin / ypart (columns)
    int g0;                // first pass of the group
    int k0;                // first entry of xt inside the group
    int G;                 // passes in the group
    int nslice;            // carry-scan slices (sub-sweep x class x row x column)
    const int4 *segs;      // the plan's cross-tile segments (pass, first tile, end tile)
    const int32_t *xtpos;  // each pass's position in xt (-1: its segments fit in a tile)
    double *runex;         // the runs' within-tile carries of the cross-tile passes (Cfg::RUNEX; null
                           //   in d = 3, whose workspace has no room for them, or when the schedule
                           //   declines them):
                           //   [2 dirs][xt pass of the group][ntile][column block][NSUB][NSLOT][lane]
    double a;
};

// Static configuration of a sweep instance.  A workgroup is one wave.  Its 64
// lanes are WCOL right-hand-side columns times RUNS runs: lane (run, col)
// scans the E consecutive positions run*E .. run*E+E-1 of a tile of
// T = RUNS*E positions for one column.  The runs of a column are joined by a
// lane scan of log2(RUNS) steps; tiles of a segment are joined through the
// tile aggregates and the tile carry scan.  The tile's geometry is staged once
// in LDS and read by every column (broadcast).
// GJ selects the lengthscale-derivative sweep: -1 the kernel itself; j in
// 0..D-2 the product with the factor of non-scan coordinate j differentiated;
// D-1 the scan coordinate's factor differentiated (for the L1 form: the
// derivative of its single profile).  PK is the kernel's channel count
// (nu + 1/2); P, the scan state's, is PK + 1 when the scan coordinate
// carries the derivative.
template <int D_, int P_, bool PROD_, int WCOL_, int E_, int GJ_ = -1>
struct Cfg {
    static constexpr int D = D_;
    static constexpr int PK = P_;
    static constexpr int GJ = GJ_;
    static constexpr bool DSCAN = GJ_ == D_ - 1;
    static constexpr int P = DSCAN ? P_ + 1 : P_;
    static_assert(GJ_ >= -1 && GJ_ < D_, "derivative coordinate");
    static_assert(PROD_ || GJ_ == -1 || GJ_ == D_ - 1, "the L1 derivative is the scan profile's");
    static constexpr bool PROD = PROD_;
    static constexpr int WCOL = WCOL_;
    static constexpr int RUNS = WAVE / WCOL;
    static constexpr int E = E_;
    static constexpr int T = RUNS * E;                       // tile positions
    // channels of non-scan coordinate k's factor
    static constexpr int PC0 = GJ_ == 0 && D_ > 1 ? P_ + 1 : P_;
    static constexpr int PC1 = GJ_ == 1 && D_ > 2 ? P_ + 1 : P_;
    static constexpr int NTH = PROD ? (D == 1 ? 1 : (D == 2 ? PC0 : PC0 * PC1)) : 1; // non-scan channel rows
    // source classes and how many sub-sweeps they are split over so that one
    // state fits the register file (each sub-sweep repeats the scan for its
    // classes).  Two classes in d >= 2, told apart by the x1 half: in d = 3
    // every segment of a pass lists its two orthant groups (x1 half xor x2
    // half) one after the other, the state restarting between them, and
    // inside a group the x1 half fixes the x2 half.
    static constexpr int NCLS_ALL = (D == 1) ? 1 : 2;
    static constexpr int FULLSLOT = NCLS_ALL * NTH * P;
    static constexpr int NSUB = (D == 3 && FULLSLOT > 32) ? 2 : 1;
    // The sub-sweeps run side by side, one wave each, in one workgroup that
    // stages the tile once: the staged tile's LDS is shared by the waves, and
    // every element is a target of exactly one sub-sweep (the one carrying the
    // other class), so each wave writes only its own targets' sums.
    static constexpr int NWAVE = NSUB;
    static constexpr int BLOCK = WAVE * NWAVE;
    // at least 2 waves per SIMD for the two-wave workgroups (without the bound
    // the compiler takes AGPRs as spill room and drops to one wave)
    static constexpr int MINW = NWAVE > 1 ? 2 : 1;
    static constexpr int NCLS = NCLS_ALL / NSUB;
    static constexpr int NSLOT = NCLS * NTH * P;             // doubles per state
    static constexpr int G = 2 * (D - 1);                    // staged geometry doubles
    // keep the targets' sums in registers over the sweep (runs of 4, small states)
    static constexpr bool REGOUT = E <= 4 && E * NSLOT <= 64;
    // otherwise the targets' sums of the two directions (and sub-sweeps)
    // gather per lane and reach the pass's slab once: in registers for d <= 2
    // and runs of at most 32 (a ring, see run_direction), in LDS for d = 3
    // (larger states) while the tile's sums take at most 16 KB; beyond both,
    // each direction updates the slab in place
    static constexpr bool OUTREG = !REGOUT && D <= 2 && E <= 32;
    static constexpr bool LDSOUT = !REGOUT && !OUTREG && T * WCOL <= 2048;
    static constexpr bool SUMREG = REGOUT || OUTREG;   // outv holds the run's sums
    // the tile-aggregate pre-pass stores every run's within-tile carry of the
    // cross-tile passes, so the main launch skips their aggregate pass and lane scan
    static constexpr bool RUNEX = OUTREG && WCOL >= 2;
    // elements per block of a run's loads.  Short runs take two blocks: with
    // one, the block loop disappears, every load of the run is hoisted and
    // the state spills (d = 3).  Long runs take blocks of 4 in d <= 2 (8 lifts
    // the d = 2 kernels past 128 registers) and of 8 in d = 3.
    static constexpr int BLK = E <= 8 ? E / 2 : (D <= 2 ? 4 : 8);
    // blocks per iteration of the main scan's block loop when the run's sums
    // stay in registers: unrolling lets consecutive turns of the sums' ring
    // (see run_direction) become renames instead of moves.  Runs of 32 in
    // waves of 8 or more columns take 4 (two iterations: a fully unrolled run
    // hoists every gather and spills); runs of 16 in d = 2 waves of 4 columns
    // take 2; elsewhere the unrolled loop needs more registers than it saves
    // moves.
    static constexpr int OUTU = (OUTREG && E == 32 && WCOL >= 8 && E / BLK >= 8) ? 4
                                : (OUTREG && D == 2 && E == 16 && WCOL == 4 && E / BLK >= 4) ? 2 : 1;
};

template <class C>
struct State {
    double s[C::NCLS][C::NTH][C::P];

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
            for (int h = 0; h < C::NTH; ++h)
#pragma unroll
                for (int m = 0; m < C::P; ++m) s[c][h][m] = 0.0;
    }

    // this <- M(E, t) this
    __device__ __forceinline__ void shift(double E, double t) {
#pragma unroll
        for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
            for (int h = 0; h < C::NTH; ++h) mshift(s[c][h], E, t);
    }

    // this <- this + M(E, t) o
    __device__ __forceinline__ void add_shifted(const State &o, double E, double t) {
#pragma unroll
        for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
            for (int h = 0; h < C::NTH; ++h) madd(s[c][h], o.s[c][h], E, t);
    }

    __device__ __forceinline__ double *flat() { return &s[0][0][0]; }
    __device__ __forceinline__ const double *flat() const { return &s[0][0][0]; }
};

// Geometry of one element (source and target vectors) derived from its staged offsets.
//   product form: f[th] = prod_k s_{th_k}(w_k) (source, enters the m = 0 slot),
//                 g[th] = prod_k g_{th_k}(w_k) (target, times the profile coefficients c_m);
//   L1 form:      f[m] = s_m(W), g[m] = g_m(W) with W the summed offset.
template <class C>
struct ElemVec {
    double f[C::PROD ? C::NTH : C::P];
    double g[C::PROD ? C::NTH : C::P];
};

template <class C>
__device__ __forceinline__ void elem_vectors(const double *geo, ElemVec<C> &ev) {
    if constexpr (C::D == 1) {  // no other coordinate: unit source and target
        static_assert(C::D != 1 || C::PROD, "d = 1 uses the product path");
        ev.f[0] = 1.0;
        ev.g[0] = 1.0;
        return;
    } else if constexpr (C::PROD) {
        // row th holds channel (th mod PC0) of the first coordinate and
        // (th div PC0) of the second
        double sv0[C::PC0], gv0[C::PC0];
        factor_vecs<C::PK>(geo[0], geo[1], sv0, gv0);
        if constexpr (C::D == 2) {
#pragma unroll
            for (int th = 0; th < C::NTH; ++th) {
                ev.f[th] = 1.0 * sv0[th];
                ev.g[th] = 1.0 * gv0[th];
            }
        } else {
            double sv1[C::PC1], gv1[C::PC1];
            factor_vecs<C::PK>(geo[2], geo[3], sv1, gv1);
#pragma unroll
            for (int th = 0; th < C::NTH; ++th) {
                ev.f[th] = 1.0 * sv0[th % C::PC0] * sv1[th / C::PC0];
                ev.g[th] = 1.0 * gv0[th % C::PC0] * gv1[th / C::PC0];
            }
        }
    } else {
        // L1: offsets add up; exp of the sum is the product of the exps.
        double E = 1.0, t = 0.0;
#pragma unroll
        for (int k = 0; k < C::D - 1; ++k) {
            E *= geo[2 * k];
            t += geo[2 * k + 1];
        }
        factor_vecs<C::PK>(E, t, ev.f, ev.g);
    }
}

// S[c] += vc * source vector.
template <class C>
__device__ __forceinline__ void add_class(State<C> &S, int c, const ElemVec<C> &ev, double vc) {
#pragma unroll
    for (int h = 0; h < C::NTH; ++h) {
        if constexpr (C::PROD) {
            S.s[c][h][0] = fma(ev.f[h], vc, S.s[c][h][0]);
        } else {
#pragma unroll
            for (int m = 0; m < C::P; ++m) S.s[c][h][m] = fma(ev.f[m], vc, S.s[c][h][m]);
        }
    }
}

// S[cls] += v * source vector.  The class is selected through the value
// (v or 0) rather than a branch so the state stays in registers.
template <class C>
__device__ __forceinline__ void add_source(State<C> &S, int cls, const ElemVec<C> &ev, double v) {
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c) add_class<C>(S, c, ev, (c == cls) ? v : 0.0);
}

// S[c] += M(E, t) (vc * source vector): a source entered at distance t
// (decay E) from the state's anchor, in one step.  pw[m] = t^m / m!.
template <class C>
__device__ __forceinline__ void add_class_moved(State<C> &S, int c, const ElemVec<C> &ev, double vc, double E,
                                                double t, const double (&pw)[C::P]) {
    if constexpr (C::PROD) {
        const double w = vc * E;
#pragma unroll
        for (int h = 0; h < C::NTH; ++h) {
            const double g = ev.f[h] * w;
            S.s[c][h][0] += g;
#pragma unroll
            for (int m = 1; m < C::P; ++m) S.s[c][h][m] = fma(g, pw[m], S.s[c][h][m]);
        }
    } else {
        double q[C::P];
#pragma unroll
        for (int m = 0; m < C::P; ++m) q[m] = ev.f[m] * vc;
        madd(S.s[c][0], q, E, t);
    }
}

// target vector . S[c]
template <class C>
__device__ __forceinline__ double target_dot(const State<C> &S, int c, const ElemVec<C> &ev) {
    double acc = -0.0;  // -0 is the exact additive identity: the first term needs no addition
#pragma unroll
    for (int h = 0; h < C::NTH; ++h) {
        if constexpr (C::PROD) {
            // the kernel profile has c_0 = 1, the derivative profile e_0 = 0
            double row = C::DSCAN ? 0.0 : S.s[c][h][0];
#pragma unroll
            for (int m = 1; m < C::P; ++m) row = fma(coef<C::PK, C::DSCAN>(m), S.s[c][h][m], row);
            acc = fma(ev.g[h], row, acc);
        } else {
#pragma unroll
            for (int m = 0; m < C::P; ++m) acc = fma(ev.g[m], S.s[c][h][m], acc);
        }
    }
    return acc;
}

// target vector . S[cls] (0 for no class)
template <class C>
__device__ __forceinline__ double read_target(const State<C> &S, int cls, const ElemVec<C> &ev) {
    double out = 0.0;
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c) {
        const double acc = target_dot<C>(S, c, ev);
        out = (c == cls) ? acc : out;
    }
    return out;
}

// Source / target class of an element in sub-sweep `hh`.  d = 2: the x1 half
// (sources of one half feed targets of the other).  d = 3: the same within
// an orthant group (the x2 half is the x1 half xor the group), so a source
// class feeds the targets in the opposite halves of both coordinates.  With
// NSUB = 2 each sub-sweep carries one class.
template <class C>
__device__ __forceinline__ void classes(int flags, int hh, int &scls, int &tcls) {
    if constexpr (C::D == 1) {
        scls = 0;
        tcls = 0;
    } else {
        const int s1 = flags & F_SIDE1;
        if constexpr (C::NSUB == 1) {
            scls = s1;
            tcls = 1 - s1;
        } else {
            scls = (s1 == hh) ? 0 : -1;
            tcls = (1 - s1 == hh) ? 0 : -1;
        }
    }
    if (!(flags & F_VALID)) {
        scls = -1;
        tcls = -1;
    }
}

// Whether a staged element (its flags) is a target of sub-sweep hh.
template <class C>
__device__ __forceinline__ bool is_target(int flags, int hh) {
    int sc, tc;
    classes<C>(flags, hh, sc, tc);
    return tc >= 0;
}

// Staged tile in LDS, stored [element of the run][run]: lanes of different
// runs read different banks, lanes of the same run (different columns) read
// the same address (broadcast).  Local position j lives at slot(j).
template <class C>
struct Smem {
    int32_t c[C::T];
    int32_t flags[C::T];
    // decay exp(-t) and scaled distance t = a (x_j - x_{j-1}) from the previous
    // position; both 0 at segment starts (the state restarts there) and past the
    // end; [T]: into the next tile's first position
    double est[C::T + 1];
    double st[C::T + 1];
    double xrun[2][C::RUNS];  // scan coordinate of each run's first and last position
    double xedge[2];          // scan coordinate before the tile (p0 - 1) and after it (p0 + T)
    double geo[C::G > 0 ? C::G : 1][C::T];
};

// Targets' sums of the main launch gathered in LDS ([slot][column of the wave]).
template <class C>
struct Lout {
    double v[C::LDSOUT ? C::T * C::WCOL : 1];
};

template <class C>
__device__ __forceinline__ int slot(int j) {
    return (j % C::E) * C::RUNS + j / C::E;
}

// Scan coordinate of pass position p (0 <= p < n).
template <class C>
__device__ __forceinline__ double scan_coord(const SweepArgs &A, const PassDev &ps, int64_t p) {
    if constexpr (C::D == 1) return gld(A.xc + p);
    else return gld(ps.xs + p);
}

// Stage the tile's positions: indices, flags, scan coordinate, offsets and
// the decay between consecutive positions.
template <class C>
__device__ __forceinline__ void stage_tile(const SweepArgs &A, const PassDev &ps, Smem<C> &sm,
                                           int64_t p0) {
    const int64_t n = A.n;
    const int64_t segmask = (int64_t(1) << ps.seg_log2) - 1;
    for (int j = threadIdx.x; j <= C::T; j += C::BLOCK) {
        const int64_t p = p0 + j;
        const int64_t pc = p < n ? p : n - 1;
        const double xcur = scan_coord<C>(A, ps, pc);
        if (j < C::T) {
            int flags = p < n ? F_VALID : 0;
            const int sj = slot<C>(j);
            int64_t c;
            if constexpr (C::D == 1) {
                c = pc;
            } else {
                // sequential reads of the pass's stored geometry
                const uint32_t cf = gld(ps.cf + pc);
                c = (int64_t)(cf & 0x3fffffffu);
                flags |= (cf >> 30) & 1u ? F_SIDE1 : 0;
                // past the end: zero geometry, i.e. zero source and target vectors
                const bool in = p < n;
                const double t1 = A.a * gld(ps.w1 + pc);
                sm.geo[0][sj] = in ? exp(-t1) : 0.0;
                sm.geo[1][sj] = in ? t1 : 0.0;
                if constexpr (C::D == 3) {
                    flags |= (cf >> 31) ? F_SIDE2 : 0;
                    const double t2 = A.a * gld(ps.w2 + pc);
                    sm.geo[2][sj] = in ? exp(-t2) : 0.0;
                    sm.geo[3][sj] = in ? t2 : 0.0;
                }
            }
            sm.c[sj] = (int32_t)c;
            sm.flags[sj] = flags;
            const int e = j % C::E;
            if (e == 0) sm.xrun[0][j / C::E] = xcur;
            if (e == C::E - 1) sm.xrun[1][j / C::E] = xcur;
        }
        // from the predecessor, including across the tile's edges (position p0
        // from p0 - 1, and the next tile's first position p0 + T from the last)
        bool has_prev = p < n && p > 0 && (p & segmask) != 0;
        if constexpr (C::D == 3) {
            // the state also restarts where a segment's second orthant group begins
            if (has_prev) {
                const uint32_t c0 = gld(ps.cf + p), c1 = gld(ps.cf + p - 1);
                has_prev = (((c0 ^ (c0 >> 1)) ^ (c1 ^ (c1 >> 1))) & (1u << 30)) == 0;
            }
        }
        double e = 0.0, t = 0.0, xprev = xcur;
        if (has_prev) {
            xprev = scan_coord<C>(A, ps, p - 1);
            t = A.a * (xcur - xprev);
            e = exp(-t);
        }
        if (j == 0) sm.xedge[0] = xprev;
        if (j == C::T) sm.xedge[1] = has_prev ? xcur : scan_coord<C>(A, ps, p0 + C::T - 1 < n ? p0 + C::T - 1 : n - 1);
        sm.est[j < C::T ? slot<C>(j) : C::T] = e;
        sm.st[j < C::T ? slot<C>(j) : C::T] = t;
    }
    __syncthreads();
}

template <class C>
__device__ __forceinline__ void load_geo(const Smem<C> &sm, int sj, double (&geo)[C::G > 0 ? C::G : 1]) {
#pragma unroll
    for (int k = 0; k < C::G; ++k) geo[k] = sm.geo[k][sj];
}

// Restarts of the scan state inside a tile, for the transfers that join runs
// and tiles (d = 3, where a segment's second orthant group begins mid-segment;
// in d <= 2 restarts fall only on segment boundaries, which the run groups and
// tile carries respect by construction).  A staged decay of exactly 0 marks a
// position whose state does not come from its predecessor.  For this lane's
// run r: f, a restart at one of its positions (the forward transfer from the
// previous run's last position to r's last crosses them); b, a restart after
// its first position up to the next run's first (the backward transfer from
// the next run's first position to r's first).  mf / mb: the same over the
// wave, one bit per lane (the run's WCOL lanes carry its flags).
struct Cuts {
    bool f = false, b = false;
    uint64_t mf = 0, mb = 0;
};

template <class C>
__device__ __forceinline__ Cuts tile_cuts(const Smem<C> &sm, int run) {
    Cuts c;
    if constexpr (C::D == 3) {
        bool f = false, b = false;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const bool z = sm.est[e * C::RUNS + run] == 0.0;
            f = f || z;
            if (e > 0) b = b || z;
        }
        b = b || (run + 1 < C::RUNS ? sm.est[run + 1] : sm.est[C::T]) == 0.0;
        c.f = f;
        c.b = b;
        c.mf = __ballot(f);
        c.mb = __ballot(b);
    }
    return c;
}

// Whether a restart lies between the previous tile's anchor and this run's
// entry anchor in scan direction DIR (lanes of the runs before r forward,
// after r backward).
template <class C, int DIR>
__device__ __forceinline__ bool cut_before_run(const Cuts &c, int run) {
    if constexpr (C::D != 3) {
        return false;
    } else if constexpr (DIR == 0) {
        const int lo = run * C::WCOL;
        return (c.mf & (lo >= 64 ? ~0ull : ((1ull << lo) - 1))) != 0;
    } else {
        const int hi = (run + 1) * C::WCOL;
        return (c.mb & (hi >= 64 ? 0ull : ~((1ull << hi) - 1))) != 0;
    }
}

// First element of a wave's stored within-tile run carries (element k of lane
// l at + k * WAVE + l).
template <class C>
__device__ __forceinline__ int64_t runex_index(const SweepArgs &A, int dir, int kx, int64_t tile, int cb, int hh) {
    const int ncb = A.W / C::WCOL;
    return (((((int64_t)dir * A.G + kx) * A.ntile + tile) * ncb + cb) * C::NSUB + hh) * (int64_t)C::NSLOT * WAVE;
}

template <class C>
__device__ __forceinline__ int64_t agg_index(const SweepArgs &A, int dir, int pl, int64_t tile, int col,
                                             int hh) {
    return (((((int64_t)dir * A.G + pl) * A.ntile + tile) * A.W + col) * C::NSUB + hh) * C::NSLOT;
}

// One step of the lane scan over runs: F <- F + M(E, t) F(partner), the
// partner o runs away in the scan direction (the same column's lane o*WCOL
// lanes up or down).  (t, E) is the transfer from the partner's anchor to this
// lane's anchor -- the distance, times a, spanned by the runs this lane
// already covers, and its decay -- so no exponential is evaluated here; the
// coverage then grows by the partner's.
template <class C, bool UP>
__device__ __forceinline__ void scan_step(State<C> &F, double &t, double &E, int o, bool ok) {
    const int dl = o * C::WCOL;
    const double tp = UP ? __shfl_up(t, dl, WAVE) : __shfl_down(t, dl, WAVE);
    const double Ep = UP ? __shfl_up(E, dl, WAVE) : __shfl_down(E, dl, WAVE);
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
        for (int h = 0; h < C::NTH; ++h) {
            double q[C::P];
#pragma unroll
            for (int m = 0; m < C::P; ++m)
                q[m] = UP ? __shfl_up(F.s[c][h][m], dl, WAVE) : __shfl_down(F.s[c][h][m], dl, WAVE);
            if (ok) madd(F.s[c][h], q, E, t);
        }
    if (ok) {
        t += tp;
        E *= Ep;
    }
}

// The lane scan's moves inside rows of 16 lanes go through DPP instead of LDS
// permutes.  CTRL is a DPP row shift (0x110 + n: from lane l - n, 0x100 + n:
// from lane l + n, within the row) or a wave shift by one lane (0x138: from
// lane l - 1, 0x130: from lane l + 1); lanes without a source read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// F <- F + M(E, t) F(partner) with the partner N lanes away inside the row
// (as scan_step).
template <class C, bool UP, int N>
__device__ __forceinline__ void scan_step_row(State<C> &F, double &t, double &E, bool ok) {
    constexpr int CTRL = UP ? 0x110 + N : 0x100 + N;
    const double tp = dpp_move<CTRL>(t);
    const double Ep = dpp_move<CTRL>(E);
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
        for (int h = 0; h < C::NTH; ++h) {
            double q[C::P];
#pragma unroll
            for (int m = 0; m < C::P; ++m) q[m] = dpp_move<CTRL>(F.s[c][h][m]);
            if (ok) madd(F.s[c][h], q, E, t);
        }
    if (ok) {
        t += tp;
        E *= Ep;
    }
}

// F <- F + M(E, t) F(src) for a partner lane given by number (crossing rows).
template <class C>
__device__ __forceinline__ void scan_step_lane(State<C> &F, double &t, double &E, int src, bool ok) {
    const double tp = __shfl(t, src, WAVE);
    const double Ep = __shfl(E, src, WAVE);
#pragma unroll
    for (int c = 0; c < C::NCLS; ++c)
#pragma unroll
        for (int h = 0; h < C::NTH; ++h) {
            double q[C::P];
#pragma unroll
            for (int m = 0; m < C::P; ++m) q[m] = __shfl(F.s[c][h][m], src, WAVE);
            if (ok) madd(F.s[c][h], q, E, t);
        }
    if (ok) {
        t += tp;
        E *= Ep;
    }
}

// One within-row step of the lane scan over runs O apart (O WCOL lanes).
template <class C, int DIR, int O>
__device__ __forceinline__ void row_step(State<C> &F, double &t, double &E, int lig, int Gr, int rr) {
    constexpr int RR = 16 / C::WCOL;  // runs per row
    if constexpr (O < RR) {
        if (O < Gr) {
            const bool ok = DIR == 0 ? (rr >= O && lig >= O) : (rr + O < RR && lig + O < Gr);
            scan_step_row<C, DIR == 0, O * C::WCOL>(F, t, E, ok);
        }
    }
}

// Inclusive transfer-carrying scan of the run aggregates over the runs of
// each segment group (Gr runs, a power of two; lig = the run's index in its
// group), forward (DIR 0: over the runs before) or backward (over the runs
// after); a run's lanes are its WCOL columns.  Up to 8 columns per wave:
// Hillis-Steele inside each row of 16 lanes by DPP, then the rows joined --
// for groups spanning two rows each odd row (forward; even, backward) takes
// the total of its neighbour row's last (first) run, and for groups spanning
// four rows the second half (first half) takes the total of the other half.
// Wider waves (a run per row or more): Hillis-Steele over permutes.  Either
// way each run ends with the sum over its group's runs up to it, moved to its
// anchor.
template <class C, int DIR>
__device__ __forceinline__ void lane_scan(State<C> &F, double &t, double &E, int lig, int Gr, int lane) {
    if constexpr (C::WCOL <= 8) {
        constexpr int RR = 16 / C::WCOL;
        const int rr = (lane & 15) / C::WCOL, row = lane >> 4, cc = lane % C::WCOL;
        row_step<C, DIR, 1>(F, t, E, lig, Gr, rr);
        row_step<C, DIR, 2>(F, t, E, lig, Gr, rr);
        row_step<C, DIR, 4>(F, t, E, lig, Gr, rr);
        row_step<C, DIR, 8>(F, t, E, lig, Gr, rr);
        constexpr bool UP = DIR == 0;
        if (Gr > RR) {
            // rows in pairs: forward, an odd row takes the last run of the row before;
            // backward, an even row takes the first run of the row after
            const bool ok = UP ? (row & 1) == 1 : (row & 1) == 0;
            scan_step_lane<C>(F, t, E, UP ? 16 * row - C::WCOL + cc : 16 * row + 16 + cc, ok);
        }
        if (Gr > 2 * RR) {
            // halves: forward, rows 2-3 take the last run of row 1; backward, rows
            // 0-1 take the first run of row 2
            const bool ok = UP ? row >= 2 : row < 2;
            scan_step_lane<C>(F, t, E, UP ? 32 - C::WCOL + cc : 32 + cc, ok);
        }
    } else {
#pragma unroll 1
        for (int o = 1; o < Gr; o <<= 1) {
            const bool ok = DIR == 0 ? (lig >= o) : (lig + o < Gr);
            scan_step<C, DIR == 0>(F, t, E, o, ok);
        }
    }
}

// The previous run's value in the scan direction (the same column's lane
// WCOL lanes down for DIR 0, up for DIR 1).
template <class C, int DIR>
__device__ __forceinline__ double run_neighbour(double v) {
    if constexpr (C::WCOL == 1) return dpp_move<DIR == 0 ? 0x138 : 0x130>(v);
    else return DIR == 0 ? __shfl_up(v, C::WCOL, WAVE) : __shfl_down(v, C::WCOL, WAVE);
}

// Process element e of the lane's run in a scan step: move the state to the
// element (or reset at a segment boundary), read the target value, add the
// source.  Returns the target value.
template <class C, int DIR, bool TARGET>
__device__ __forceinline__ double scan_elem(const Smem<C> &sm, State<C> &S, int e, int i, int run, int hh,
                                            double v) {
    const int sj = e * C::RUNS + run;
    const int fl = sm.flags[sj];
    // move the state from the previous position in the scan direction (the
    // anchor of any carry) with the staged decay and distance; both are 0 at a
    // segment start (forward) or past a segment end (backward), which restarts
    // the state
    int ej;
    if constexpr (DIR == 0) {
        ej = sj;
    } else {
        ej = (e + 1 < C::E) ? sj + C::RUNS : (run + 1 < C::RUNS ? run + 1 : C::T);
    }
    S.shift(sm.est[ej], sm.st[ej]);
    double geo[C::G > 0 ? C::G : 1];
    load_geo<C>(sm, sj, geo);
    ElemVec<C> ev;
    elem_vectors<C>(geo, ev);
    double out = 0.0;
    if constexpr (C::D >= 2 && C::NCLS == 2) {
        // two classes, told apart by the x1 half alone: sources of half s
        // feed the targets of half 1 - s.  A position past the end has zero
        // staged geometry (a zero source vector), so it needs no class test.
        const bool s1 = fl & F_SIDE1;
        if constexpr (TARGET) {
            const double t0 = target_dot<C>(S, 0, ev), t1 = target_dot<C>(S, 1, ev);
            out = s1 ? t0 : t1;
        }
        add_class<C>(S, 0, ev, s1 ? 0.0 : v);
        add_class<C>(S, 1, ev, s1 ? v : 0.0);
    } else {
        int sc, tc;
        classes<C>(fl, hh, sc, tc);
        if constexpr (TARGET) out = read_target<C>(S, tc, ev);
        add_source<C>(S, sc, ev, v);
    }
    return out;
}

// Both run aggregates of this lane's run in one walk over it (increasing
// positions): Ff, anchored at the run's last position, by the state
// recurrence of the forward direction; Fb, anchored at its first position,
// adds each source moved by its distance and decay from that position, which
// accumulate along the walk.  Only for runs inside one segment (segments
// longer than a tile); a restart inside the run (d = 3, between orthant
// groups) stages a zero decay, which zeroes the later sources' weights in Fb
// (they do not reach the run's first position) and the earlier state in Ff.
template <class C>
__device__ __forceinline__ void run_aggregates(const SweepArgs &A, const Smem<C> &sm, int run, int col, int hh,
                                               State<C> &Ff, State<C> &Fb) {
    Ff.zero();
    Fb.zero();
    double D = 0.0, Ec = 1.0;  // a (x_e - x_first), exp(-D)
    const double *vcol = A.vin + col;
#pragma unroll 1
    for (int b = 0; b < C::E; b += C::BLK) {
        double vb[C::BLK];
#pragma unroll
        for (int k = 0; k < C::BLK; ++k) {
            // clamped indices: a position past the end adds nothing
            const int sj = (b + k) * C::RUNS + run;
            vb[k] = gld(vcol + (int64_t)sm.c[sj] * A.W);
        }
#pragma unroll
        for (int k = 0; k < C::BLK; ++k) {
            const int e = b + k;
            const int sj = e * C::RUNS + run;
            scan_elem<C, 0, false>(sm, Ff, e, e, run, hh, vb[k]);
            // the staged step into position e (from e - 1); none for the first
            const double st = sm.st[sj], es = sm.est[sj];
            D = e > 0 ? D + st : D;
            Ec = e > 0 ? Ec * es : Ec;
            double pw[C::P];
            pw[0] = 1.0;
#pragma unroll
            for (int m = 1; m < C::P; ++m) pw[m] = pw[m - 1] * D * (1.0 / m);
            double geo[C::G > 0 ? C::G : 1];
            load_geo<C>(sm, sj, geo);
            ElemVec<C> ev;
            elem_vectors<C>(geo, ev);
            const int fl = sm.flags[sj];
            if constexpr (C::D >= 2 && C::NCLS == 2) {
                const bool s1 = fl & F_SIDE1;
                add_class_moved<C>(Fb, 0, ev, s1 ? 0.0 : vb[k], Ec, D, pw);
                add_class_moved<C>(Fb, 1, ev, s1 ? vb[k] : 0.0, Ec, D, pw);
            } else {
                int sc, tc;
                classes<C>(fl, hh, sc, tc);
#pragma unroll
                for (int c = 0; c < C::NCLS; ++c) add_class_moved<C>(Fb, c, ev, (c == sc) ? vb[k] : 0.0, Ec, D, pw);
            }
        }
    }
}

// One scan direction over this lane's run, with every carry.
// DIR 0: forward (increasing positions; sources at or before the target in
//        the last coordinate: delta_last = +1);
// DIR 1: backward (decreasing positions; sources strictly after: delta_last = -1).
// MODE 0: target values go to outv (short runs) or to the pass's slab (long
//         runs: the backward direction, run first, stores; the forward adds);
// MODE 1: the tile's total is written to the aggregates.
template <class C, int MODE, int DIR>
__device__ __forceinline__ void run_direction(const SweepArgs &A, const PassDev &ps, const Smem<C> &sm,
                                              int hh, int64_t tile, int pl, int col, int run,
                                              const double (&vr)[C::REGOUT ? C::E : 1],
                                              double (&outv)[C::SUMREG ? C::E : 1], double *slab, double *lout,
                                              const Cuts &cu, const State<C> *Fpre = nullptr) {
    const int seg = 1 << (ps.seg_log2 < 30 ? ps.seg_log2 : 30);
    const bool cut_run = DIR == 0 ? cu.f : cu.b;  // restart between the previous anchor and this run's
    // runs per segment group (1 when segments fit in a run)
    const int Gr = seg <= C::E ? 1 : (seg >= C::T ? C::RUNS : seg / C::E);
    const int lig = run & (Gr - 1);
    const double a = A.a;
    const double xbeg = sm.xrun[DIR == 0 ? 0 : 1][run];
    const double xend = sm.xrun[DIR == 0 ? 1 : 0][run];
    const double *vcol = A.vin + col;

    State<C> Ex;  // carry entering the run, anchored at xex
    Ex.zero();
    double xex = xbeg;

    if (Gr > 1) {
        // cross-tile passes: the pre-pass stored this run's within-tile carry
        bool stored = false;
        if constexpr (MODE == 0 && C::RUNEX) stored = seg > C::T && A.ntile > 1 && A.runex != nullptr;
        State<C> Frun;  // MODE 1: the run's own aggregate
        if (stored) {
            const int kx = gld(A.xtpos + A.g0 + pl) - A.k0;
            const double *src = A.runex + runex_index<C>(A, DIR, kx, tile, col / C::WCOL, hh) + threadIdx.x;
#pragma unroll
            for (int k = 0; k < C::NSLOT; ++k) Ex.flat()[k] = gld(src + k * WAVE);
            // anchored at the previous run's last position in the scan direction
            const bool has = DIR == 0 ? (run > 0) : (run < C::RUNS - 1);
            const int rp = DIR == 0 ? (run > 0 ? run - 1 : 0) : (run + 1 < C::RUNS ? run + 1 : run);
            const double xp = sm.xrun[DIR == 0 ? 1 : 0][rp];
            if (has) xex = xp;
        } else {
            // ---- run aggregate (anchored at xend); MODE 1 has both directions' already
            State<C> F;
            F.zero();
            if constexpr (MODE == 1) {
                F = *Fpre;
            } else if constexpr (C::REGOUT) {
#pragma unroll
                for (int i = 0; i < C::E; ++i) {
                    const int e = DIR == 0 ? i : C::E - 1 - i;
                    scan_elem<C, DIR, false>(sm, F, e, i, run, hh, vr[e]);
                }
            } else {
#pragma unroll 1
                for (int b = 0; b < C::E; b += C::BLK) {
                    double vb[C::BLK];
#pragma unroll
                    for (int k = 0; k < C::BLK; ++k) {
                        // staged indices are clamped to valid points: load unconditionally
                        // (a position past the end adds nothing: it has no source class or
                        // a zero source vector)
                        const int e = DIR == 0 ? b + k : C::E - 1 - b - k;
                        const int sj = e * C::RUNS + run;
                        vb[k] = gld(vcol + (int64_t)sm.c[sj] * A.W);
                    }
#pragma unroll
                    for (int k = 0; k < C::BLK; ++k) {
                        const int e = DIR == 0 ? b + k : C::E - 1 - b - k;
                        scan_elem<C, DIR, false>(sm, F, e, b + k, run, hh, vb[k]);
                    }
                }
            }
            if constexpr (MODE == 1) Frun = F;
            // ---- inclusive scan over the runs of this column.  Initial transfer: from
            // the previous run's anchor to this run's (none for a group's first run).
            double tr = 0.0, Er = 1.0;
            {
                const double xo = run_neighbour<C, DIR>(xend);
                const bool has = DIR == 0 ? (lig > 0) : (lig < Gr - 1);
                if (has) {
                    tr = a * (DIR == 0 ? xend - xo : xo - xend);
                    Er = exp(-tr);
                    if constexpr (C::D == 3)
                        if (cut_run) Er = 0.0;
                }
            }
            lane_scan<C, DIR>(F, tr, Er, lig, Gr, (int)(threadIdx.x % WAVE));
            // exclusive value
            {
                const double xp = run_neighbour<C, DIR>(xend);
                const bool has = DIR == 0 ? (lig > 0) : (lig < Gr - 1);
#pragma unroll
                for (int k = 0; k < C::NSLOT; ++k) {
                    const double q = run_neighbour<C, DIR>(F.flat()[k]);
                    Ex.flat()[k] = has ? q : 0.0;
                }
                if (has) xex = xp;
            }
        }
        if constexpr (MODE == 1) {
            if (C::RUNEX && A.runex != nullptr) {
                // every run's within-tile carry, for the main launch
                const int kx = gld(A.xtpos + A.g0 + pl) - A.k0;
                double *dst = A.runex + runex_index<C>(A, DIR, kx, tile, col / C::WCOL, hh) + threadIdx.x;
#pragma unroll
                for (int k = 0; k < C::NSLOT; ++k) gst(dst + k * WAVE, Ex.flat()[k]);
            }
            // tile total: inclusive value of the run that ends the tile in this direction
            if (run == (DIR == 0 ? C::RUNS - 1 : 0)) {
                State<C> tot = Ex;
                const double t = a * (DIR == 0 ? xend - xex : xex - xend);
                tot.shift(cut_run ? 0.0 : exp(-t), t);
                tot.add_shifted(Frun, 1.0, 0.0);
                double *dst = A.agg + agg_index<C>(A, DIR, pl, tile, col, hh);
#pragma unroll
                for (int k = 0; k < C::NSLOT; ++k) gst(dst + k, tot.flat()[k]);
                if (col == 0 && hh == 0) {
                    const int64_t ai = ((int64_t)DIR * A.G + pl) * A.ntile + tile;
                    gst(A.anc + ai, xend);
                    // decay across the tile from the previous tile's anchor; 1 for the
                    // segment's first tile in the scan direction (no predecessor)
                    const int64_t tps = seg / C::T;
                    const bool first = DIR == 0 ? (tile % tps) == 0 : (((tile + 1) % tps) == 0 || tile + 1 == A.ntile);
                    const double xo = sm.xedge[DIR == 0 ? 0 : 1];
                    const bool cut_tile = (DIR == 0 ? cu.mf : cu.mb) != 0;  // a restart inside the tile's span
                    gst(A.dec + ai, first ? 1.0 : (cut_tile ? 0.0 : exp(-a * (DIR == 0 ? xend - xo : xo - xend))));
                }
            }
            return;
        }
        // ---- carry from the other tiles of the segment (tile carry scan)
        if (seg > C::T && A.ntile > 1) {
            const int64_t tps = seg / C::T;
            const bool has_nb = DIR == 0 ? (tile % tps) != 0 : (((tile + 1) % tps) != 0 && tile + 1 < A.ntile);
            if (has_nb) {
                State<C> cf;
                const double *src = A.car + agg_index<C>(A, DIR, pl, tile, col, hh);
#pragma unroll
                for (int k = 0; k < C::NSLOT; ++k) cf.flat()[k] = gld(src + k);
                const double anc = gld(A.anc + ((int64_t)DIR * A.G + pl) * A.ntile + (DIR == 0 ? tile - 1 : tile + 1));
                if (run == (DIR == 0 ? 0 : C::RUNS - 1)) xex = anc;
                const double t = a * (DIR == 0 ? xex - anc : anc - xex);
                Ex.add_shifted(cf, cut_before_run<C, DIR>(cu, run) ? 0.0 : exp(-t), t);
            }
        }
    }
    if constexpr (MODE == 0) {
        // ---- the scan proper: targets read the state, then sources enter it
        State<C> S = Ex;
        if constexpr (C::REGOUT) {
#pragma unroll
            for (int i = 0; i < C::E; ++i) {
                const int e = DIR == 0 ? i : C::E - 1 - i;
                outv[e] += scan_elem<C, DIR, true>(sm, S, e, i, run, hh, vr[e]);
            }
        } else {
            auto block = [&](int b) {
                double vb[C::BLK], ob[C::BLK];
                int64_t addr[C::BLK];
#pragma unroll
                for (int k = 0; k < C::BLK; ++k) {
                    const int e = DIR == 0 ? b + k : C::E - 1 - b - k;
                    const int sj = e * C::RUNS + run;
                    // with one wave per sub-sweep a wave writes only its own targets
                    // (each element is a target of exactly one sub-sweep)
                    const bool valid = C::NWAVE > 1 ? is_target<C>(sm.flags[sj], hh) : (sm.flags[sj] & F_VALID) != 0;
                    const int64_t ad = (int64_t)sm.c[sj] * A.W + col;  // clamped: always in range
                    addr[k] = valid ? ad : -1;
                    vb[k] = gld(A.vin + ad);  // unused past the end (no source class)
                    // the slab already holds this element's earlier values unless this is
                    // its first write of the pass (the backward direction of its first
                    // sub-sweep: sub-sweep 0 when they run one after another, its own
                    // wave's when they run side by side)
                    if constexpr (!C::LDSOUT && !C::OUTREG) {
                        if (DIR == 0 || (C::NWAVE == 1 && hh > 0)) {
                            const double lo = gld(slab + ad);
                            ob[k] = valid ? lo : 0.0;
                        } else {
                            ob[k] = 0.0;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < C::BLK; ++k) {
                    const int e = DIR == 0 ? b + k : C::E - 1 - b - k;
                    const double val = scan_elem<C, DIR, true>(sm, S, e, b + k, run, hh, vb[k]);
                    if constexpr (C::OUTREG) {
                        // ring slot of element e in this block (see the rotation below)
                        const int q = DIR == 0 ? k : C::E - 1 - k;
                        outv[q] = (DIR == 0 || hh > 0) ? outv[q] + val : val;
                    } else if constexpr (C::LDSOUT) {
                        // this lane's own entry: no other lane of the wave touches it, and
                        // with one wave per sub-sweep the other wave skips it
                        double &o = lout[(e * C::RUNS + run) * C::WCOL + col % C::WCOL];
                        if constexpr (C::NWAVE > 1) {
                            if (is_target<C>(sm.flags[e * C::RUNS + run], hh)) o = DIR == 0 ? o + val : val;
                        } else {
                            o = (DIR == 0 || hh > 0) ? o + val : val;
                        }
                    } else {
                        if (addr[k] >= 0) gst(slab + addr[k], ob[k] + val);
                    }
                }
                if constexpr (C::OUTREG) {
                    // The run's sums form a ring in registers, indexed by constants in
                    // this rolled loop: a block works on the ring's first (forward) or
                    // last (backward) BLK slots, then the ring turns by BLK toward
                    // them.  After E / BLK blocks it has turned once, so slot e holds
                    // element e again between directions.
                    double r[C::E];
#pragma unroll
                    for (int i = 0; i < C::E; ++i) r[i] = outv[(i + (DIR == 0 ? C::BLK : C::E - C::BLK)) % C::E];
#pragma unroll
                    for (int i = 0; i < C::E; ++i) outv[i] = r[i];
                }
            };
#pragma unroll C::OUTU
            for (int b = 0; b < C::E; b += C::BLK) block(b);
        }
    }
}

// MODE 0: one (pass, tile, column block) of the group; targets' sums go to
// the pass's slab.  MODE 1: tile aggregates of the passes whose segments span
// several tiles.
template <class C, int MODE>
__device__ __forceinline__ void sweep_body(const SweepArgs &A, Smem<C> &sm, double *lout, int64_t bx, int by) {
    int pass;
    int64_t tile;
    if constexpr (MODE == 0) {
        pass = A.g0 + (int)(bx / A.ntile);
        tile = bx % A.ntile;
    } else {
        pass = A.xt[A.k0 + (int)(bx / A.ntile)];
        tile = bx % A.ntile;
    }
    const int pl = pass - A.g0;
    const PassDev ps = A.passes[pass];
    const int lane = threadIdx.x % WAVE;
    const int col = by * C::WCOL + lane % C::WCOL;
    const int run = lane / C::WCOL;
    const int64_t p0 = tile * C::T;
    stage_tile<C>(A, ps, sm, p0);
    const Cuts cu = tile_cuts<C>(sm, run);
    double *slab = A.ypart + (int64_t)pl * A.n * A.W;

    double vr[C::REGOUT ? C::E : 1], outv[C::SUMREG ? C::E : 1];
    if constexpr (C::OUTREG) {
#pragma unroll
        for (int e = 0; e < C::E; ++e) outv[e] = 0.0;
    }
    if constexpr (C::REGOUT) {
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int sj = e * C::RUNS + run;
            vr[e] = gld(A.vin + (int64_t)sm.c[sj] * A.W + col);  // clamped index; unused past the end
            outv[e] = 0.0;
        }
    }

    // sub-sweeps: one per wave when they run side by side, else one after another
    const int hh0 = C::NWAVE > 1 ? (int)(threadIdx.x / WAVE) : 0;
    const int hh1 = C::NWAVE > 1 ? hh0 + 1 : C::NSUB;
#pragma unroll 1
    for (int hh = hh0; hh < hh1; ++hh) {
        if constexpr (MODE == 1) {
            State<C> Ff, Fb;
            run_aggregates<C>(A, sm, run, col, hh, Ff, Fb);
            run_direction<C, MODE, 1>(A, ps, sm, hh, tile, pl, col, run, vr, outv, slab, lout, cu, &Fb);
            run_direction<C, MODE, 0>(A, ps, sm, hh, tile, pl, col, run, vr, outv, slab, lout, cu, &Ff);
        } else {
            run_direction<C, MODE, 1>(A, ps, sm, hh, tile, pl, col, run, vr, outv, slab, lout, cu);
            run_direction<C, MODE, 0>(A, ps, sm, hh, tile, pl, col, run, vr, outv, slab, lout, cu);
        }
    }

    if constexpr (MODE == 0 && C::SUMREG) {
        // With 16 or more columns per wave a run's lanes write whole 128-byte lines
        // of the slab, which a later launch reads once: streaming stores keep them
        // from displacing the gathered weight rows in L2.  Narrower rows are
        // partial lines, which need L2 to merge them.
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int sj = e * C::RUNS + run;
            if (sm.flags[sj] & F_VALID) {
                double *o = slab + (int64_t)sm.c[sj] * A.W + col;
                if constexpr (C::WCOL >= 16)
                    __builtin_nontemporal_store(outv[e], (__attribute__((address_space(1))) double *)o);
                else
                    gst(o, outv[e]);
            }
        }
    }
    if constexpr (MODE == 0 && C::LDSOUT) {
        // one write of each target's sums to the pass's slab (the waves of the
        // sub-sweeps take alternate elements, after both have finished)
        if constexpr (C::NWAVE > 1) __syncthreads();
        for (int e = (int)(threadIdx.x / WAVE); e < C::E; e += C::NWAVE) {
            const int sj = e * C::RUNS + run;
            if (sm.flags[sj] & F_VALID) gst(slab + (int64_t)sm.c[sj] * A.W + col, lout[sj * C::WCOL + lane % C::WCOL]);
        }
    }
}

template <class C, int MODE>
__global__ __launch_bounds__(C::BLOCK, C::MINW) void sweep_kernel(SweepArgs A) {
    __shared__ Smem<C> sm;
    if constexpr (MODE == 0 && C::LDSOUT) {
        __shared__ Lout<C> lo;
        sweep_body<C, MODE>(A, sm, lo.v, blockIdx.x, blockIdx.y);
    } else {
        sweep_body<C, MODE>(A, sm, nullptr, blockIdx.x, blockIdx.y);
    }
}

// Batched: every item (problem, block x, block y) of a table runs the same body
// with its problem's arguments, one workgroup per item.  (A persistent grid
// walking the table kept about 40 more VGPRs live across items and lost one
// wave per SIMD of occupancy in most configurations.)
template <class C, int MODE>
__global__ __launch_bounds__(C::BLOCK, C::MINW) void sweep_batch_kernel(const SweepArgs *__restrict__ descs, const int4 *__restrict__ items, int nitems) {
    __shared__ Smem<C> sm;
    double *lout = nullptr;
    if constexpr (MODE == 0 && C::LDSOUT) {
        __shared__ Lout<C> lo;
        lout = lo.v;
    }
    const int i = blockIdx.x;
    if (i >= nitems) return;
    const int4 it = items[i];
    const SweepArgs A = descs[it.x];
    sweep_body<C, MODE>(A, sm, lout, it.y, it.z);
}

// Exclusive scans of the tile aggregates over the tiles of each segment, in
// both directions: car[t] = the sum over the segment's tiles before t
// (forward) or after t (backward) of their aggregates, moved to the anchor
// next to t.  One wave per (segment, direction, slice): a slice is one
// (sub-sweep, class, channel row, column) P-vector.  Lanes take chunks of
// consecutive tiles, scan them serially, join the chunks with a lane scan and
// write the tiles' exclusive values.  `segs` lists (pass, first tile, end
// tile) of the segments that span several tiles; blockIdx.x indexes them.
// Segments of at most CARRY_SMALL tiles: one thread per (direction, slice)
// scans the segment's tiles serially (loads issued in blocks of 8 ahead of the
// updates).
constexpr int CARRY_SMALL = 32;

template <class C>
__device__ __forceinline__ void carry_small(const SweepArgs &A, int pass, int64_t t0, int64_t t1, int by) {
    // one thread per (direction, slice): the two scan directions run side by side
    const int sd = by * 256 + (int)threadIdx.x;
    if (sd >= 2 * A.nslice) return;
    const int dir = sd / A.nslice;
    const int sl = sd - dir * A.nslice;
    const int pl = pass - A.g0;
    const int colw = sl % C::WCOL;
    const int rowcb = sl / C::WCOL;
    constexpr int ROWS = C::NSUB * C::NCLS * C::NTH;
    const int row = rowcb % ROWS;
    const int cb = rowcb / ROWS;
    const int hh = row / (C::NCLS * C::NTH);
    const int ch = row % (C::NCLS * C::NTH);
    const int col = cb * C::WCOL + colw;
    const double a = A.a;
    const int64_t nt = t1 - t0;
    {
        const int64_t base = ((int64_t)dir * A.G + pl) * A.ntile;
        const double *anc = A.anc + base;
        const double *dec = A.dec + base;
        auto off = [&](int64_t t) -> int64_t { return agg_index<C>(A, dir, pl, t, col, hh) + (int64_t)ch * C::P; };
        double ex[C::P];
#pragma unroll
        for (int m = 0; m < C::P; ++m) ex[m] = 0.0;
        double xw = 0.0;
#pragma unroll 1
        for (int64_t b = 0; b < nt; b += 8) {
            double xb[8], db[8], gb[8][C::P];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const bool in = b + k < nt;
                const int64_t t = dir == 0 ? t0 + (in ? b + k : 0) : t1 - 1 - (in ? b + k : 0);
                xb[k] = gld(anc + t);
                db[k] = gld(dec + t);
#pragma unroll
                for (int m = 0; m < C::P; ++m) gb[k][m] = in ? gld(A.agg + off(t) + m) : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (b + k >= nt) break;
                const int64_t t = dir == 0 ? t0 + b + k : t1 - 1 - b - k;
                if (b + k > 0) {
#pragma unroll
                    for (int m = 0; m < C::P; ++m) gst(A.car + off(t) + m, ex[m]);
                    const double tt = a * (dir == 0 ? xb[k] - xw : xw - xb[k]);
                    mshift(ex, db[k], tt);
                }
#pragma unroll
                for (int m = 0; m < C::P; ++m) ex[m] += gb[k][m];
                xw = xb[k];
            }
        }
    }
}

template <class C>
__device__ __forceinline__ void carry_body(const SweepArgs &A, int64_t bx, int by) {
    const int4 sg = A.segs[bx];
    const int nslice = A.nslice;
    const int pass = sg.x;
    const int64_t t0 = sg.y, t1 = sg.z;
    if (t1 - t0 <= CARRY_SMALL) {
        carry_small<C>(A, pass, t0, t1, by);
        return;
    }
    const int pl = pass - A.g0;
    const int lane = threadIdx.x & (WAVE - 1);
    // one wave per (direction, slice): the two scan directions run side by side
    const int sd = by * 4 + threadIdx.x / WAVE;
    if (sd >= 2 * nslice) return;
    const int dir = sd / nslice;
    const int sl = sd - dir * nslice;
    const int colw = sl % C::WCOL;
    const int rowcb = sl / C::WCOL;  // (column block, row)
    constexpr int ROWS = C::NSUB * C::NCLS * C::NTH;
    const int row = rowcb % ROWS;
    const int cb = rowcb / ROWS;
    const int hh = row / (C::NCLS * C::NTH);
    const int ch = row % (C::NCLS * C::NTH);
    const int col = cb * C::WCOL + colw;
    const double a = A.a;
    const int64_t nt = t1 - t0;
    const int64_t chunk = (nt + WAVE - 1) / WAVE;
    const int64_t lo = t0 + lane * chunk;
    const int64_t hi = lo + chunk < t1 ? lo + chunk : t1;
    const int nact = (int)((nt + chunk - 1) / chunk);  // lanes holding tiles
    const bool active = lane < nact;
    const int64_t cnt = active ? hi - lo : 0;
    {
        const int64_t base = ((int64_t)dir * A.G + pl) * A.ntile;
        const double *anc = A.anc + base;
        const double *dec = A.dec + base;
        auto off = [&](int64_t t) -> int64_t { return agg_index<C>(A, dir, pl, t, col, hh) + (int64_t)ch * C::P; };
        // the chunk's tiles in the scan direction: cb0, cb0 + step, ...
        const int64_t cb0 = dir == 0 ? lo : hi - 1;
        const int64_t step = dir == 0 ? 1 : -1;
        // the segment's first tile in the scan direction: in lane 0 (forward) or in the
        // last active lane (backward), always as the chunk's first tile
        const bool seg_first = dir == 0 ? lane == 0 : lane == nact - 1;
        // ---- chunk aggregate, anchored at the chunk's last tile, and the chunk's
        // transfer (distance x a and decay) from the previous chunk's last anchor.
        // The first block's anchors, aggregates and decays stay in registers.
        double acc[C::P];
#pragma unroll
        for (int m = 0; m < C::P; ++m) acc[m] = 0.0;
        double xs8[8], g8[8][C::P], e8[8], tt8[8];
        double Ech = 1.0;
        double xprev = active ? anc[cb0] : anc[t1 - 1];
        const double xfirst = xprev;
        for (int64_t b = 0; b < cnt; b += 8) {
            double xb[8], db[8], gb[8][C::P];
#pragma unroll
            for (int k = 0; k < 8; ++k) {  // loads first, then the dependent updates
                const bool in = b + k < cnt;
                const int64_t t = in ? cb0 + step * (b + k) : cb0;
                xb[k] = gld(anc + t);
                db[k] = gld(dec + t);
#pragma unroll
                for (int m = 0; m < C::P; ++m) gb[k][m] = in ? gld(A.agg + off(t) + m) : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (b + k >= cnt) break;
                const double x = xb[k];
                const double tt = a * (dir == 0 ? x - xprev : xprev - x);
                const double E = (b + k == 0) ? 1.0 : db[k];  // exp(-tt), stored per tile
                Ech *= db[k];
                mshift(acc, E, tt);
#pragma unroll
                for (int m = 0; m < C::P; ++m) acc[m] += gb[k][m];
                xprev = x;
                if (b == 0) {
                    xs8[k] = x;
                    e8[k] = db[k];
                    tt8[k] = tt;
#pragma unroll
                    for (int m = 0; m < C::P; ++m) g8[k][m] = gb[k][m];
                }
            }
        }
        // inactive lanes hold a zero state and an identity transfer
        const double xa = xprev;
        const double xbefore = dir == 0 ? __shfl_up(xa, 1, WAVE) : __shfl_down(xa, 1, WAVE);
        double tr = 0.0, Er = 1.0;
        if (active && !seg_first) {
            tr = a * (dir == 0 ? xa - xbefore : xbefore - xa);
            Er = Ech;
        }
        (void)xfirst;
        // ---- inclusive lane scan toward the direction, transfers carried along
        for (int o = 1; o < WAVE; o <<= 1) {
            const double tp = dir == 0 ? __shfl_up(tr, o, WAVE) : __shfl_down(tr, o, WAVE);
            const double Ep = dir == 0 ? __shfl_up(Er, o, WAVE) : __shfl_down(Er, o, WAVE);
            double q[C::P];
#pragma unroll
            for (int m = 0; m < C::P; ++m) q[m] = dir == 0 ? __shfl_up(acc[m], o, WAVE) : __shfl_down(acc[m], o, WAVE);
            const bool ok = dir == 0 ? (lane >= o) : (lane + o < WAVE);
            if (ok) {
                madd(acc, q, Er, tr);
                tr += tp;
                Er *= Ep;
            }
        }
        // ---- exclusive value entering the chunk, anchored at the previous chunk's last tile
        double ex[C::P];
        {
            const bool has = dir == 0 ? (lane > 0) : (lane < WAVE - 1);
#pragma unroll
            for (int m = 0; m < C::P; ++m) {
                const double q = dir == 0 ? __shfl_up(acc[m], 1, WAVE) : __shfl_down(acc[m], 1, WAVE);
                ex[m] = has ? q : 0.0;
            }
        }
        if (!active) return;
        // ---- walk the chunk: each tile's carry is the running value anchored at the
        // previous tile's anchor; then the tile is included
        auto include = [&](double E, double tt, const double *g) {
            mshift(ex, E, tt);
#pragma unroll
            for (int m = 0; m < C::P; ++m) ex[m] += g[m];
        };
        if (cnt <= 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k >= cnt) break;
                const int64_t t = cb0 + step * k;
                if (k == 0 && seg_first) {
#pragma unroll
                    for (int m = 0; m < C::P; ++m) ex[m] += g8[0][m];
                } else {
#pragma unroll
                    for (int m = 0; m < C::P; ++m) gst(A.car + off(t) + m, ex[m]);
                    const double tt = k == 0 ? a * (dir == 0 ? xs8[0] - xbefore : xbefore - xs8[0]) : tt8[k];
                    include(e8[k], tt, g8[k]);
                }
            }
        } else {
            double xw = xbefore;
            for (int64_t b = 0; b < cnt; b += 8) {
                double xb[8], db[8], gb[8][C::P];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const bool in = b + k < cnt;
                    const int64_t t = in ? cb0 + step * (b + k) : cb0;
                    xb[k] = gld(anc + t);
                    db[k] = gld(dec + t);
#pragma unroll
                    for (int m = 0; m < C::P; ++m) gb[k][m] = in ? gld(A.agg + off(t) + m) : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (b + k >= cnt) break;
                    const int64_t t = cb0 + step * (b + k);
                    if (b + k == 0 && seg_first) {
#pragma unroll
                        for (int m = 0; m < C::P; ++m) ex[m] += gb[k][m];
                    } else {
#pragma unroll
                        for (int m = 0; m < C::P; ++m) gst(A.car + off(t) + m, ex[m]);
                        const double tt = a * (dir == 0 ? xb[k] - xw : xw - xb[k]);
                        include(db[k], tt, gb[k]);
                    }
                    xw = xb[k];
                }
            }
        }
    }
}

// A product's carry scans over a group's cross-tile segments (A.segs: the
// group's first): blocks [0, nsmall) give each segment ysmall slice groups of
// 256 threads and serve the segments of at most CARRY_SMALL tiles (the others
// return); the next blocks give the wider segments, listed in `big` (indices
// into the plan's table, first s0), ybig slice groups of 4 waves each.
template <class C>
__global__ __launch_bounds__(256) void carry_kernel(SweepArgs A, int64_t nsmall, int ysmall, int ybig,
                                                    const int32_t *big, int s0) {
    const int64_t b = blockIdx.x;
    if (b < nsmall) {
        const int64_t sg = b / ysmall;
        const int4 g = A.segs[sg];
        if (g.z - g.y > CARRY_SMALL) return;
        carry_body<C>(A, sg, (int)(b - sg * ysmall));
    } else {
        const int64_t j = b - nsmall;
        const int64_t k = j / ybig;
        carry_body<C>(A, (int64_t)gld(big + k) - s0, (int)(j - k * ybig));
    }
}

// Batched carry scans: items (problem, segment, slice group).
template <class C>
__global__ __launch_bounds__(256) void carry_batch_kernel(const SweepArgs *__restrict__ descs, const int4 *__restrict__ items, int nitems) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int4 it = items[i];
        const SweepArgs A = descs[it.x];
        carry_body<C>(A, it.y, it.z);
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
constexpr int BS1 = 256;

inline unsigned grid_1d(int64_t n) {
    int64_t g = (n + BS1 - 1) / BS1;
    if (g > 65535 * 8) g = 65535 * 8;
    return (unsigned)(g < 1 ? 1 : g);
}

inline int tile_index(int T) { return T >= 1024 ? 3 : (T >= 512 ? 2 : (T >= 256 ? 1 : 0)); }

// When the plan's profiling is on, record an event before the main sweep
// launch on its stream and return the closing event to record after it.
mm_status profile_begin(mm_plan p, int passes_covered, hipStream_t s, hipEvent_t *ev1) {
    *ev1 = nullptr;
    if (!p->profile) return MM_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MM_HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return MM_OK;  // a captured launch is not bracketed
    if (p->prof_used >= 4096) {
        double ms = 0.0;
        int64_t cnt = 0;
        MM_TRY(profile_flush(p, &ms, &cnt));
    }
    if (p->prof_used >= p->prof_events.size()) {
        hipEvent_t e0, e1;
        // timing events without the system-scope release fence: the fence writes
        // back the L2 after the bracketed launch and would be timed with it
        MM_HIP_TRY(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
        MM_HIP_TRY(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
        p->prof_events.push_back({e0, e1});
    }
    MM_HIP_TRY(hipEventRecord(p->prof_events[p->prof_used].first, s));
    *ev1 = p->prof_events[p->prof_used].second;
    p->prof_used++;
    p->prof_units += (int64_t)passes_covered;
    return MM_OK;
}

// The passes of plan p applied to vin, summed into yacc (added to it with add).
// With tail non-null, the last pass group's slabs are left unsummed in the
// plan's partial-slab buffer for the caller to fold into its output:
// tail[0] = that group's passes, tail[1] = 1 when yacc holds no earlier group.
template <class C>
mm_status run_passes(mm_plan p, const double *vin, double *yacc, int W, hipStream_t s, bool add = false,
                     int *tail = nullptr, const SweepWs *ws = nullptr, int runex = 1) {
    double *const ws_agg = ws ? ws->agg : static_cast<double *>(p->agg.ptr);
    double *const ws_part = ws ? ws->part : static_cast<double *>(p->part.ptr);
    static_assert(C::T == 128 || C::T == 256 || C::T == 512 || C::T == 1024, "tile sizes with a cross-tile pass list");
    const KParams kp = kparams(p->kernel, p->d);
    const int64_t n = p->n;
    const int ncb = W / C::WCOL;
    const int64_t ntile = (n + C::T - 1) / C::T;
    const int npass = (int)p->passes.size();
    const int64_t len = n * W;
    if (npass == 0) {
        if (tail) {
            tail[0] = 0;
            tail[1] = 1;
            return MM_OK;
        }
        if (add) return MM_OK;
        hipLaunchKernelGGL(zero_kernel, dim3(grid_1d(len)), dim3(BS1), 0, s, yacc, len);
        MM_HIP_TRY(hipGetLastError());
        return MM_OK;
    }
    const int ti = tile_index(C::T);
    const std::vector<int> &xt = p->xt_host[ti];
    const int gmax = group_passes(p, W);
    SweepArgs A{};
    A.xc = static_cast<const double *>(p->xc.ptr);
    A.passes = static_cast<const PassDev *>(p->pass_dev.ptr);
    A.xt = static_cast<const int32_t *>(p->pass_xt[ti].ptr);
    A.vin = vin;
    A.ypart = ws_part;
    A.n = n;
    A.ntile = ntile;
    A.W = W;
    A.a = kp.a;
    const size_t aggslab = (size_t)2 * gmax * ntile * W * C::NSUB * C::NSLOT;
    A.agg = ws_agg;
    A.car = A.agg + aggslab;
    A.anc = A.car + aggslab;
    A.dec = A.anc + (size_t)2 * gmax * ntile;
    A.runex = (p->d <= 2 && runex) ? A.dec + (size_t)2 * gmax * ntile : nullptr;  // see agg_bytes_for
    A.xtpos = static_cast<const int32_t *>(p->pass_xtpos[ti].ptr);
    for (int g0 = 0; g0 < npass; g0 += gmax) {
        const int G = npass - g0 < gmax ? npass - g0 : gmax;
        A.g0 = g0;
        A.G = G;
        // passes of the group whose segments span tiles: a contiguous range of xt
        int k0 = 0;
        while (k0 < (int)xt.size() && xt[k0] < g0) ++k0;
        int k1 = k0;
        while (k1 < (int)xt.size() && xt[k1] < g0 + G) ++k1;
        A.k0 = k0;
        if (k1 > k0 && ntile > 1) {
            const dim3 gx((unsigned)((k1 - k0) * ntile), (unsigned)ncb);
            hipLaunchKernelGGL((sweep_kernel<C, 1>), gx, dim3(C::BLOCK), 0, s, A);
            // segments of the group's cross-tile passes: a contiguous range of the plan's table
            const std::vector<int> &so = p->seg_off[ti];
            const int s0 = so[k0], s1 = so[k1];
            const int nslice = C::NSUB * C::NCLS * C::NTH * W;
            A.nslice = nslice;
            A.segs = static_cast<const int4 *>(p->seg_tab[ti].ptr) + s0;
            if (s1 > s0) {
                const std::vector<int> &bo = p->big_off[ti];
                const int b0 = bo[k0], b1 = bo[k1];
                const int ysmall = (2 * nslice + 255) / 256, ybig = (2 * nslice + 3) / 4;
                const int64_t nsmall = (int64_t)(s1 - s0) * ysmall;
                const int64_t nblk = nsmall + (int64_t)(b1 - b0) * ybig;
                const int32_t *big = static_cast<const int32_t *>(p->seg_big[ti].ptr);
                if (nblk > INT32_MAX) {
                    set_error("carry scan: %lld blocks exceed the grid limit", (long long)nblk);
                    return MM_ERR_ARG;
                }
                hipLaunchKernelGGL((carry_kernel<C>), dim3((unsigned)nblk), dim3(256), 0, s, A, nsmall, ysmall, ybig,
                                   big ? big + b0 : nullptr, s0);
            }
        }
        hipEvent_t ev1 = nullptr;
        if (!ws) MM_TRY(profile_begin(p, G, s, &ev1));  // (profiling creates events: not with a caller workspace)
        hipLaunchKernelGGL((sweep_kernel<C, 0>), dim3((unsigned)(G * ntile), (unsigned)ncb), dim3(C::BLOCK), 0, s, A);
        if (ev1) MM_HIP_TRY(hipEventRecord(ev1, s));
        if (tail && g0 + G >= npass) {
            tail[0] = G;
            tail[1] = g0 == 0 ? 1 : 0;
        } else {
            hipLaunchKernelGGL(accum_kernel, dim3(grid_1d(len)), dim3(BS1), 0, s,
                               static_cast<const double *>(ws_part), G, len, yacc, g0 == 0 && !add ? 1 : 0);
        }
    }
    MM_HIP_TRY(hipGetLastError());
    return MM_OK;
}

// Lane layout by the schedule: WCOL = sc.wb columns per wave and runs of E
// positions.  The default run length (sc.e = 0) gives tiles of 256 positions
// (E = 256 * WCOL / 64); in d = 2 with more than 8 columns the 4-column blocks
// take runs of 32 (tiles of 512: measured 5% faster at 16 columns, slower at 5
// to 8 and in d = 1 and 3).  The kernels of the headline configurations (the
// product form with nu = 3/2 in d = 2 and nu = 5/2 in d = 3) also come with
// the schedules the autotuner searches: blocks of 1 to 32 columns and tiles of
// 128 to 1024 positions.  with_cfg calls f(Tag<Cfg<...>>) for the
// configuration of (d, nu, form, schedule, W).
template <class C>
struct Tag {
    using type = C;
};

template <int D, int P, bool PROD>
constexpr bool TUNED = PROD && ((D == 2 && P == 2) || (D == 3 && P == 3));

// The extra (column block, run length) pairs of the tuned configurations.
constexpr int NTUNED = 8;
constexpr int TUNED_WB[NTUNED] = {1, 1, 4, 8, 8, 16, 16, 32};
constexpr int TUNED_E[NTUNED] = {8, 16, 8, 16, 32, 32, 64, 64};

template <int D, int P, bool PROD, int GJ = -1, class F>
mm_status with_wb(const Sched &sc, int W, F &&f) {
    if constexpr (GJ == -1 && TUNED<D, P, PROD>) {
        if (sc.wb == 1 && sc.e == 8) return f(Tag<Cfg<D, P, PROD, 1, 8, GJ>>{});
        if (sc.wb == 1 && sc.e == 16) return f(Tag<Cfg<D, P, PROD, 1, 16, GJ>>{});
        if (sc.wb == 4 && sc.e == 8) return f(Tag<Cfg<D, P, PROD, 4, 8, GJ>>{});
        if (sc.wb == 8 && sc.e == 16) return f(Tag<Cfg<D, P, PROD, 8, 16, GJ>>{});
        if (sc.wb == 8 && sc.e == 32) return f(Tag<Cfg<D, P, PROD, 8, 32, GJ>>{});
        if (sc.wb == 16 && sc.e == 32) return f(Tag<Cfg<D, P, PROD, 16, 32, GJ>>{});
        if (sc.wb == 16 && sc.e == 64) return f(Tag<Cfg<D, P, PROD, 16, 64, GJ>>{});
        if (sc.wb == 32 && sc.e == 64) return f(Tag<Cfg<D, P, PROD, 32, 64, GJ>>{});
    }
    const int WB = sc.wb;
    if (WB == 32) return f(Tag<Cfg<D, P, PROD, 32, 128, GJ>>{});
    if (WB == 4 && sc.e == 32) return f(Tag<Cfg<D, P, PROD, 4, 32, GJ>>{});
    if constexpr (D == 2)
        if (WB == 4 && W > 8 && sc.e == 0) return f(Tag<Cfg<D, P, PROD, 4, 32, GJ>>{});
    if (WB == 4) return f(Tag<Cfg<D, P, PROD, 4, 16, GJ>>{});
    if (WB == 2) return f(Tag<Cfg<D, P, PROD, 2, 8, GJ>>{});
    return f(Tag<Cfg<D, P, PROD, 1, 4, GJ>>{});
}

// Whether (wb, e) names a compiled configuration of the kernel class at width W
// (e = 0: the default run length of the block).
inline bool sched_compiled(int d, const KParams &kp, const Sched &sc, int W) {
    if (sc.wb < 1 || W % sc.wb != 0) return false;
    if (sc.e == 0) return sc.wb == 1 || sc.wb == 2 || sc.wb == 4 || sc.wb == 32;
    const bool base = (sc.wb == 1 && sc.e == 4) || (sc.wb == 2 && sc.e == 8) || (sc.wb == 4 && sc.e == 16) ||
                      (sc.wb == 4 && sc.e == 32) || (sc.wb == 32 && sc.e == 128);
    if (base) return true;
    const bool tuned = kp.prod && ((d == 2 && kp.P == 2) || (d == 3 && kp.P == 3));
    if (!tuned) return false;
    for (int k = 0; k < NTUNED; ++k)
        if (TUNED_WB[k] == sc.wb && TUNED_E[k] == sc.e) return true;
    return false;
}

template <int D, class F>
mm_status with_p(const KParams &kp, const Sched &sc, int W, F &&f) {
    if (kp.P == 1) return with_wb<D, 1, true>(sc, W, f);
    if constexpr (D == 1) {
        if (kp.P == 2) return with_wb<D, 2, true>(sc, W, f);
        return with_wb<D, 3, true>(sc, W, f);
    } else {
        if (kp.P == 2) return kp.prod ? with_wb<D, 2, true>(sc, W, f) : with_wb<D, 2, false>(sc, W, f);
        return kp.prod ? with_wb<D, 3, true>(sc, W, f) : with_wb<D, 3, false>(sc, W, f);
    }
}

template <class F>
mm_status with_cfg(int d, const KParams &kp, const Sched &sc, int W, F &&f) {
    if (d == 1) return with_p<1>(kp, sc, W, f);
    if (d == 2) return with_p<2>(kp, sc, W, f);
    return with_p<3>(kp, sc, W, f);
}

// Arguments of a problem's single pass group (all passes) for configuration C,
// with caller-owned aggregate and partial-slab workspaces.
template <class C>
SweepArgs make_args(mm_plan p, const double *vin, double *agg, double *part, int W, int gmax, int runex = 1) {
    const KParams kp = kparams(p->kernel, p->d);
    const int ti = tile_index(C::T);
    const int64_t ntile = (p->n + C::T - 1) / C::T;
    SweepArgs A{};
    A.xc = static_cast<const double *>(p->xc.ptr);
    A.passes = static_cast<const PassDev *>(p->pass_dev.ptr);
    A.xt = static_cast<const int32_t *>(p->pass_xt[ti].ptr);
    A.vin = vin;
    A.ypart = part;
    A.n = p->n;
    A.ntile = ntile;
    A.W = W;
    A.a = kp.a;
    const size_t aggslab = (size_t)2 * gmax * ntile * W * C::NSUB * C::NSLOT;
    A.agg = agg;
    A.car = A.agg + aggslab;
    A.anc = A.car + aggslab;
    A.dec = A.anc + (size_t)2 * gmax * ntile;
    A.runex = (p->d <= 2 && runex) ? A.dec + (size_t)2 * gmax * ntile : nullptr;  // see agg_bytes_for
    A.xtpos = static_cast<const int32_t *>(p->pass_xtpos[ti].ptr);
    A.nslice = C::NSUB * C::NCLS * C::NTH * W;
    A.segs = static_cast<const int4 *>(p->seg_tab[ti].ptr);
    A.g0 = 0;
    A.k0 = 0;
    A.G = (int)p->passes.size();
    return A;
}

}  // namespace
}  // namespace mm
