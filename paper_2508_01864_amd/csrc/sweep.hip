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

// Kernel arguments for one pass.
struct SweepArgs {
    const double *xc;      // d x n canonical coordinates
    const int32_t *ord;    // pass order
    const int32_t *ord2;   // d = 3: level-l1 (x1, x2) order
    const double *vin;     // n x W point-major canonical input
    double *yacc;          // n x W point-major accumulator
    double *aggF;          // tile aggregates (forward / backward)
    double *aggB;
    double *ancF;          // tile anchors: last / first scan coordinate
    double *ancB;
    const double *carF;    // tile carries from the tile scan
    const double *carB;
    int64_t n;
    int W;                 // leading width of vin / yacc (columns)
    int l1, l2;
    int seg_log2;
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
};

// Stage the tile's positions: indices, flags, scan coordinate and offsets.
template <class C>
__device__ __forceinline__ void stage_tile(const SweepArgs &A, Smem<C> &sm, int64_t p0) {
    const int64_t n = A.n;
    const int64_t segmask = (int64_t(1) << A.seg_log2) - 1;
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
            c = A.ord[pc];
            const int l = A.l1;
            flags |= (int)((c >> l) & 1) ? F_SIDE1 : 0;
            int64_t sp = ((c >> (l + 1)) << (l + 1)) + (int64_t(1) << l);
            if (sp > n - 1) sp = n - 1;
            const double w = fabs(A.xc[c] - A.xc[sp]);
            const double t = A.a * w;
            sm.geo[0][j] = exp(-t);
            sm.geo[1][j] = t;
            sm.xs[j] = A.xc[n + c];
        } else {
            const int64_t q = A.ord[pc];
            c = A.ord2[q];
            const int l1 = A.l1, l2 = A.l2;
            flags |= (int)((c >> l1) & 1) ? F_SIDE1 : 0;
            flags |= (int)((q >> l2) & 1) ? F_SIDE2 : 0;
            int64_t sp1 = ((c >> (l1 + 1)) << (l1 + 1)) + (int64_t(1) << l1);
            if (sp1 > n - 1) sp1 = n - 1;
            int64_t sq2 = ((q >> (l2 + 1)) << (l2 + 1)) + (int64_t(1) << l2);
            if (sq2 > n - 1) sq2 = n - 1;
            const double w1 = fabs(A.xc[c] - A.xc[sp1]);
            const double w2 = fabs(A.xc[n + c] - A.xc[n + A.ord2[sq2]]);
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

// One scan direction over this thread's run of E positions, with every carry.
// DIR 0: forward (positions in increasing order, sources at or before the
//        target in the last coordinate: delta_last = +1);
// DIR 1: backward (decreasing order, sources strictly after: delta_last = -1).
// MODE 0 accumulates target values into outv; MODE 1 writes the tile's total.
template <class C, int MODE, int DIR>
__device__ __forceinline__ void run_direction(const SweepArgs &A, Smem<C> &sm, int hh, int tile,
                                              int rb, int nrb, double (&outv)[C::E][C::R]) {
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = tid / WAVE;
    const int j0 = tid * C::E;
    const int seg = 1 << (A.seg_log2 < 30 ? A.seg_log2 : 30);
    const int G = seg <= C::E ? 1 : (seg >= C::T ? WG : seg / C::E);
    const bool cross_tile = seg > C::T;
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
                double *dst = (DIR == 0 ? A.aggF : A.aggB) +
                              ((int64_t)(tile * nrb + rb) * C::NHALF + hh) * C::NSLOT;
#pragma unroll
                for (int i = 0; i < C::NSLOT; ++i) dst[i] = tot.flat()[i];
                if (rb == 0 && hh == 0) (DIR == 0 ? A.ancF : A.ancB)[tile] = xend;
            }
            return;
        }
        // ---- carry from the neighbouring tile of the same segment
        if (cross_tile) {
            const int64_t ntile = (A.n + C::T - 1) / C::T;
            const int tps = seg / C::T;
            const bool has_nb = DIR == 0 ? (tile % tps) != 0
                                         : (((tile + 1) % tps) != 0 && tile + 1 < ntile);
            if (has_nb) {
                State<C> cf;
                const double *src = (DIR == 0 ? A.carF : A.carB) +
                                    ((int64_t)(tile * nrb + rb) * C::NHALF + hh) * C::NSLOT;
#pragma unroll
                for (int i = 0; i < C::NSLOT; ++i) cf.flat()[i] = src[i];
                const double anc = DIR == 0 ? A.ancF[tile - 1] : A.ancB[tile + 1];
                if (tid == (DIR == 0 ? 0 : WG - 1)) xex = anc;
                const double t = a * (DIR == 0 ? xex - anc : anc - xex);
                Ex.add_shifted(cf, exp(-t), t);
            }
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

// MODE 0: full sweep (targets written); MODE 1: tile aggregates only.
template <class C, int MODE>
__global__ __launch_bounds__(WG) void sweep_kernel(SweepArgs A) {
    __shared__ Smem<C> sm;
    const int tile = blockIdx.x;
    const int rb = blockIdx.y;
    const int nrb = gridDim.y;
    const int64_t p0 = (int64_t)tile * C::T;
    stage_tile<C>(A, sm, p0);

    double outv[C::E][C::R];
#pragma unroll
    for (int e = 0; e < C::E; ++e)
#pragma unroll
        for (int r = 0; r < C::R; ++r) outv[e][r] = 0.0;

#pragma unroll 1
    for (int hh = 0; hh < C::NHALF; ++hh) {
        run_direction<C, MODE, 0>(A, sm, hh, tile, rb, nrb, outv);
        run_direction<C, MODE, 1>(A, sm, hh, tile, rb, nrb, outv);
    }

    if constexpr (MODE == 0) {
        const int j0 = threadIdx.x * C::E;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int j = j0 + e;
            if (sm.flags[j] & F_VALID) {
                double *dst = A.yacc + (int64_t)sm.c[j] * A.W + rb * C::R;
#pragma unroll
                for (int r = 0; r < C::R; ++r) dst[r] += outv[e][r];
            }
        }
    }
}

// Exclusive scan of tile aggregates inside each segment (one thread per
// independent slice: half, class, channel row, right-hand side).
template <class C>
__global__ __launch_bounds__(WG) void tile_scan_kernel(SweepArgs A, int tps, int64_t ntile,
                                                       double *carF, double *carB) {
    const int seg = blockIdx.x;
    const int rb = blockIdx.y;
    const int nrb = gridDim.y;
    constexpr int SLICES = C::NHALF * C::NCLS * C::NTH * C::R;
    const int64_t t0 = (int64_t)seg * tps;
    int64_t t1 = t0 + tps;
    if (t1 > ntile) t1 = ntile;
    const double a = A.a;
    for (int sl = threadIdx.x; sl < SLICES; sl += WG) {
        const int r = sl % C::R;
        const int rest = sl / C::R;          // (half, class, row)
        const int hh = rest / (C::NCLS * C::NTH);
        const int ch = rest % (C::NCLS * C::NTH);
        auto off = [&](int64_t t, int m) -> int64_t {
            return ((t * nrb + rb) * C::NHALF + hh) * C::NSLOT + ((int64_t)ch * C::P + m) * C::R + r;
        };
        // forward
        double acc[C::P];
#pragma unroll
        for (int m = 0; m < C::P; ++m) acc[m] = 0.0;
        double ax = A.ancF[t0];
        for (int64_t t = t0; t < t1; ++t) {
            const double x = A.ancF[t];
            if (t > t0) {
                const double tt = a * (x - ax);
                const double E = exp(-tt);
                // carry into tile t is acc anchored at ancF[t-1] (= ax)
#pragma unroll
                for (int m = 0; m < C::P; ++m) carF[off(t, m)] = acc[m];
                if constexpr (C::P == 3) acc[2] = E * (acc[2] + tt * acc[1] + 0.5 * tt * tt * acc[0]);
                if constexpr (C::P >= 2) acc[1] = E * (acc[1] + tt * acc[0]);
                acc[0] = E * acc[0];
            } else {
#pragma unroll
                for (int m = 0; m < C::P; ++m) carF[off(t, m)] = 0.0;
            }
#pragma unroll
            for (int m = 0; m < C::P; ++m) acc[m] += A.aggF[off(t, m)];
            ax = x;
        }
        // backward
#pragma unroll
        for (int m = 0; m < C::P; ++m) acc[m] = 0.0;
        ax = A.ancB[t1 - 1];
        for (int64_t t = t1 - 1; t >= t0; --t) {
            const double x = A.ancB[t];
            if (t < t1 - 1) {
                const double tt = a * (ax - x);
                const double E = exp(-tt);
#pragma unroll
                for (int m = 0; m < C::P; ++m) carB[off(t, m)] = acc[m];
                if constexpr (C::P == 3) acc[2] = E * (acc[2] + tt * acc[1] + 0.5 * tt * tt * acc[0]);
                if constexpr (C::P >= 2) acc[1] = E * (acc[1] + tt * acc[0]);
                acc[0] = E * acc[0];
            } else {
#pragma unroll
                for (int m = 0; m < C::P; ++m) carB[off(t, m)] = 0.0;
            }
#pragma unroll
            for (int m = 0; m < C::P; ++m) acc[m] += A.aggB[off(t, m)];
            ax = x;
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side dispatch.
// ---------------------------------------------------------------------------
constexpr int E_RUN = 4;

template <class C>
mm_status run_passes(mm_plan p, const double *vin, double *yacc, int W, hipStream_t s) {
    const KParams kp = kparams(p->kernel, p->d);
    const int64_t n = p->n;
    const int nrb = W / C::R;
    const int64_t ntile = (n + C::T - 1) / C::T;
    const size_t slab = (size_t)ntile * nrb * C::NHALF * C::NSLOT;
    double *base = static_cast<double *>(p->agg.ptr);
    SweepArgs A{};
    A.xc = static_cast<const double *>(p->xc.ptr);
    A.vin = vin;
    A.yacc = yacc;
    A.n = n;
    A.W = W;
    A.a = kp.a;
    A.aggF = base;
    A.aggB = base + slab;
    A.carF = base + 2 * slab;
    A.carB = base + 3 * slab;
    A.ancF = base + 4 * slab;
    A.ancB = base + 4 * slab + ntile;
    for (const Pass &ps : p->passes) {
        A.ord = ps.ord;
        A.ord2 = ps.ord2;
        A.l1 = ps.l1;
        A.l2 = ps.l2;
        A.seg_log2 = ps.seg_log2;
        dim3 grid((unsigned)ntile, (unsigned)nrb);
        if ((int64_t(1) << ps.seg_log2) > C::T && ntile > 1) {
            hipLaunchKernelGGL((sweep_kernel<C, 1>), grid, dim3(WG), 0, s, A);
            const int tps = (int)((int64_t(1) << ps.seg_log2) / C::T);
            const int64_t nseg = (ntile + tps - 1) / tps;
            hipLaunchKernelGGL((tile_scan_kernel<C>), dim3((unsigned)nseg, (unsigned)nrb), dim3(WG), 0, s,
                               A, tps, ntile, const_cast<double *>(A.carF), const_cast<double *>(A.carB));
        }
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
        }
        hipLaunchKernelGGL((sweep_kernel<C, 0>), grid, dim3(WG), 0, s, A);
        if (ev1) MM_HIP_TRY(hipEventRecord(ev1, s));
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

size_t sweep_agg_bytes(int64_t n, int d, int W, const mm_kernel &k) {
    (void)k;
    (void)d;
    // per tile and right-hand side at most NHALF*NCLS*NTH*P <= 108 doubles
    // (d = 3, product form, nu = 5/2), for each of the four arrays
    const int64_t ntile = (n + WG * E_RUN - 1) / (WG * E_RUN);
    const int64_t per_rhs = 128;
    return (size_t)(4 * ntile * (int64_t)W * per_rhs + 2 * ntile + 16) * sizeof(double);
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
