// Lengthscale-derivative sweeps: yacc <- sum over the D&C passes of the
// off-diagonal sums of l dK/dl applied to vin (unscaled by the output scale).
//
// With t = a r, l d/dl k(a r) = -t k'(t) is a profile in the same scaled
// power basis with one more channel (sweep_core.h).  The L1 form's kernel
// is k(a ||u||_1), so its derivative is that profile of the summed offset:
// one sweep.  The product form's kernel is prod_k k(a |u_k|), so
//     l dK/dl = sum_j [l dk/dl](a |u_j|) prod_{k != j} k(a |u_k|),
// one sweep per coordinate j with factor j replaced by the derivative
// profile; the sweeps add into the same output.  This restates the
// lengthscale gradients of the Section 2.3 examples (L1 nu = 1/2, 3/2, 5/2
// and the product nu = 3/2 example) for every nu and form.  The diagonal of
// K does not depend on l, so it contributes nothing.

#include "sweep_core.h"

namespace mm {
namespace {

template <int D, int P, bool PROD, class F>
mm_status with_gj(int gj, int WBlk, int W, F &&f) {
    const Sched WB{WBlk, 0, 1};  // the derivative sweeps run the default schedule of the block
    if constexpr (!PROD) {
        (void)gj;
        return with_wb<D, P, false, D - 1>(WB, W, f);
    } else {
        if constexpr (D >= 3)
            if (gj == 2) return with_wb<D, P, true, 2>(WB, W, f);
        if constexpr (D >= 2)
            if (gj == 1) return with_wb<D, P, true, 1>(WB, W, f);
        return with_wb<D, P, true, 0>(WB, W, f);
    }
}

template <int D, class F>
mm_status with_p_gj(const KParams &kp, int gj, int WB, int W, F &&f) {
    if (kp.P == 1) return with_gj<D, 1, true>(gj, WB, W, f);
    if constexpr (D == 1) {
        if (kp.P == 2) return with_gj<D, 2, true>(gj, WB, W, f);
        return with_gj<D, 3, true>(gj, WB, W, f);
    } else {
        if (kp.P == 2) return kp.prod ? with_gj<D, 2, true>(gj, WB, W, f) : with_gj<D, 2, false>(gj, WB, W, f);
        return kp.prod ? with_gj<D, 3, true>(gj, WB, W, f) : with_gj<D, 3, false>(gj, WB, W, f);
    }
}

}  // namespace

mm_status sweep_all_dl(mm_plan p, const double *vin, double *yacc, int W, int WB, hipStream_t s) {
    const KParams kp = kparams(p->kernel, p->d);
    if ((WB != 1 && WB != 2 && WB != 4 && WB != 32) || W % WB != 0) {
        set_error("internal: width %d does not match the block %d", W, WB);
        return MM_ERR_ARG;
    }
    const int d = p->d;
    // product form: one sweep per differentiated coordinate; L1: one sweep
    const int nsweep = kp.prod ? d : 1;
    for (int j = 0; j < nsweep; ++j) {
        const int gj = kp.prod ? j : d - 1;
        auto run = [&](auto t) {
            using C = typename decltype(t)::type;
            return run_passes<C>(p, vin, yacc, W, s, j > 0);
        };
        mm_status st;
        if (d == 1) st = with_p_gj<1>(kp, gj, WB, W, run);
        else if (d == 2) st = with_p_gj<2>(kp, gj, WB, W, run);
        else st = with_p_gj<3>(kp, gj, WB, W, run);
        if (st != MM_OK) return st;
    }
    return MM_OK;
}

}  // namespace mm
