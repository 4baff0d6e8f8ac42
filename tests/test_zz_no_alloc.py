"""matern_mvm_noalloc, the product without device allocation, through the C ABI:
bitwise equal to matern_mvm (the same kernels on the same plan) on two calls in a
row, the second with a smaller input, and refusal of sizes beyond its scratch."""
import numpy as np
import pytest

import paper_2508_01864_amd as mm
import workloads
from gpu_util import MVM_TOL, mvm_errors, say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _pair(plan, v, nrhs):
    import torch
    vc = to_gpu(np.ascontiguousarray(np.atleast_2d(v.T) if v.ndim > 1 else v[None, :]))
    y_ref = torch.empty_like(vc)
    y_na = torch.full_like(vc, float("nan"))
    plan.mvm_raw(vc, y_ref, nrhs)
    plan.mvm_noalloc_raw(vc, y_na, nrhs)
    return to_np(y_ref), to_np(y_na)


def test_noalloc_equals_matern_mvm_twice_then_smaller(oracle_lib):
    # first call: the headline shape at 4 columns (multi-tile, cross-tile passes)
    p1 = workloads.config2(n=100_000, nrhs=4)
    plan1 = mm.Plan(to_gpu(p1.x), mm.Kernel(3, "product", 0.1))
    say("noalloc call 1: d=2 n=100000 nrhs=4")
    a, b = _pair(plan1, p1.v, 4)
    assert np.array_equal(a, b)
    # the oracle on sampled rows of the first call
    rows = np.random.default_rng(5).choice(p1.n, 64, replace=False)
    yref, yabs = oracle_lib.mvm(p1.x, p1.v, 3, "product", 0.1, z=p1.x[rows], with_abs=True)
    comp, nrm = mvm_errors(b.T[rows], yref, yabs)
    assert comp <= MVM_TOL and nrm <= MVM_TOL
    # second call: a smaller problem of another dimension and kernel, one column,
    # on the same (shared) scratch
    p2 = workloads.random_problem(4242, 3001, 3, 5, "product", 0.2)
    plan2 = mm.Plan(to_gpu(p2.x), mm.Kernel(5, "product", 0.2))
    say("noalloc call 2: d=3 n=3001 nrhs=1")
    a2, b2 = _pair(plan2, p2.v, 1)
    assert np.array_equal(a2, b2)
    yref2, yabs2 = oracle_lib.mvm(p2.x, p2.v, 5, "product", 0.2, with_abs=True)
    comp, nrm = mvm_errors(b2[0], yref2, yabs2)
    assert comp <= MVM_TOL and nrm <= MVM_TOL
    # and the first plan again (the scratch keeps the last call's contents)
    a3, b3 = _pair(plan1, p1.v, 4)
    assert np.array_equal(a3, b3) and np.array_equal(b3, b)
    plan2.close()
    plan1.close()


def test_noalloc_refuses_sizes_beyond_its_scratch():
    import torch
    p = workloads.config2(n=100_000)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
    vc = to_gpu(np.random.default_rng(1).standard_normal((8, p.n)))
    yc = torch.empty_like(vc)
    with pytest.raises(mm.MaternError) as e:
        plan.mvm_noalloc_raw(vc, yc, 8)
    say("refused: %s" % e.value)
    assert e.value.status == mm.MM_ERR_ARG and "scratch" in str(e.value)
    plan.close()
