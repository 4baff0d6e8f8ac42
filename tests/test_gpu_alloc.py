"""The caller allocator (mm_set_allocator) on the GPU: with torch's caching
allocator registered, every library buffer comes from torch and goes back to
it, and results are bitwise those of the default allocator."""
import numpy as np
import pytest

import paper_2508_01864_amd as mm
import workloads
from gpu_util import say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _run(x, v, y):
    plan = mm.Plan(to_gpu(x), mm.Kernel(3, "product", 0.1))
    out = plan.mvm(to_gpu(v))
    alpha, beta, _ = plan.cg_solve(to_gpu(y), 0.01, fixed_effects=True, rtol=1e-10)
    res = (to_np(out), to_np(alpha), beta)
    return plan, res


def test_torch_allocator_serves_every_buffer(oracle_lib):
    import torch
    p = workloads.random_problem(9700, 3000, 2, 3, "product", 0.1)
    y = np.sin(4 * p.x[:, 0]) + 0.1 * p.v
    plan, ref = _run(p.x, p.v, y)
    plan.close()
    mm.use_torch_allocator(True)
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
        after_plan = torch.cuda.memory_allocated()
        plan.close()
        assert after_plan - base > 8 * 3000 * 2          # the plan's buffers are torch's
        plan, got = _run(p.x, p.v, y)
        before_close = torch.cuda.memory_allocated()
        plan.close()
        after_close = torch.cuda.memory_allocated()
        say("torch allocator: plan %d bytes, released %d bytes" % (after_plan - base, before_close - after_close))
        assert before_close - after_close >= after_plan - base
    finally:
        mm.use_torch_allocator(False)
    for a, b in zip(ref[:2], got[:2]):
        assert np.array_equal(a, b)
    assert np.array_equal(ref[2], got[2])
