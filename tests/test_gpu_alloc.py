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


def test_allocator_switch_with_live_objects():
    """Objects created under one allocator are released through it after the
    process has switched allocators (the callbacks stay alive)."""
    p = workloads.random_problem(9701, 2000, 2, 3, "product", 0.1)
    mm.use_torch_allocator(True)
    try:
        plan_a = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
        ya = to_np(plan_a.mvm(to_gpu(p.v)))
        mm.use_torch_allocator(True)              # a second registration replaces the first
        plan_b = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
    finally:
        mm.use_torch_allocator(False)             # back to hipMalloc with both plans alive
    plan_c = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
    yb = to_np(plan_b.mvm(to_gpu(p.v)))
    yc = to_np(plan_c.mvm(to_gpu(p.v)))
    plan_a.close()                                # frees through the first pair of callbacks
    plan_b.close()
    plan_c.close()
    assert np.array_equal(ya, yb) and np.array_equal(ya, yc)


def test_nomem_from_the_caller_allocator():
    """An allocator that runs out (returns NULL) makes the call fail with
    MM_ERR_NOMEM; buffers obtained before the failure are returned to it."""
    import ctypes
    import torch
    p = workloads.random_problem(9702, 3000, 2, 3, "product", 0.1)
    x = to_gpu(p.x)
    for allow in (0, 3):
        live = {}

        def _alloc(nbytes, stream, ctx):
            if len(live) >= allow:
                return None
            ptr = int(torch.cuda.caching_allocator_alloc(int(nbytes)))
            live[ptr] = nbytes
            return ptr

        def _free(ptr, stream, ctx):
            live.pop(int(ptr))
            torch.cuda.caching_allocator_delete(int(ptr))

        fa, ff = mm._ALLOC_FN(_alloc), mm._FREE_FN(_free)
        mm._allocator_refs.append((fa, ff))
        L = mm.lib()
        assert L.mm_set_allocator(ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ff, ctypes.c_void_p), None) == 0
        try:
            with pytest.raises(mm.MaternError) as e:
                mm.Plan(x, mm.Kernel(3, "product", 0.1))
        finally:
            mm.use_torch_allocator(False)
        say("allocator allowing %d buffers: %s" % (allow, e.value))
        assert e.value.status == mm.MM_ERR_NOMEM
        assert not live                           # every buffer it gave went back
    # a plan's product workspace is allocated at the first product: NOMEM there too
    plan = mm.Plan(x, mm.Kernel(3, "product", 0.1))
    fa = mm._ALLOC_FN(lambda n, s, c: None)
    ff = mm._FREE_FN(lambda ptr, s, c: None)
    mm._allocator_refs.append((fa, ff))
    assert mm.lib().mm_set_allocator(ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ff, ctypes.c_void_p), None) == 0
    try:
        with pytest.raises(mm.MaternError) as e:
            plan.mvm(to_gpu(p.v))
    finally:
        mm.use_torch_allocator(False)
    assert e.value.status == mm.MM_ERR_NOMEM
    y = to_np(plan.mvm(to_gpu(p.v)))              # usable again with hipMalloc
    assert np.all(np.isfinite(y))
    plan.close()
