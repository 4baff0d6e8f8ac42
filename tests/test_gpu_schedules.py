"""Scan schedules (mm_plan_set_schedule): every compiled (column block, run
length, stored run carries) schedule of a plan's products gives the oracle's
product within the parity tolerance, at several widths, with tiles of 128 to
1024 positions, segments wider than a tile and a ragged last tile; a batch and
a solver follow the schedule of their plan (bitwise equal to the plan's own
product / solve alone)."""
import numpy as np
import pytest

import paper_2508_01864_amd as mm
from paper_2508_01864_amd import autotune
import workloads
from gpu_util import MVM_TOL, SOLVE_TOL, mvm_errors, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

CASES = [(2, 3, 5001, 1), (2, 3, 5001, 4), (2, 3, 5001, 8), (2, 3, 5001, 32),
         (3, 5, 2500, 1), (3, 5, 2500, 8), (3, 5, 2500, 32), (2, 5, 3000, 4)]


@pytest.mark.parametrize("d,two_nu,n,nrhs", CASES)
def test_every_schedule_matches_the_oracle(oracle_lib, d, two_nu, n, nrhs):
    import torch
    p = workloads.random_problem(1300 + 10 * d + n + nrhs, n, d, two_nu, "product", 0.1 if d == 2 else 0.2,
                                 nrhs=max(nrhs, 2))
    v = p.v[:, :nrhs]
    yref, yabs = oracle_lib.mvm(p.x, v, two_nu, "product", p.ell, with_abs=True, shared_kernel=True)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(two_nu, "product", p.ell))
    width = autotune.product_width(nrhs)
    vc = to_gpu(np.ascontiguousarray(v.T))
    yc = torch.empty_like(vc)
    for wb, e, rx in autotune.schedule_candidates(d, two_nu, "product", width):
        plan.set_schedule(width, wb, e, bool(rx))
        assert plan.schedule(width) == (wb, e, bool(rx))
        plan.mvm_raw(vc, yc, nrhs)
        comp, nrm = mvm_errors(to_np(yc).T, yref, yabs)
        say("d=%d nu=%d/2 n=%d nrhs=%d schedule (%d, %d, %d): comp %.2e nrm %.2e" %
            (d, two_nu, n, nrhs, wb, e, rx, comp, nrm))
        assert comp <= MVM_TOL and nrm <= MVM_TOL, (wb, e, rx)
    plan.close()


def test_schedule_rules():
    p = workloads.random_problem(1400, 300, 2, 1, "product", 0.2)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(1, "product", 0.2))
    assert plan.schedule(32) == (32, 128, True)
    assert plan.schedule(8) == (4, 16, True)
    with pytest.raises(mm.MaternError):
        plan.set_schedule(32, 16, 32)          # compiled only for the tuned kernel classes
    with pytest.raises(mm.MaternError):
        plan.set_schedule(4, 8, 16)            # 8 does not divide 4
    plan.set_schedule(4, 2, 8, False)
    assert plan.schedule(4) == (2, 8, False)
    plan.set_kernel(mm.Kernel(3, "product", 0.2))
    assert plan.schedule(4) == (4, 16, True)   # cleared with the kernel
    plan.close()


def test_batch_and_solver_follow_the_plan_schedule(oracle_lib):
    import torch
    probs = [workloads.random_problem(1500 + k, n, 2, 3, "product", 0.1) for k, n in enumerate((2000, 4500, 3100))]
    plans = [mm.Plan(to_gpu(q.x), mm.Kernel(3, "product", 0.1)) for q in probs]
    plans[0].set_schedule(4, 4, 8)
    plans[0].set_schedule(1, 1, 16)
    plans[1].set_schedule(4, 2, 8, False)
    plans[1].set_schedule(1, 1, 8)
    # products: one column, batched against alone
    vcs = [to_gpu(q.v).view(1, -1) for q in probs]
    alone = []
    for pl, vc in zip(plans, vcs):
        y = torch.empty_like(vc)
        pl.mvm_raw(vc, y, 1)
        alone.append(to_np(y))
    mb = mm.MvmBatch(plans, nrhs=1, use_graph=True)
    ycs = [torch.empty_like(vc) for vc in vcs]
    mb.run_raw(vcs, ycs)
    mb.close()
    for a, b in zip(alone, ycs):
        assert np.array_equal(a, to_np(b))
    # solves with fixed effects (width 4): alone against a batch, and the oracle
    ys = [workloads.field_sin_cos(q.x) + 0.05 * q.v for q in probs]
    ref = []
    for pl, y in zip(plans, ys):
        a, b, info = pl.cg_solve(to_gpu(y), 0.02, fixed_effects=True, rtol=1e-11)
        ref.append((to_np(a), b))
    from gpu_util import converged
    solvers = [mm.Solver(pl, to_gpu(y), 0.02, fixed_effects=True, rtol=1e-11) for pl, y in zip(plans, ys)]
    batch = mm.SolverBatch(solvers, use_graph=True)
    passed = [False] * len(solvers)
    for _ in range(2000):
        batch.iterate(8)
        if converged(solvers, batch.poll(), passed):
            break
    for k, (s, (a0, b0)) in enumerate(zip(solvers, ref)):
        a, b, info = s.finish()
        assert np.array_equal(to_np(a), a0) and np.array_equal(b, b0)
        q = probs[k]
        bref, aref = oracle_lib.gls(q.x, ys[k], 3, "product", 0.1, 1.0, 0.02)
        err = float(np.linalg.norm(to_np(a) - aref) / np.linalg.norm(aref))
        say("solve %d schedule %s: err %.2e" % (k, plans[k].schedule(4), err))
        assert err <= SOLVE_TOL
        s.close()
    batch.close()
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("runex", [True, False])
def test_carry_scan_paths_at_the_threshold(oracle_lib, runex):
    """A lone 32-column product on 128-position tiles (16 columns per wave, runs of
    32) whose passes have segments of exactly 32 tiles (scanned one thread per
    slice), 64 tiles (a wave per slice) and a ragged top segment of 97 tiles:
    12365 points."""
    import torch
    n, nrhs = 12365, 32
    p = workloads.random_problem(1700 + int(runex), n, 2, 3, "product", 0.1, nrhs=nrhs)
    yref, yabs = oracle_lib.mvm(p.x, p.v, 3, "product", p.ell, with_abs=True, shared_kernel=True)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", p.ell))
    plan.set_schedule(32, 16, 32, runex)
    vc = to_gpu(np.ascontiguousarray(p.v.T))
    yc = torch.empty_like(vc)
    plan.mvm_raw(vc, yc, nrhs)
    comp, nrm = mvm_errors(to_np(yc).T, yref, yabs)
    say("carry threshold: n=%d runex=%d comp %.2e nrm %.2e" % (n, runex, comp, nrm))
    assert comp <= MVM_TOL and nrm <= MVM_TOL
    plan.close()


def test_streamed_slabs_across_reused_buffers(oracle_lib):
    """Products on the 16-column schedule write their pass slabs with streaming
    stores.  Alternating inputs on one plan (the slab buffers reused each time)
    must reproduce each product bit for bit and match the oracle."""
    import torch
    n, nrhs = 9001, 32
    p = workloads.random_problem(1800, n, 2, 3, "product", 0.1, nrhs=nrhs)
    q = workloads.random_problem(1801, n, 2, 3, "product", 0.1, nrhs=nrhs)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", p.ell))
    plan.set_schedule(32, 16, 32, True)
    va = to_gpu(np.ascontiguousarray(p.v.T))
    vb = to_gpu(np.ascontiguousarray(q.v.T))
    outs = []
    for v in (va, vb, va, vb, va):
        y = torch.empty_like(v)
        plan.mvm_raw(v, y, nrhs)
        outs.append(to_np(y))
    assert np.array_equal(outs[0], outs[2]) and np.array_equal(outs[0], outs[4])
    assert np.array_equal(outs[1], outs[3])
    for v, y in ((p.v, outs[4]), (q.v, outs[3])):
        yref, yabs = oracle_lib.mvm(p.x, v, 3, "product", p.ell, with_abs=True, shared_kernel=True)
        comp, nrm = mvm_errors(y.T, yref, yabs)
        assert comp <= MVM_TOL and nrm <= MVM_TOL, (comp, nrm)
    plan.close()


@pytest.mark.parametrize("cfg", ["config2", "config3"])
def test_every_schedule_at_the_headline_size(oracle_lib, cfg):
    """The two timed 32-column products at full size: d = 2, N = 100 000, nu = 3/2,
    lengthscale 0.1 (x ~ U[0,1]^2), and d = 3, N = 500 000, nu = 5/2, lengthscale 0.3
    (x ~ N(0, I3), Rademacher columns), product form.  Every compiled schedule (the
    autotuner picks among exactly these) against the oracle on sampled target rows,
    and each schedule's product bitwise equal when repeated."""
    import torch
    if cfg == "config2":
        p = workloads.config2(nrhs=32)
        d, v, nrows = 2, p.v, 480
    else:
        p = workloads.config3()
        d, v, nrows = 3, p.probes, 200
    rows = np.random.default_rng(11).choice(p.n, nrows, replace=False)
    yref, yabs = oracle_lib.mvm(p.x, v, p.two_nu, "product", p.ell, z=p.x[rows], with_abs=True,
                                shared_kernel=True)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(p.two_nu, "product", p.ell))
    vc = to_gpu(np.ascontiguousarray(v.T))
    yc = torch.empty_like(vc)
    y2 = torch.empty_like(vc)
    cands = autotune.schedule_candidates(d, p.two_nu, "product", 32)
    assert (16, 32, 1) in cands if d == 2 else (32, 128, 1) in cands
    for wb, e, rx in cands:
        plan.set_schedule(32, wb, e, bool(rx))
        plan.mvm_raw(vc, yc, 32)
        plan.mvm_raw(vc, y2, 32)
        comp, nrm = mvm_errors(to_np(yc).T[rows], yref, yabs)
        say("%s, schedule (%d, %d, %d): comp %.2e nrm %.2e" % (cfg, wb, e, rx, comp, nrm))
        assert comp <= MVM_TOL and nrm <= MVM_TOL, (wb, e, rx)
        assert torch.equal(yc, y2), (wb, e, rx)
    plan.close()


EDGE_CASES = [(2, 3, "product", n) for n in (1, 2, 3, 31, 127, 128, 129, 255, 256, 257, 513)] + \
             [(3, 5, "product", n) for n in (1, 2, 129, 511, 512, 513, 1025)] + \
             [(d, 3, "l1", n) for d in (2, 3) for n in (1, 129, 256, 257, 1025)]


@pytest.mark.parametrize("d,two_nu,form,n", EDGE_CASES)
def test_every_schedule_at_tile_edges(oracle_lib, d, two_nu, form, n):
    """Plans of one point up to a few tiles, sized at and around the 128- to 1024-position
    tiles (no cross-tile pass, exactly one full tile, a one-position last tile): every
    schedule of the tuned classes (product form, d = 2 nu = 3/2 and d = 3 nu = 5/2) and
    of the L1 form at 4 and 32 columns against the whole oracle product."""
    import torch
    p = workloads.random_problem(7000 + 10 * d + n, n, d, two_nu, form, 0.1 * (d - 1), nrhs=32)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(two_nu, form, p.ell))
    for nrhs in (4, 32):
        v = p.v[:, :nrhs]
        yref, yabs = oracle_lib.mvm(p.x, v, two_nu, form, p.ell, with_abs=True, shared_kernel=True)
        vc = to_gpu(np.ascontiguousarray(v.T))
        yc = torch.empty_like(vc)
        for wb, e, rx in autotune.schedule_candidates(d, two_nu, form, nrhs):
            plan.set_schedule(nrhs, wb, e, bool(rx))
            plan.mvm_raw(vc, yc, nrhs)
            comp, nrm = mvm_errors(to_np(yc).T, yref, yabs)
            assert comp <= MVM_TOL and nrm <= MVM_TOL, (n, nrhs, wb, e, rx, comp, nrm)
    plan.close()
