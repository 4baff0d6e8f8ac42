"""Solver objects and batched iteration of independent GP problems.

A problem's iterates must not depend on the problems sharing its batch: every
solve here is compared bitwise with the same problem solved alone through
gp_cg_solve, for batches of uneven n, d, nu and lengthscale, with and without
HIP-graph replay, and the batched result is also checked against the
oracle's direct solve at the solve tolerance.
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
import workloads
from gpu_util import SOLVE_TOL, converged, say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _problems(seed, count, ds, n_lo, n_hi):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        d = int(ds[k % len(ds)])
        two_nu = int(rng.choice([1, 3, 5]))
        ell = float(np.exp(rng.uniform(np.log(0.05), np.log(0.5))))
        x = rng.uniform(0, 1, size=(n, d))
        trend = 0.3 + x @ rng.standard_normal(d)
        y = trend + workloads.field_sin_cos(x) + 0.1 * rng.standard_normal(n)
        out.append(dict(x=x, y=y, d=d, two_nu=two_nu, ell=ell, sig2=float(rng.uniform(0.01, 0.1))))
    return out


def _solve_alone(pr, fe, rtol, maxit):
    plan = mm.Plan(to_gpu(pr["x"]), mm.Kernel(pr["two_nu"], workloads.solve_form(pr["two_nu"], pr["d"]),
                                              pr["ell"]))
    alpha, beta, info = plan.cg_solve(to_gpu(pr["y"]), pr["sig2"], fixed_effects=fe, rtol=rtol, maxit=maxit)
    out = (to_np(alpha), beta, info)
    plan.close()
    return out


def _solve_batched(probs, fe, rtol, maxit, use_graph, chunk=8):
    plans, solvers = [], []
    for pr in probs:
        plan = mm.Plan(to_gpu(pr["x"]), mm.Kernel(pr["two_nu"], workloads.solve_form(pr["two_nu"], pr["d"]),
                                                  pr["ell"]))
        plans.append(plan)
        solvers.append(mm.Solver(plan, to_gpu(pr["y"]), pr["sig2"], fixed_effects=fe, rtol=rtol))
    batch = mm.SolverBatch(solvers, use_graph=use_graph)
    done = 0
    passed = [False] * len(solvers)
    while done < maxit:
        batch.iterate(chunk)
        done += chunk
        # unrelated eager work on the same stream between graph replays
        _ = to_gpu(np.arange(1000.0)).sum()
        if converged(solvers, batch.poll(), passed):
            break
    outs = []
    for s in solvers:
        alpha, beta, info = s.finish()
        outs.append((to_np(alpha), beta, info))
    batch.close()
    for s in solvers:
        s.close()
    for p in plans:
        p.close()
    return outs


def test_solver_steps_equal_gp_cg_solve(oracle_lib):
    """create / iterate / poll / finish gives gp_cg_solve's result bitwise."""
    pr = _problems(7, 1, [2], 2500, 2500)[0]
    a0, b0, i0 = _solve_alone(pr, True, 1e-10, 5000)
    plan = mm.Plan(to_gpu(pr["x"]), mm.Kernel(pr["two_nu"], workloads.solve_form(pr["two_nu"], 2), pr["ell"]))
    s = mm.Solver(plan, to_gpu(pr["y"]), pr["sig2"], fixed_effects=True, rtol=1e-10)
    while True:
        s.iterate(5)
        act, brk, info = s.poll()
        assert brk == 0
        if act == 0 and s.check(tighten=True)[0]:
            break
    alpha, beta, info = s.finish()
    say("steps: iters %d vs %d" % (info["iters"], i0["iters"]))
    assert info["iters"] == i0["iters"]
    assert np.array_equal(to_np(alpha), a0)
    assert np.array_equal(beta, b0)
    s.close()
    plan.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_alone_uneven(oracle_lib, use_graph):
    """Uneven (n, d, nu, ell, sigma2), one column each: bitwise equal to solo solves."""
    probs = _problems(11, 7, [1, 2, 3], 40, 4000)
    probs.append(dict(x=np.array([[0.3]]), y=np.array([1.5]), d=1, two_nu=3, ell=0.2, sig2=0.05))   # n = 1
    probs.append(dict(x=np.array([[0.1, 0.2], [0.4, 0.4]]), y=np.array([1.0, -2.0]), d=2, two_nu=5,
                      ell=0.3, sig2=0.05))                                                            # n = 2
    say("batch graph=%s sizes %s" % (use_graph, [len(p["y"]) for p in probs]))
    outs = _solve_batched(probs, False, 1e-10, 20000, use_graph)
    for pr, (a, _, info) in zip(probs, outs):
        a0, _, i0 = _solve_alone(pr, False, 1e-10, 20000)
        assert info["status"] == "MM_OK"
        assert info["iters"] == i0["iters"]
        assert np.array_equal(a, a0), "n=%d d=%d" % (len(pr["y"]), pr["d"])


def test_batch_gls_mixed_dims_equals_alone(oracle_lib):
    """Fixed effects: d = 1 (3 columns) and d = 2 (4 columns) share a width of 4."""
    probs = _problems(23, 5, [1, 2], 300, 3000)
    outs = _solve_batched(probs, True, 1e-10, 20000, True)
    for pr, (a, b, info) in zip(probs, outs):
        a0, b0, i0 = _solve_alone(pr, True, 1e-10, 20000)
        assert info["iters"] == i0["iters"]
        assert np.array_equal(a, a0)
        assert np.array_equal(b, b0)


def test_batch_gls_all_dims_matches_oracle_and_alone(oracle_lib):
    """d = 3 with fixed effects (5 columns, width 8) mixed with d = 1, 2 (width 4)."""
    probs = _problems(31, 5, [1, 2, 3], 500, 1500)
    outs = _solve_batched(probs, True, 1e-12, 20000, True)
    for pr, (a, b, info) in zip(probs, outs):
        form = workloads.solve_form(pr["two_nu"], pr["d"])
        bref, aref = oracle.gls(pr["x"], pr["y"], pr["two_nu"], form, pr["ell"], 1.0, pr["sig2"])
        say("d=%d n=%d iters %d err %.2e" % (pr["d"], len(pr["y"]), info["iters"], rel(a, aref)))
        assert rel(a, aref) <= SOLVE_TOL
        assert np.max(np.abs(b - bref)) <= SOLVE_TOL * max(1.0, np.max(np.abs(bref)))
        a0, b0, _ = _solve_alone(pr, True, 1e-12, 20000)
        assert np.array_equal(a, a0) and np.array_equal(b, b0)


def test_batch_schedule_does_not_change_results(oracle_lib):
    probs = _problems(41, 4, [2, 3], 500, 3000)
    ref = None
    for sched in [(1, 64), (8, 2048), (3, 7)]:
        plans = [mm.Plan(to_gpu(p["x"]), mm.Kernel(p["two_nu"], workloads.solve_form(p["two_nu"], p["d"]),
                                                    p["ell"])) for p in probs]
        solvers = [mm.Solver(pl, to_gpu(p["y"]), p["sig2"]) for pl, p in zip(plans, probs)]
        b = mm.SolverBatch(solvers, use_graph=True)
        b.set_schedule(*sched)
        b.iterate(40)
        res = [to_np(s.finish(raise_on_error=False)[0]) for s in solvers]
        if ref is None:
            ref = res
        else:
            for r0, r1 in zip(ref, res):
                assert np.array_equal(r0, r1)
        b.close()
        for s in solvers:
            s.close()
        for pl in plans:
            pl.close()


def test_live_solvers_pin_their_plan(oracle_lib):
    x1 = to_gpu(np.random.default_rng(0).uniform(0, 1, (200, 1)))
    y = to_gpu(np.ones(200))
    p1 = mm.Plan(x1, mm.Kernel(3, "product", 0.2))
    s1 = mm.Solver(p1, y, 0.05, fixed_effects=True)
    with pytest.raises(mm.MaternError) as e:
        p1.set_kernel(mm.Kernel(1, "product", 0.3))
    assert e.value.status == mm.MM_ERR_ARG
    with pytest.raises(mm.MaternError) as e:
        p1.close()
    assert e.value.status == mm.MM_ERR_ARG
    s1.close()
    p1.set_kernel(mm.Kernel(1, "product", 0.3))
    p1.close()


@pytest.mark.parametrize("use_graph,nrhs", [(False, 1), (True, 1), (True, 4)])
def test_mvm_batch_equals_matern_mvm(oracle_lib, use_graph, nrhs):
    """Batched products of uneven problems: bitwise the single-plan products, over
    repeated runs with new input and output buffers."""
    rng = np.random.default_rng(77)
    probs = []
    for k in range(9):
        n = int(np.exp(rng.uniform(np.log(2), np.log(6000)))) if k else 1
        d = 1 + k % 3
        two_nu = [1, 3, 5][(k // 3) % 3]
        form = "l1" if (k % 4 == 3 and two_nu > 1) else "product"
        probs.append((rng.uniform(0, 1, (n, d)), two_nu, form, float(np.exp(rng.uniform(np.log(0.05), np.log(0.5))))))
    plans = [mm.Plan(to_gpu(x), mm.Kernel(t, f, l, 1.7)) for x, t, f, l in probs]
    batch = mm.MvmBatch(plans, nrhs=nrhs, use_graph=use_graph)
    for rep in range(3):
        vs = [to_gpu(rng.standard_normal((p.n, nrhs)) if nrhs > 1 else rng.standard_normal(p.n)) for p in plans]
        ys = batch.run(vs, shift=0.03)
        for (x, t, f, l), p, v, y in zip(probs, plans, vs, ys):
            y0 = p.mvm(v, shift=0.03)
            assert np.array_equal(to_np(y), to_np(y0)), "rep %d n=%d d=%d" % (rep, p.n, p.d)
    # one problem against the oracle
    x, t, f, l = probs[4]
    v = rng.standard_normal(plans[4].n)
    vs = [to_gpu(rng.standard_normal(p.n) if nrhs == 1 else rng.standard_normal((p.n, nrhs))) for p in plans]
    vs[4] = to_gpu(v if nrhs == 1 else np.repeat(v[:, None], nrhs, axis=1))
    ys = batch.run(vs)
    yref, yabs = oracle.mvm(x, v, t, f, l, s2=1.7, with_abs=True)
    got = to_np(ys[4]) if nrhs == 1 else to_np(ys[4])[:, 0]
    assert np.max(np.abs(got - yref) / yabs) <= 1e-10
    batch.close()
    for p in plans:
        p.close()
