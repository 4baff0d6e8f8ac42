"""Pivoted Cholesky preconditioner and preconditioned CG (Appendix A,
'Preconditioning') against the oracle.

* The factor: same pivots as the oracle's greedy pivoted Cholesky, and L
  equal to the oracle's within round-off.
* The solve: preconditioned CG reaches the oracle's direct solution (rtol
  1e-12, relative error <= 1e-8), with GLS fixed effects too, in fewer
  iterations than plain CG, and bitwise the same result alone and in a batch.
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


@pytest.mark.parametrize("d,two_nu,form", [(1, 3, "product"), (2, 3, "product"), (2, 1, "product"),
                                           (3, 5, "product"), (2, 3, "l1")])
def test_factor_matches_oracle(oracle_lib, d, two_nu, form):
    rng = np.random.default_rng(40 + d + two_nu)
    n, k, ell, s2 = 700, 30, 0.2, 1.3
    x = rng.uniform(0, 1, (n, d))
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, form, ell, s2))
    pc = mm.Precond(plan, max_rank=k)
    rank, tres, t0 = pc.info()
    Lg, gp = pc.factor()
    L = to_np(Lg)
    Lo, piv, res = oracle.pivoted_cholesky(x, two_nu, form, ell, s2, k)
    say("d=%d nu=%d/2 %s rank %d trace %.6e / %.6e (oracle %.6e)" % (d, two_nu, form, rank, tres, t0, res))
    assert rank == Lo.shape[1] == k
    assert abs(t0 - n * s2) <= 1e-9 * n * s2
    # pivots are integers decided in FP64 on both sides: compared exactly
    assert gp.tolist() == piv.tolist()
    assert np.max(np.abs(L - Lo)) <= 1e-10 * np.max(np.abs(Lo))
    assert abs(tres - res) <= 1e-8 * t0
    pc.close()
    plan.close()


def test_tolerance_and_full_rank(oracle_lib):
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (64, 2))
    plan = mm.Plan(to_gpu(x), mm.Kernel(1, "product", 0.5))
    pc = mm.Precond(plan, max_rank=64, tol=1e-3)
    rank, tres, t0 = pc.info()
    Lo, piv, res = oracle.pivoted_cholesky(x, 1, "product", 0.5, 1.0, 64, tol=1e-3)
    assert rank == Lo.shape[1] < 64
    assert tres <= 1e-3 * t0
    pc.close()
    full = mm.Precond(plan, max_rank=64)
    L = to_np(full.factor()[0])
    K = oracle.kernel_matrix(x, 1, "product", 0.5, 1.0)
    assert np.max(np.abs(L @ L.T - K)) <= 1e-10
    full.close()
    plan.close()


@pytest.mark.parametrize("d,two_nu", [(1, 5), (2, 3), (3, 3)])
def test_pcg_matches_direct_solve(oracle_lib, d, two_nu):
    n, ell, sig2 = 1500, 0.15, 0.01
    p = workloads.random_problem(900 + d, n, d, two_nu, "product", ell)
    y = workloads.field_sin_cos(p.x) + 0.1 * np.random.default_rng(3).standard_normal(n)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(two_nu, "product", ell))
    pc = mm.Precond(plan, max_rank=100)
    a_pc, _, i_pc = plan.cg_solve(to_gpu(y), sig2, rtol=1e-12, maxit=20000, precond=pc)
    a_cg, _, i_cg = plan.cg_solve(to_gpu(y), sig2, rtol=1e-12, maxit=20000)
    ref = oracle.gp_solve(p.x, y, two_nu, "product", ell, 1.0, sig2)
    say("d=%d nu=%d/2: pcg %d iters (err %.2e), cg %d iters" % (d, two_nu, i_pc["iters"], rel(to_np(a_pc), ref),
                                                              i_cg["iters"]))
    assert rel(to_np(a_pc), ref) <= SOLVE_TOL
    assert i_pc["iters"] < i_cg["iters"]
    pc.close()
    plan.close()


def test_pcg_gls_and_batch_equal_alone(oracle_lib):
    rng = np.random.default_rng(11)
    probs = []
    for d in (1, 2, 3, 2):
        n = int(rng.integers(600, 1500))
        x = rng.uniform(0, 1, (n, d))
        beta = rng.standard_normal(d + 1)
        y = oracle.design_matrix(x) @ beta + workloads.field_sin_cos(x) + 0.1 * rng.standard_normal(n)
        probs.append((x, y, d))
    alone = []
    for x, y, d in probs:
        plan = mm.Plan(to_gpu(x), mm.Kernel(3, workloads.solve_form(3, d), 0.2))
        pc = mm.Precond(plan, max_rank=40)
        a, b, info = plan.cg_solve(to_gpu(y), 0.02, fixed_effects=True, rtol=1e-12, precond=pc)
        bref, aref = oracle.gls(x, y, 3, workloads.solve_form(3, d), 0.2, 1.0, 0.02)
        assert rel(to_np(a), aref) <= SOLVE_TOL
        assert np.max(np.abs(b - bref)) <= SOLVE_TOL * max(1.0, np.max(np.abs(bref)))
        alone.append((to_np(a), b, info["iters"]))
        pc.close()
        plan.close()
    plans = [mm.Plan(to_gpu(x), mm.Kernel(3, workloads.solve_form(3, d), 0.2)) for x, y, d in probs]
    pcs = [mm.Precond(pl, max_rank=40) for pl in plans]
    # one problem without preconditioner shares the batch
    solvers = [mm.Solver(pl, to_gpu(y), 0.02, fixed_effects=True, rtol=1e-12, precond=pc if i != 3 else None)
               for i, (pl, pc, (x, y, d)) in enumerate(zip(plans, pcs, probs))]
    batch = mm.SolverBatch(solvers, use_graph=True)
    passed = [False] * len(solvers)
    for _ in range(400):
        batch.iterate(8)
        if converged(solvers, batch.poll(), passed):
            break
    for i, (s, (a0, b0, it0)) in enumerate(zip(solvers, alone)):
        a, b, info = s.finish()
        if i != 3:
            assert info["iters"] == it0
            assert np.array_equal(to_np(a), a0) and np.array_equal(b, b0)
        s.close()
    batch.close()
    for pc in pcs:
        pc.close()
    for pl in plans:
        pl.close()
