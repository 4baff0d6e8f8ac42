"""GPU conjugate-gradient solve, GLS fixed effects and predictor vs the oracle.

CG is run to rtol 1e-12 and compared with the direct Cholesky solution of the
oracle: relative 2-norm error <= 1e-8.  Status paths (not positive definite,
no convergence) are forced from the host with valid inputs.
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
import workloads
from gpu_util import MVM_TOL, SOLVE_TOL, say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("d,two_nu", [(1, 1), (1, 5), (2, 3), (2, 5), (3, 3)])
def test_cg_matches_cholesky(oracle_lib, d, two_nu):
    n, ell, sig2 = 1500, 0.15, 0.01
    p = workloads.random_problem(600 + d + two_nu, n, d, two_nu, "product", ell)
    y = workloads.field_sin_cos(p.x) + 0.1 * np.random.default_rng(1).standard_normal(n)
    say("cg d=%d nu=%d/2" % (d, two_nu))
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(two_nu, "product", ell))
    alpha, _, info = plan.cg_solve(to_gpu(y), sig2, rtol=1e-12, maxit=20000)
    ref = oracle.gp_solve(p.x, y, two_nu, "product", ell, 1.0, sig2)
    say("iters", info["iters"], "err", rel(to_np(alpha), ref))
    assert rel(to_np(alpha), ref) <= SOLVE_TOL
    plan.close()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gls_fixed_effects(oracle_lib, d):
    """beta = (H^T A^-1 H)^-1 H^T A^-1 y and alpha = A^-1 (y - H beta) (Section 3.2)."""
    n, ell, sig2 = 1200, 0.2, 0.02
    rng = np.random.default_rng(50 + d)
    x = rng.uniform(0, 1, size=(n, d))
    beta_true = rng.standard_normal(d + 1)
    y = oracle.design_matrix(x) @ beta_true + workloads.field_sin_cos(x) + 0.1 * rng.standard_normal(n)
    two_nu = 3
    form = workloads.solve_form(two_nu, d)
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, form, ell))
    alpha, beta, info = plan.cg_solve(to_gpu(y), sig2, fixed_effects=True, rtol=1e-12)
    bref, aref = oracle.gls(x, y, two_nu, form, ell, 1.0, sig2)
    say("gls d=%d iters %d beta %s ref %s" % (d, info["iters"], beta, bref))
    assert np.max(np.abs(beta - bref)) <= SOLVE_TOL * max(1.0, np.max(np.abs(bref)))
    assert rel(to_np(alpha), aref) <= SOLVE_TOL
    # predictor at new points with the GPU estimates vs the oracle predictor
    z = rng.uniform(0, 1, size=(300, d))
    mean = to_np(plan.predict(alpha, to_gpu(z), beta=beta))
    mref = oracle.predict(x, to_np(alpha), z, two_nu, form, ell, 1.0, beta=beta)
    _, kabs = oracle.mvm(x, np.abs(to_np(alpha)), two_nu, form, ell, z=z, with_abs=True)
    scale = kabs + np.abs(oracle.design_matrix(z)) @ np.abs(beta)
    assert np.max(np.abs(mean - mref) / scale) <= MVM_TOL
    plan.close()


def test_predict_at_training_points_identity(oracle_lib):
    """H beta + K alpha = y - sigma^2 alpha at z = x, with the GPU solve."""
    n, d, ell, sig2 = 2000, 2, 0.1, 0.05
    p = workloads.config2(n=n)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", ell))
    alpha, beta, _ = plan.cg_solve(to_gpu(p.y), sig2, fixed_effects=True, rtol=1e-12)
    mean = to_np(plan.predict(alpha, to_gpu(p.x), beta=beta))
    a = to_np(alpha)
    assert np.max(np.abs(mean - (p.y - sig2 * a))) <= 1e-7 * np.max(np.abs(p.y))
    plan.close()


def test_multi_column_cg(oracle_lib):
    n, d, ell, sig2 = 1500, 2, 0.12, 0.01
    p = workloads.random_problem(88, n, d, 5, "product", ell, nrhs=5)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(5, "product", ell))
    X, info = plan.cg_solve_multi(to_gpu(p.v), sig2, rtol=1e-12)
    A = oracle.kernel_matrix(p.x, 5, "product", ell, 1.0, sigma2=sig2)
    ref = oracle.cholesky_solve(oracle.cholesky(A), p.v)
    for c in range(5):
        assert rel(to_np(X)[:, c], ref[:, c]) <= SOLVE_TOL
    assert info["converged_cols"] == 5
    plan.close()


def test_config2_subsample_solve(oracle_lib):
    """Configuration 2's solve on its first 5000 points vs Cholesky."""
    p = workloads.config2(n=100_000)
    xs, ys = p.x[:5000], p.y[:5000]
    plan = mm.Plan(to_gpu(xs), mm.Kernel(3, "product", 0.1))
    alpha, _, info = plan.cg_solve(to_gpu(ys), 0.01, rtol=1e-12, maxit=20000)
    ref = oracle.gp_solve(xs, ys, 3, "product", 0.1, 1.0, 0.01)
    say("config2 5k solve iters", info["iters"], "err", rel(to_np(alpha), ref))
    assert rel(to_np(alpha), ref) <= SOLVE_TOL
    plan.close()


def test_l1_form_refused_for_solves(oracle_lib):
    p = workloads.random_problem(3, 500, 2, 3, "l1", 0.1)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "l1", 0.1))
    with pytest.raises(mm.MaternError) as e:
        plan.cg_solve(to_gpu(p.v), 0.01)
    assert e.value.status == mm.MM_ERR_NOTPD
    plan.close()


def test_no_convergence_reported(oracle_lib):
    p = workloads.random_problem(4, 800, 2, 3, "product", 0.1)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
    alpha, _, info = plan.cg_solve(to_gpu(p.v), 0.01, rtol=1e-14, maxit=3, raise_on_error=False)
    assert info["status"] == "MM_ERR_NOCONV" and info["iters"] == 3
    assert np.all(np.isfinite(to_np(alpha)))
    plan.close()


def test_config2_full_solve_oracle_residual(oracle_lib):
    """Configuration 2's metric solve (N = 100,000, fixed effects, rtol 1e-8):
    the residual y - H beta - (K + sigma^2 I) alpha recomputed with the oracle's
    dense product over every row must meet rtol (Appendix A, Algorithm 2;
    Section 3.2), and the library's own recomputed residual must agree with it."""
    p = workloads.config2()
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
    alpha, beta, info = plan.cg_solve(to_gpu(p.y), 0.01, fixed_effects=True, rtol=1e-8, maxit=20000)
    a = to_np(alpha)
    say("config2 n=100000: iters %d, recurrence %.3e, library residual %.4e" %
        (info["iters"], info["relres_max"], info["true_relres"]))
    ka = oracle.mvm(p.x, a, 3, "product", 0.1)
    res = p.y - oracle.design_matrix(p.x) @ beta - ka - 0.01 * a
    rel_res = float(np.linalg.norm(res) / np.linalg.norm(p.y))
    say("oracle residual %.4e (oracle on %d threads)" % (rel_res, oracle.num_threads()))
    assert info["status"] == "MM_OK"
    assert rel_res <= 1e-8
    assert info["true_relres"] <= 1e-8
    # both evaluate the same residual; its rounding is ~eps ||K|alpha|| / (1e-8 ||y||)
    assert abs(info["true_relres"] - rel_res) <= 1e-3 * rel_res
    plan.close()


def test_check_mid_solve_restarts_and_converges(oracle_lib):
    """mm_solver_check on a solver that has not converged: its recomputed
    residual matches the oracle's for the current iterate, the solve restarts
    from it, and the continued solve still reaches the Cholesky solution."""
    n, d, ell, sig2 = 1500, 2, 0.15, 0.01
    p = workloads.random_problem(611, n, d, 3, "product", ell)
    y = workloads.field_sin_cos(p.x) + 0.1 * np.random.default_rng(2).standard_normal(n)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", ell))
    s = mm.Solver(plan, to_gpu(y), sig2, rtol=1e-12)
    s.iterate(7)
    passed, trel = s.check(tighten=True)
    alpha7, _, _ = s.finish(raise_on_error=False)
    a7 = to_np(alpha7)
    ref7 = np.linalg.norm(y - oracle.mvm(p.x, a7, 3, "product", ell) - sig2 * a7) / np.linalg.norm(y)
    say("after 7 iterations: library residual %.6e, oracle %.6e" % (trel, ref7))
    assert not passed
    assert abs(trel - ref7) <= 1e-6 * ref7
    for _ in range(4000):
        s.iterate(8)
        act, brk, _ = s.poll()
        assert brk == 0
        if act == 0 and s.check(tighten=True)[0]:
            break
    alpha, _, info = s.finish()
    ref = oracle.gp_solve(p.x, y, 3, "product", ell, 1.0, sig2)
    say("restarted solve: iters %d err %.2e residual %.2e" % (info["iters"], rel(to_np(alpha), ref),
                                                             info["true_relres"]))
    assert info["true_relres"] <= 1e-12
    assert rel(to_np(alpha), ref) <= SOLVE_TOL
    s.close()
    plan.close()
