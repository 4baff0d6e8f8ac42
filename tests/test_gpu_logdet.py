"""Stochastic log-determinant on the GPU (Appendix A, Algorithm 2 and eq.
approximationLogDet) against the oracle.

* Per probe, CG run to convergence makes the Lanczos quadrature equal the
  quadratic form z^T log(K + sigma^2 I) z of the dense eigendecomposition.
* The estimate over Rademacher probes equals log det within five standard
  deviations of the Hutchinson estimator (computed exactly from log(A)).
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
from gpu_util import say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,two_nu", [(1, 1), (2, 3), (3, 5)])
def test_logdet_quadratures_and_estimate(oracle_lib, d, two_nu):
    rng = np.random.default_rng(70 + d)
    n, ell, sig2, nprobes = 700, 0.2, 0.05, 16
    x = rng.uniform(0, 1, (n, d))
    Z = rng.choice([-1.0, 1.0], size=(n, nprobes))
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, "product", ell))
    est, quad, steps = plan.logdet(sig2, to_gpu(Z), steps=n, rtol=1e-11)
    A = oracle.kernel_matrix(x, two_nu, "product", ell, 1.0, sigma2=sig2)
    exact_q = oracle.quad_log_exact(A, Z)
    ld = oracle.logdet_exact(A)
    w, Q = np.linalg.eigh(A)
    logA = (Q * np.log(w)) @ Q.T
    sd = np.sqrt(2.0 * (np.sum(logA ** 2) - np.sum(np.diag(logA) ** 2)) / nprobes)
    say("d=%d nu=%d/2 steps %s est %.6f exact %.6f sd %.3f max quad err %.2e" %
        (d, two_nu, steps.tolist()[:4], est, ld, sd, np.max(np.abs(quad - exact_q) / np.abs(exact_q))))
    assert np.max(np.abs(quad - exact_q) / np.abs(exact_q)) <= 1e-6
    assert abs(est - np.mean(quad)) <= 1e-12 * abs(est)
    assert abs(est - ld) <= 5.0 * sd
    plan.close()


def test_logdet_fixed_steps_matches_oracle_lanczos(oracle_lib):
    """With a fixed small number of steps (no stop test) the GPU's Lanczos
    quadrature equals the oracle's CG-Lanczos quadrature of the same length."""
    rng = np.random.default_rng(8)
    n, steps = 500, 12
    x = rng.uniform(0, 1, (n, 2))
    Z = rng.standard_normal((n, 3))
    plan = mm.Plan(to_gpu(x), mm.Kernel(3, "product", 0.15))
    _, quad, msteps = plan.logdet(0.02, to_gpu(Z), steps=steps, rtol=0.0)
    A = oracle.kernel_matrix(x, 3, "product", 0.15, 1.0, sigma2=0.02)
    for i in range(3):
        al, be = oracle.cg_lanczos(A, Z[:, i], steps)
        q = oracle.logquad_from_cg(al, be, float(Z[:, i] @ Z[:, i]))
        assert msteps[i] == len(be) == steps
        assert abs(quad[i] - q) <= 1e-9 * abs(q)
    plan.close()


@pytest.mark.parametrize("d,two_nu", [(2, 3), (3, 5)])
def test_preconditioned_logdet_matches_oracle(oracle_lib, d, two_nu):
    """gp_logdet_pc (Appendix A, the preconditioned log-determinant): with the same
    standard normal draws and a fixed number of steps, each probe's term equals the
    oracle's dense PCG-Lanczos quadrature (the oracle's own pivoted Cholesky,
    whose pivots the GPU factor reproduces), log det P equals Sylvester's form,
    and run to convergence the estimate lies within five standard errors of the
    dense Cholesky log-determinant."""
    import torch
    rng = np.random.default_rng(90 + d)
    n, ell, sig2, rank, nprobes = 900, 0.2, 0.03, 24, 20
    x = rng.uniform(0, 1, (n, d))
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, "product", ell))
    pc = mm.Precond(plan, max_rank=rank)
    assert pc.info()[0] == rank
    G1 = rng.standard_normal((rank, nprobes))
    G2 = rng.standard_normal((n, nprobes))
    A = oracle.kernel_matrix(x, two_nu, "product", ell, 1.0, sigma2=sig2)
    L, _, _ = oracle.pivoted_cholesky(x, two_nu, "product", ell, 1.0, rank)
    steps = 10
    _, quad, msteps, ldp = plan.logdet_pc(sig2, pc, to_gpu(G1), to_gpu(G2), steps=steps, rtol=0.0)
    _, qref = oracle.logdet_pc_estimate(A, L, sig2, G1, G2, steps)
    err = np.max(np.abs(quad - qref) / np.abs(qref))
    say("pc logdet d=%d fixed %d steps: max term err %.2e, log det P %.6f" % (d, steps, err, ldp))
    assert np.all(msteps == steps)
    assert err <= 1e-8
    assert abs(ldp - oracle.logdet_lowrank_plus_noise(L, sig2)) <= 1e-10 * abs(ldp)
    est, quad, msteps, _ = plan.logdet_pc(sig2, pc, to_gpu(G1), to_gpu(G2), steps=n, rtol=1e-11)
    ld = oracle.logdet_exact(A)
    se = np.std(quad, ddof=1) / np.sqrt(nprobes)
    say("pc logdet d=%d converged: est %.6f exact %.6f se %.4f steps %s" % (d, est, ld, se, msteps.tolist()[:4]))
    assert abs(est - ld) <= 5.0 * se + 1e-9 * abs(ld)
    pc.close()
    plan.close()
