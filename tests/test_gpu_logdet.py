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
