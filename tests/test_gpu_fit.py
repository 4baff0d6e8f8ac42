"""Hyperparameter ascent on the GPU likelihood gradient (Section 3 ADAM and
Algorithm 1) against the dense optimum.

Data are drawn from the GP itself (the oracle's Cholesky factor of
K + sigma^2 I), so the likelihood has a well-defined maximum.  The ascent
uses stochastic gradients (Hutchinson traces), so it reaches a neighbourhood
of the maximiser: the test asks for the exact likelihood to rise, for the
fitted parameters to lie close to the dense maximiser, and for the exact
gradient there to be a small fraction of the starting one.
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
from paper_2508_01864_amd import fit
from gpu_util import say, to_gpu

pytestmark = pytest.mark.gpu


def _gp_data(seed, n, d, two_nu, ell, s2, sig):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, d))
    A = oracle.kernel_matrix(x, two_nu, "product", ell, s2, sigma2=sig)
    y = oracle.cholesky(A) @ rng.standard_normal(n)
    Z = rng.choice([-1.0, 1.0], size=(n, 31))
    return x, y, Z


def _dense_optimum(x, y, two_nu, start):
    from scipy.optimize import minimize

    def f(t):
        ell, s2, sig = np.exp(t)
        v = oracle.lml_exact(x, y, two_nu, "product", ell, s2, sig)
        g = oracle.lml_grad_exact(x, y, two_nu, "product", ell, s2, sig)
        return -v, -np.array(g) * np.exp(t)

    r = minimize(f, np.log(start), jac=True, method="L-BFGS-B")
    return np.exp(r.x)


def test_ascent_reaches_the_dense_maximiser(oracle_lib):
    n, two_nu = 1200, 1
    truth = (0.1054, 1.0, 0.3)                          # lengthscale, outputscale2, sigma2
    x, y, Z = _gp_data(31, n, 1, two_nu, *truth)
    start = (1.0, 0.25, 0.5)                            # the paper's start: l = 1, varsigma = 0.5
    opt = _dense_optimum(x, y, two_nu, truth)
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, "product", start[0], start[1]))
    res = fit.gradient_ascent(plan, to_gpu(y), start[2], to_gpu(Z), lr0=0.05, lr1=0.005, max_iter=600,
                              grad_tol=1e-6, param_tol=0.0, rtol=1e-7, maxit=n)
    plan.close()
    got = np.array([res.lengthscale, res.outputscale2, res.sigma2])
    say("ascent: %d iters (%s), fit %s, dense optimum %s" % (res.iters, res.stopped, got, opt))
    l0 = oracle.lml_exact(x, y, two_nu, "product", *start)
    l1 = oracle.lml_exact(x, y, two_nu, "product", *got)
    lopt = oracle.lml_exact(x, y, two_nu, "product", *opt)
    say("exact lml: start %.4f fit %.4f optimum %.4f" % (l0, l1, lopt))
    assert l1 > l0 + 0.9 * (lopt - l0)                  # most of the possible rise
    assert np.max(np.abs(np.log(got / opt))) <= 0.15
    g0 = np.array(oracle.lml_grad_exact(x, y, two_nu, "product", *start))
    g1 = np.array(oracle.lml_grad_exact(x, y, two_nu, "product", *got))
    assert np.linalg.norm(g1 * got) <= 0.05 * np.linalg.norm(g0 * np.array(start))


def test_algorithm1_fixed_effects_round_trip(oracle_lib):
    n, two_nu = 900, 3
    rng = np.random.default_rng(33)
    x, y0, Z = _gp_data(34, n, 2, two_nu, 0.2, 1.0, 0.05)
    beta_true = np.array([2.0, -1.0, 0.5])
    y = y0 + oracle.design_matrix(x) @ beta_true
    res = fit.algorithm1(to_gpu(x), to_gpu(y), mm.Kernel(two_nu, "product", 0.5, 0.5), 0.2, to_gpu(Z),
                         eps_beta=1e-2, max_rounds=4, lr0=0.05, lr1=0.005, max_iter=300, grad_tol=1e-6,
                         param_tol=0.0, rtol=1e-7, maxit=n)
    say("algorithm 1: rounds %d l %.4f s2 %.4f sigma2 %.4f beta %s" %
        (res.rounds, res.lengthscale, res.outputscale2, res.sigma2, res.beta))
    # the returned beta is the GLS estimate at the fitted parameters
    bref, _ = oracle.gls(x, y, two_nu, "product", res.lengthscale, res.outputscale2, res.sigma2)
    assert np.max(np.abs(res.beta - bref)) <= 1e-3 * max(1.0, np.max(np.abs(bref)))
    assert all(np.isfinite([res.lengthscale, res.outputscale2, res.sigma2]))
    assert res.sigma2 > 0 and res.lengthscale > 0 and res.outputscale2 > 0
