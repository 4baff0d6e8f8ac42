"""Pins of the oracle's lengthscale derivative, log marginal likelihood and
posterior variance (Section 2.3 gradients, eq. gp_log_likelihood, eq.
gp_log_likelihood_derivative, Appendix A trace estimator, eq. gp_variance).

The derivative is checked against central finite differences of the oracle's
kernel matrix (its C code, an independent route to the same numbers); the
likelihood gradient against finite differences of the likelihood; the trace
estimator against the exact trace on a probe basis; the variance against its
one-point closed form and its limits.
"""
import numpy as np
import pytest

import oracle


def _fd_dell(x, two_nu, form, ell, s2, h_rel=1e-5):
    h = h_rel * ell
    Kp = oracle.kernel_matrix(x, two_nu, form, ell + h, s2)
    Km = oracle.kernel_matrix(x, two_nu, form, ell - h, s2)
    return (Kp - Km) / (2.0 * h)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("two_nu", [1, 3, 5])
@pytest.mark.parametrize("form", ["product", "l1"])
def test_derivative_matches_finite_differences(oracle_lib, d, two_nu, form):
    rng = np.random.default_rng(10 * d + two_nu)
    x = rng.uniform(0, 1, (40, d))
    ell, s2 = 0.3, 1.7
    D = oracle.dkernel_matrix_dell(x, two_nu, form, ell, s2)
    F = _fd_dell(x, two_nu, form, ell, s2)
    assert np.max(np.abs(D - F)) <= 1e-7 * np.max(np.abs(D))
    assert np.all(D >= 0.0)                      # correlations grow with the lengthscale
    assert np.all(np.diag(D) == 0.0)             # K_ii = s2 for every lengthscale
    assert np.allclose(D, D.T, rtol=0, atol=0)   # symmetric


def test_rectangular_derivative_matches_square(oracle_lib):
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (30, 2))
    z = rng.uniform(0, 1, (7, 2))
    D = oracle.dkernel_matrix_dell(np.vstack([x, z]), 5, "product", 0.2, 1.0)
    R = oracle.dkernel_matrix_dell(x, 5, "product", 0.2, 1.0, z=z)
    assert np.array_equal(R, D[30:, :30])


def test_one_dimensional_forms_agree(oracle_lib):
    # in one dimension the L1 and product forms are the same kernel
    x = np.random.default_rng(6).uniform(0, 1, (25, 1))
    for two_nu in (1, 3, 5):
        a = oracle.dkernel_matrix_dell(x, two_nu, "l1", 0.25, 1.0)
        b = oracle.dkernel_matrix_dell(x, two_nu, "product", 0.25, 1.0)
        assert np.allclose(a, b, rtol=1e-14, atol=0)


@pytest.mark.parametrize("d,two_nu", [(1, 1), (2, 3), (3, 5)])
def test_lml_gradient_matches_finite_differences(oracle_lib, d, two_nu):
    rng = np.random.default_rng(20 + d)
    x = rng.uniform(0, 1, (50, d))
    y = np.sin(3 * x.sum(axis=1)) + 0.1 * rng.standard_normal(50)
    ell, s2, sig = 0.4, 1.3, 0.05
    g = oracle.lml_grad_exact(x, y, two_nu, "product", ell, s2, sig)

    def f(e, a, b):
        return oracle.lml_exact(x, y, two_nu, "product", e, a, b)

    h = 1e-5
    fd = [(f(ell + h * ell, s2, sig) - f(ell - h * ell, s2, sig)) / (2 * h * ell),
          (f(ell, s2, sig + h * sig) - f(ell, s2, sig - h * sig)) / (2 * h * sig),
          (f(ell, s2 + h * s2, sig) - f(ell, s2 - h * s2, sig)) / (2 * h * s2)]
    for a, b in zip(g, fd):
        assert abs(a - b) <= 1e-6 * max(1.0, abs(b))


def test_lml_of_identity_covariance_closed_form(oracle_lib):
    # s2 -> 0: A = sigma2 I, L = -|y|^2/(2 sigma2) - n/2 log sigma2 - n/2 log 2 pi
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 1, (20, 2))
    y = rng.standard_normal(20)
    sig = 0.7
    v = oracle.lml_exact(x, y, 3, "product", 0.3, 1e-300, sig)
    ref = -0.5 * y @ y / sig - 10 * np.log(sig) - 10 * np.log(2 * np.pi)
    assert abs(v - ref) <= 1e-12 * abs(ref)


def test_hutchinson_on_a_probe_basis_is_the_trace(oracle_lib):
    rng = np.random.default_rng(9)
    n = 40
    x = rng.uniform(0, 1, (n, 2))
    A = oracle.kernel_matrix(x, 3, "product", 0.2, 1.0, sigma2=0.1)
    D = oracle.dkernel_matrix_dell(x, 3, "product", 0.2, 1.0)
    # probes sqrt(n) e_i: the mean of the terms is sum_i (A^-1 D)_ii exactly
    Z = np.sqrt(n) * np.eye(n)
    est = np.mean(oracle.hutchinson_terms(A, D, Z))
    exact = np.trace(np.linalg.solve(A, D))
    assert abs(est - exact) <= 1e-10 * abs(exact)
    # and Rademacher probes estimate it without bias (loose statistical check)
    R = rng.choice([-1.0, 1.0], size=(n, 4000))
    t = oracle.hutchinson_terms(A, D, R)
    assert abs(np.mean(t) - exact) <= 5 * np.std(t) / np.sqrt(t.size)


def test_posterior_variance_closed_forms(oracle_lib):
    rng = np.random.default_rng(11)
    s2, sig = 1.6, 0.03
    # one training point: var = s2 - k^2 / (s2 + sigma2)
    x1 = rng.uniform(0, 1, (1, 2))
    z = rng.uniform(0, 1, (5, 2))
    k = np.array([oracle.kernel(zz, x1[0], 3, "product", 0.3, s2) for zz in z])
    v = oracle.posterior_variance(x1, z, 3, "product", 0.3, s2, sig)
    assert np.allclose(v, s2 - k * k / (s2 + sig), rtol=1e-13, atol=0)
    # far from every training point the prior variance remains
    x = rng.uniform(0, 1, (30, 2))
    far = np.array([[50.0, 50.0]])
    assert abs(oracle.posterior_variance(x, far, 5, "product", 0.2, s2, sig)[0] - s2) <= 1e-15
    # at a training point the variance is below the noise level, and never negative
    vt = oracle.posterior_variance(x, x[:5], 1, "product", 0.2, s2, sig)
    assert np.all(vt > 0) and np.all(vt < sig)
