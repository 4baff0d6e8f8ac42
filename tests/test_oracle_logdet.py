"""Pins of the oracle's Lanczos log-determinant quadrature (Appendix A,
Algorithm 2 and eq. approximationLogDet) against closed forms and dense
linear algebra."""
import numpy as np

import oracle


def test_scalar_matrix_closed_form():
    c = 3.7
    A = c * np.eye(30)
    z = np.random.default_rng(0).standard_normal(30)
    # CG solves c I exactly in one step (alpha = 1/c) and stops there; the
    # Lanczos matrix of that step is the 1x1 matrix [c] (its beta is zero)
    al, be = oracle.cg_lanczos(A, z, 10, rtol=1e-14)
    assert len(al) == 1 and len(be) == 0
    assert abs(al[0] - 1.0 / c) <= 1e-15
    q = oracle.logquad_from_cg(al, np.array([0.0]), float(z @ z))
    assert abs(q - np.log(c) * float(z @ z)) <= 1e-12 * abs(q)


def test_converged_quadrature_equals_quadratic_form(oracle_lib):
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (60, 2))
    A = oracle.kernel_matrix(x, 3, "product", 0.3, 1.0, sigma2=0.1)
    Z = rng.choice([-1.0, 1.0], size=(60, 4))
    exact = oracle.quad_log_exact(A, Z)
    for i in range(4):
        al, be = oracle.cg_lanczos(A, Z[:, i], 60)
        q = oracle.logquad_from_cg(al, be, float(Z[:, i] @ Z[:, i]))
        assert abs(q - exact[i]) <= 1e-6 * abs(exact[i])


def test_tridiagonal_spectrum_inside_matrix_spectrum(oracle_lib):
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (80, 1))
    A = oracle.kernel_matrix(x, 5, "product", 0.2, 1.0, sigma2=0.05)
    lam = np.linalg.eigvalsh(A)
    al, be = oracle.cg_lanczos(A, rng.standard_normal(80), 25)
    t = np.linalg.eigvalsh(oracle.lanczos_tridiagonal(al, be))
    assert t.min() >= lam.min() * (1 - 1e-9) and t.max() <= lam.max() * (1 + 1e-9)


def test_probe_basis_gives_exact_logdet(oracle_lib):
    """Summing z^T log(A) z over an orthonormal basis gives trace(log A) = log det A."""
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (40, 3))
    A = oracle.kernel_matrix(x, 1, "product", 0.4, 1.0, sigma2=0.2)
    q = oracle.quad_log_exact(A, np.eye(40)).sum()
    assert abs(q - oracle.logdet_exact(A)) <= 1e-10 * abs(q)
