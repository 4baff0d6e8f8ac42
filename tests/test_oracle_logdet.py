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


# ---- the preconditioned variant (Appendix A, preconditioned log-determinant) ----

def _kmat(seed, n, d, two_nu, ell, sig2):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, d))
    K = oracle.kernel_matrix(x, two_nu, "product", ell, 1.0)
    return x, K, K + sig2 * np.eye(n)


def test_sylvester_logdet_of_the_preconditioner(oracle_lib):
    x, K, _ = _kmat(11, 70, 2, 3, 0.3, 0.05)
    L, _, _ = oracle.pivoted_cholesky(x, 3, "product", 0.3, 1.0, 12)
    P = L @ L.T + 0.05 * np.eye(70)
    sign, ref = np.linalg.slogdet(P)
    assert sign > 0
    assert abs(oracle.logdet_lowrank_plus_noise(L, 0.05) - ref) <= 1e-10 * abs(ref)


def test_pcg_lanczos_without_preconditioner_is_cg(oracle_lib):
    _, _, A = _kmat(12, 50, 1, 5, 0.2, 0.1)
    b = np.random.default_rng(13).standard_normal(50)
    a1, b1 = oracle.cg_lanczos(A, b, 12)
    a2, b2, rz0 = oracle.pcg_lanczos(A, b, lambda r: r, 12)
    assert np.allclose(a1, a2, rtol=1e-13, atol=0) and np.allclose(b1, b2, rtol=1e-13, atol=0)
    assert abs(rz0 - b @ b) <= 1e-14 * (b @ b)


def test_converged_preconditioned_quadrature(oracle_lib):
    """Run to convergence, (b^T P^-1 b) e_1^T log(T) e_1 equals
    u^T log(P^{-1/2} A P^{-1/2}) u with u = P^{-1/2} b (dense eigendecompositions)."""
    x, K, A = _kmat(14, 60, 2, 3, 0.3, 0.05)
    L, _, _ = oracle.pivoted_cholesky(x, 3, "product", 0.3, 1.0, 10)
    P = L @ L.T + 0.05 * np.eye(60)
    wp, Qp = np.linalg.eigh(P)
    Ph = Qp @ np.diag(wp ** -0.5) @ Qp.T           # P^{-1/2}
    B = Ph @ A @ Ph
    b = np.random.default_rng(15).standard_normal(60)
    u = Ph @ b
    exact = oracle.quad_log_exact(B, u)[0]
    al, be, rz0 = oracle.pcg_lanczos(A, b, lambda r: oracle.woodbury_apply(L, 0.05, r), 60)
    q = oracle.logquad_from_cg(al, be, rz0)
    assert abs(rz0 - u @ u) <= 1e-10 * (u @ u)
    assert abs(q - exact) <= 1e-6 * abs(exact)


def test_preconditioned_estimate_is_unbiased_on_a_small_problem(oracle_lib):
    """The mean over many N(0, P) probes approaches log det A within a few
    standard errors; an exact preconditioner (P = A) makes every term vanish."""
    x, K, A = _kmat(16, 80, 2, 3, 0.3, 0.05)
    L, _, _ = oracle.pivoted_cholesky(x, 3, "product", 0.3, 1.0, 15)
    rng = np.random.default_rng(17)
    G1 = rng.standard_normal((L.shape[1], 400))
    G2 = rng.standard_normal((80, 400))
    est, q = oracle.logdet_pc_estimate(A, L, 0.05, G1, G2, 80)
    ref = oracle.logdet_exact(A)
    se = np.std(q, ddof=1) / np.sqrt(len(q))
    assert abs(est - ref) <= 5 * se + 1e-9 * abs(ref)
    # full rank: P = K + sigma^2 I = A, the quadratures are log(1) = 0
    Lf, _, _ = oracle.pivoted_cholesky(x, 3, "product", 0.3, 1.0, 80)
    est_f, q_f = oracle.logdet_pc_estimate(A, Lf, 0.05, rng.standard_normal((Lf.shape[1], 3)),
                                           rng.standard_normal((80, 3)), 10)
    assert np.max(np.abs(q_f)) <= 1e-6 * 80
    assert abs(est_f - ref) <= 1e-6 * abs(ref)
