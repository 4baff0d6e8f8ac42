"""Host part of the stochastic log-determinant: the library's Lanczos
quadrature e_1^T log(T) e_1 against the oracle's (dense eigendecomposition),
no GPU needed."""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm


@pytest.mark.parametrize("m", [1, 2, 3, 7, 40, 150])
def test_quadrature_matches_dense_eigendecomposition(m):
    rng = np.random.default_rng(m)
    alpha = rng.uniform(0.05, 2.0, m)
    beta = rng.uniform(0.01, 0.9, m)
    q = mm.lanczos_logquad(alpha, beta[: m - 1])
    ref = oracle.logquad_from_cg(alpha, np.append(beta[: m - 1], 0.0) if m > 1 else np.array([0.0]), 1.0)
    assert abs(q - ref) <= 1e-12 * max(1.0, abs(ref))


def test_quadrature_of_cg_coefficients(oracle_lib):
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, (120, 2))
    A = oracle.kernel_matrix(x, 3, "product", 0.25, 1.0, sigma2=0.05)
    z = rng.choice([-1.0, 1.0], 120)
    al, be = oracle.cg_lanczos(A, z, 120, rtol=1e-13)
    m = len(be)
    q = mm.lanczos_logquad(al[:m], be[: m - 1]) * float(z @ z)
    exact = oracle.quad_log_exact(A, z)[0]
    assert abs(q - exact) <= 1e-6 * abs(exact)


def test_quadrature_refuses_a_non_positive_spectrum():
    """A Lanczos matrix with a non-positive eigenvalue (which a breakdown of CG
    would leave) has no logarithm: MM_ERR_BREAKDOWN."""
    with pytest.raises(mm.MaternError) as e:
        mm.lanczos_logquad(np.array([-1.0]), np.array([]))
    assert e.value.status == mm.MM_ERR_BREAKDOWN
    # T = [[1, 3], [3, 1]]: eigenvalues 4 and -2
    a0, b0 = 1.0, 9.0                      # T[0][1] = sqrt(b0) / a0 = 3
    a1 = 1.0 / (1.0 - b0 / a0)             # T[1][1] = 1/a1 + b0/a0 = 1
    with pytest.raises(mm.MaternError) as e:
        mm.lanczos_logquad(np.array([a0, a1]), np.array([b0]))
    assert e.value.status == mm.MM_ERR_BREAKDOWN
