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
