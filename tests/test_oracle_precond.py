"""Pins of the oracle's pivoted Cholesky and Woodbury preconditioner
(Appendix A, 'Preconditioning'), against properties fixed by the
mathematics rather than by re-typing the algorithm."""
import numpy as np
import pytest

import oracle


def _pts(n, d, seed=3):
    return np.random.default_rng(seed).uniform(0, 1, (n, d))


@pytest.mark.parametrize("d,two_nu", [(1, 1), (2, 3), (3, 5)])
def test_full_rank_reconstructs_K(oracle_lib, d, two_nu):
    x = _pts(40, d)
    K = oracle.kernel_matrix(x, two_nu, "product", 0.3, 1.3)
    L, piv, res = oracle.pivoted_cholesky(x, two_nu, "product", 0.3, 1.3, 40)
    assert L.shape == (40, 40) and sorted(piv.tolist()) == list(range(40))
    assert np.max(np.abs(L @ L.T - K)) <= 1e-12 * np.max(np.abs(K))
    assert res <= 1e-10
    # a Cholesky factor of K permuted to pivot order: lower triangular there
    Lp = L[piv]
    assert np.max(np.abs(np.triu(Lp, 1))) <= 1e-13
    assert np.allclose(Lp, np.linalg.cholesky(K[np.ix_(piv, piv)]), rtol=0, atol=1e-12)


def test_low_rank_is_exact_on_pivots_and_diagonal_residual(oracle_lib):
    x = _pts(80, 2, seed=5)
    K = oracle.kernel_matrix(x, 3, "product", 0.2, 1.0)
    L, piv, res = oracle.pivoted_cholesky(x, 3, "product", 0.2, 1.0, 12)
    A = L @ L.T
    # interpolation property: rows and columns of the pivots are reproduced exactly
    assert np.max(np.abs(A[piv] - K[piv])) <= 1e-12
    # the residual K - L L^T is positive semi-definite, its trace is the residual
    R = K - A
    assert np.min(np.linalg.eigvalsh(R)) >= -1e-12
    assert abs(np.trace(R) - res) <= 1e-10
    # greedy: pivots are the largest residual diagonals, first pivot the smallest index
    assert piv[0] == 0
    traces = [oracle.pivoted_cholesky(x, 3, "product", 0.2, 1.0, k)[2] for k in (2, 4, 8, 12)]
    assert all(a > b for a, b in zip(traces, traces[1:]))


def test_tolerance_stops_early(oracle_lib):
    x = _pts(60, 1, seed=7)
    L, piv, res = oracle.pivoted_cholesky(x, 5, "product", 0.5, 1.0, 60, tol=1e-6)
    assert L.shape[1] < 60
    assert res <= 1e-6 * 60


def test_woodbury_is_the_inverse_of_the_preconditioner(oracle_lib):
    x = _pts(50, 2, seed=9)
    L, _, _ = oracle.pivoted_cholesky(x, 3, "product", 0.3, 1.0, 10)
    s2 = 0.05
    P = L @ L.T + s2 * np.eye(50)
    r = np.random.default_rng(1).standard_normal((50, 3))
    z = oracle.woodbury_apply(L, s2, r)
    assert np.max(np.abs(P @ z - r)) <= 1e-10 * np.max(np.abs(r))
