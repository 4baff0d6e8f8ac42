"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests touches the GPU or the HIP library.  Each pin is chosen so
that a plausible mistake in the oracle (a dropped polynomial term, a wrong
sqrt(2 nu) factor, a transposed operand, a lost diagonal, a wrong form) fails
at least one of them:

* profiles vs the Bessel-function definition (eq. matern_general, SciPy's
  independent K_nu), vs the general explicit sum (eq. matern_explicit) and vs
  the coefficients printed in Appendix C (tests/golden);
* MVMs on 1-D grids and tensor grids vs geometric / arithmetico-geometric
  closed forms;
* the paper's weighted-ECDF decomposition (Props. 1-2, the Matern examples of
  Section 2.3) evaluated by brute-force masked sums vs the dense oracle, with
  ties and duplicated points;
* invariants: symmetry, translation, reflection, axis and point permutation,
  scaling, linearity, positivity, the diagonal and both lengthscale limits;
* compensated summation vs math.fsum;
* Cholesky / solve vs LAPACK, positive definiteness (and the documented
  indefiniteness of the L1 form at nu >= 3/2, d >= 2);
* GLS vs OLS in the vanishing-outputscale limit, the GLS normal equations and
  the posterior-mean identity at the training points.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import decomposition as dec
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NUS = (1, 3, 5)


def _eval_expr(tok: str) -> float:
    val = 1.0
    for fac in tok.strip().split("*"):
        fac = fac.strip()
        if fac.startswith("sqrt(") and fac.endswith(")"):
            val *= math.sqrt(float(Fraction(fac[5:-1])))
        else:
            val *= float(Fraction(fac))
    return val


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([c.strip() for c in line.split("|")])
    return rows


def _rel(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.asarray(scale)))


# --------------------------------------------------------------------------
# Profiles
# --------------------------------------------------------------------------

@pytest.mark.parametrize("two_nu", NUS)
def test_profile_matches_bessel_definition(oracle_lib, two_nu):
    """k_nu(r) = (sqrt(2nu) r)^nu / (2^(nu-1) Gamma(nu)) K_nu(sqrt(2nu) r) (eq. matern_general)."""
    nu = two_nu / 2.0
    r = np.linspace(1e-3, 6.0, 400)
    t = np.sqrt(2 * nu) * r
    ref = t ** nu / (2 ** (nu - 1) * sp.gamma(nu)) * sp.kv(nu, t)
    got = oracle.profile(two_nu, r)
    assert np.max(np.abs(got - ref)) < 1e-13
    assert oracle.profile(two_nu, np.array([0.0]))[0] == 1.0


@pytest.mark.parametrize("p", [0, 1, 2])
def test_profile_matches_explicit_sum(oracle_lib, p):
    """eq. matern_explicit: sum_i p!/(i!(p-i)!) (2p-i)!/(2p)! (2 sqrt(2p+1) u)^i exp(-sqrt(2p+1) u)."""
    u = np.linspace(0.0, 8.0, 300)
    s = math.sqrt(2 * p + 1)
    poly = sum(math.comb(p, i) * math.factorial(2 * p - i) / math.factorial(2 * p)
               * (2 * s * u) ** i for i in range(p + 1))
    ref = poly * np.exp(-s * u)
    assert np.max(np.abs(oracle.profile(2 * p + 1, u) - ref)) < 1e-14


def test_profile_matches_printed_coefficients(oracle_lib):
    """Appendix C printed profiles (tests/golden/matern_profiles.txt)."""
    u = np.linspace(0.0, 5.0, 101)
    seen = 0
    for two_nu, rate, coefs in _read_golden("matern_profiles.txt"):
        two_nu = int(two_nu)
        c = [_eval_expr(t) for t in coefs.split(",")]
        ref = sum(ci * u ** i for i, ci in enumerate(c)) * np.exp(-_eval_expr(rate) * u)
        if two_nu in NUS:
            assert np.max(np.abs(oracle.profile(two_nu, u) - ref)) < 1e-14
            seen += 1
        # the printed higher-order profiles must agree with the general explicit sum too
        p = (two_nu - 1) // 2
        s = math.sqrt(2 * p + 1)
        poly = sum(math.comb(p, i) * math.factorial(2 * p - i) / math.factorial(2 * p)
                   * (2 * s * u) ** i for i in range(p + 1))
        assert np.max(np.abs(poly * np.exp(-s * u) - ref)) < 1e-13
    assert seen == 3


def test_printed_bessel_closed_forms_match_scipy():
    """Appendix C K_{n+1/2} closed forms (tests/golden/bessel_half_integer.txt) vs SciPy."""
    u = np.linspace(0.05, 10.0, 200)
    for two_nu, coefs in _read_golden("bessel_half_integer.txt"):
        nu = int(two_nu) / 2.0
        b = [_eval_expr(t) for t in coefs.split(",")]
        ref = math.sqrt(math.pi / 2) * np.exp(-u) * sum(bi * u ** i for i, bi in enumerate(b)) / u ** nu
        assert np.max(np.abs(sp.kv(nu, u) - ref) / ref) < 1e-12


# --------------------------------------------------------------------------
# Closed-form MVMs on grids
# --------------------------------------------------------------------------

def _geo_sums(rho, m):
    """S0, S1, S2 = sum_{k=0}^{m} k^q rho^k in closed form (vectorised over m)."""
    m = np.asarray(m, dtype=np.float64)
    S0 = (1 - rho ** (m + 1)) / (1 - rho)
    S1 = rho * (1 - (m + 1) * rho ** m + m * rho ** (m + 1)) / (1 - rho) ** 2
    S2 = rho * (1 + rho - (m + 1) ** 2 * rho ** m + (2 * m * m + 2 * m - 1) * rho ** (m + 1)
                - m * m * rho ** (m + 2)) / (1 - rho) ** 3
    return S0, S1, S2


def _grid_row_sums(n, h, ell, two_nu):
    """(K 1)_j on the 1-D grid x_i = i h with the unit-outputscale profile, in closed form."""
    c = math.sqrt(two_nu) * h / ell
    rho = math.exp(-c)
    j = np.arange(n)
    A0, A1, A2 = _geo_sums(rho, j)
    B0, B1, B2 = _geo_sums(rho, n - 1 - j)
    out = A0 + B0 - 1.0
    if two_nu >= 3:
        out = out + c * (A1 + B1)
    if two_nu == 5:
        out = out + c * c / 3.0 * (A2 + B2)
    return out


@pytest.mark.parametrize("two_nu", NUS)
def test_mvm_1d_grid_closed_form(oracle_lib, two_nu):
    n, h, ell, s2 = 300, 0.01, 0.05, 1.7
    x = (np.arange(n) * h)[:, None]
    y = oracle.mvm(x, np.ones(n), two_nu, "l1", ell, s2)
    ref = s2 * _grid_row_sums(n, h, ell, two_nu)
    assert _rel(y, ref, ref) < 1e-12


@pytest.mark.parametrize("two_nu", NUS)
@pytest.mark.parametrize("d", [2, 3])
def test_mvm_tensor_grid_product_closed_form(oracle_lib, two_nu, d):
    """Product form on a tensor grid with v = 1 factorises into 1-D closed forms."""
    sizes = [7, 5, 4][:d]
    hs = [0.03, 0.05, 0.02][:d]
    ell = 0.07
    axes = [np.arange(s) * h for s, h in zip(sizes, hs)]
    mesh = np.meshgrid(*axes, indexing="ij")
    x = np.column_stack([m.ravel() for m in mesh])
    y = oracle.mvm(x, np.ones(x.shape[0]), two_nu, "product", ell, 1.0)
    ref = np.ones_like(y)
    idx = np.meshgrid(*[np.arange(s) for s in sizes], indexing="ij")
    for k in range(d):
        rows = _grid_row_sums(sizes[k], hs[k], ell, two_nu)
        ref = ref * rows[idx[k].ravel()]
    assert _rel(y, ref, ref) < 1e-12


@pytest.mark.parametrize("d", [1, 2, 3])
def test_l1_and_product_coincide_at_nu_half(oracle_lib, d):
    """eq. matern_l1_12 remark: the two multivariate forms coincide for nu = 1/2."""
    p = workloads.random_problem(7 + d, 250, d, 1, "l1", 0.2)
    a = oracle.mvm(p.x, p.v, 1, "l1", p.ell, 1.3)
    b = oracle.mvm(p.x, p.v, 1, "product", p.ell, 1.3)
    _, s = oracle.mvm(p.x, p.v, 1, "l1", p.ell, 1.3, with_abs=True)
    assert _rel(a, b, s) < 1e-14


def test_l1_and_product_differ_at_nu_three_halves(oracle_lib):
    p = workloads.random_problem(3, 100, 2, 3, "l1", 0.3)
    a = oracle.mvm(p.x, p.v, 3, "l1", p.ell)
    b = oracle.mvm(p.x, p.v, 3, "product", p.ell)
    assert np.max(np.abs(a - b)) > 1e-3


# --------------------------------------------------------------------------
# The paper's decomposition, by brute-force masked ECDF sums
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("two_nu", NUS)
@pytest.mark.parametrize("ties", [False, True])
def test_l1_decomposition_matches_dense(oracle_lib, d, two_nu, ties):
    p = workloads.random_problem(100 + 10 * d + two_nu + (5 if ties else 0), 90, d, two_nu,
                                 "l1", 0.6, nrhs=2, ties=ties)
    dense, s = oracle.mvm(p.x, p.v, two_nu, "l1", p.ell, 0.8, with_abs=True)
    assert _rel(dec.matern_l1(p.x, p.v, two_nu, p.ell, 0.8), dense, s) < 1e-11
    assert _rel(dec.prop1_l1(p.x, p.v, two_nu, p.ell, 0.8), dense, s) < 1e-11


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("two_nu", NUS)
@pytest.mark.parametrize("ties", [False, True])
def test_product_decomposition_matches_dense(oracle_lib, d, two_nu, ties):
    p = workloads.random_problem(200 + 10 * d + two_nu + (5 if ties else 0), 80, d, two_nu,
                                 "product", 0.6, ties=ties)
    dense, s = oracle.mvm(p.x, p.v, two_nu, "product", p.ell, 1.1, with_abs=True)
    assert _rel(dec.prop2_product(p.x, p.v, two_nu, p.ell, 1.1), dense, s) < 1e-11
    if two_nu == 3:
        assert _rel(dec.matern_product_32(p.x, p.v, p.ell, 1.1), dense, s) < 1e-11


def test_decomposition_rectangular_targets(oracle_lib):
    """Targets distinct from the sources (the predict case)."""
    p = workloads.random_problem(5, 70, 2, 5, "l1", 0.5)
    z = np.random.default_rng(9).uniform(0, 1, size=(40, 2))
    dense, s = oracle.mvm(p.x, p.v, 5, "l1", p.ell, z=z, with_abs=True)
    assert _rel(dec.matern_l1(p.x, p.v, 5, p.ell, z=z), dense, s) < 1e-11
    dense, s = oracle.mvm(p.x, p.v, 5, "product", p.ell, z=z, with_abs=True)
    assert _rel(dec.prop2_product(p.x, p.v, 5, p.ell, z=z), dense, s) < 1e-11


def test_product_32_literal_reading_fails(oracle_lib):
    """The literal printed pi weights (a product of theta_k factors) do not reproduce
    the kernel sum; this documents why the oracle takes the coordinate-subset reading."""
    p = workloads.random_problem(11, 40, 2, 3, "product", 0.5)
    x, v, a = p.x, p.v, math.sqrt(3.0) / p.ell
    out = 0.0
    import itertools
    for theta in itertools.product((0, 1), repeat=2):
        for delta in itertools.product((-1.0, 1.0), repeat=2):
            delta = np.array(delta)
            dz = dx = x * delta
            pi0 = np.prod([theta[k] * (1 + a * dz[:, k]) for k in range(2)], axis=0)
            pi1 = np.prod([(1 - theta[k]) * (-a * dx[:, k]) for k in range(2)], axis=0)
            w = v * pi1 * np.exp(a * dx.sum(axis=1))
            out = out + pi0 * np.exp(-a * dz.sum(axis=1)) * dec.ecdf(dz, delta, dx, w)
    dense = oracle.mvm(x, v, 3, "product", p.ell)
    assert np.max(np.abs(out - dense)) > 1e-3


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("form", ["l1", "product"])
@pytest.mark.parametrize("two_nu", NUS)
def test_invariants(oracle_lib, form, two_nu):
    rng = np.random.default_rng(42 + two_nu)
    n, d, ell, s2 = 150, 3, 0.25, 1.4
    x = rng.uniform(0, 1, size=(n, d))
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    y, s = oracle.mvm(x, v, two_nu, form, ell, s2, with_abs=True)
    tol = 1e-13

    # symmetry u^T (K v) = v^T (K u)
    ku = oracle.mvm(x, u, two_nu, form, ell, s2)
    assert abs(u @ y - v @ ku) <= 1e-12 * (np.abs(u) @ s)
    # translation
    assert _rel(oracle.mvm(x + np.array([3.0, -1.5, 0.25]), v, two_nu, form, ell, s2), y, s) < tol
    # reflection of each coordinate (exercises every orthant)
    for k in range(d):
        xr = x.copy()
        xr[:, k] = -xr[:, k]
        assert _rel(oracle.mvm(xr, v, two_nu, form, ell, s2), y, s) < tol
    # axis permutation
    assert _rel(oracle.mvm(x[:, [2, 0, 1]], v, two_nu, form, ell, s2), y, s) < tol
    # point permutation equivariance
    perm = rng.permutation(n)
    assert _rel(oracle.mvm(x[perm], v[perm], two_nu, form, ell, s2), y[perm], s[perm]) < tol
    # scaling (x, ell) -> (c x, c ell)
    assert _rel(oracle.mvm(3.5 * x, v, two_nu, form, 3.5 * ell, s2), y, s) < 1e-12
    # linearity
    y2 = oracle.mvm(x, 2.0 * v - 0.5 * u, two_nu, form, ell, s2)
    assert _rel(y2, 2.0 * y - 0.5 * ku, 2 * s + 0.5 * oracle.mvm(x, u, two_nu, form, ell, s2, with_abs=True)[1]) < 1e-13
    # positivity: K v >= 0 for v >= 0
    assert np.all(oracle.mvm(x, np.abs(v), two_nu, form, ell, s2) >= 0.0)
    # diagonal: (K e_j)_j = s2
    e = np.zeros(n)
    e[17] = 1.0
    assert oracle.mvm(x, e, two_nu, form, ell, s2)[17] == s2
    # ell -> 0: y -> s2 v ; ell -> infinity: y -> s2 sum(v)
    assert _rel(oracle.mvm(x, v, two_nu, form, 1e-9, s2), s2 * v, np.abs(v) + 1e-300) < 1e-12
    big = oracle.mvm(x, v, two_nu, form, 1e9, s2)
    assert np.max(np.abs(big - s2 * v.sum())) < 1e-6 * s2 * np.abs(v).sum()


def test_multi_rhs_entry_matches_single(oracle_lib):
    p = workloads.random_problem(77, 120, 2, 5, "product", 0.3, nrhs=5)
    a = oracle.mvm(p.x, p.v, 5, "product", p.ell)
    b = oracle.mvm(p.x, p.v, 5, "product", p.ell, shared_kernel=True)
    assert np.array_equal(a, b)
    for r in range(5):
        assert np.array_equal(a[:, r], oracle.mvm(p.x, p.v[:, r], 5, "product", p.ell))


# --------------------------------------------------------------------------
# Compensated summation
# --------------------------------------------------------------------------

def test_compensated_rows_match_fsum(oracle_lib):
    rng = np.random.default_rng(5)
    n = 400
    x = rng.uniform(0, 1, size=(n, 2))
    v = rng.standard_normal(n) * 10.0 ** rng.uniform(-8, 8, size=n)
    K = oracle.kernel_matrix(x, 3, "product", 0.4)
    y = oracle.mvm(x, v, 3, "product", 0.4)
    for j in range(0, n, 37):
        exact = math.fsum(K[j, :] * v)
        assert abs(y[j] - exact) <= 2.5e-16 * abs(exact) + 1e-30 * np.sum(np.abs(K[j] * v))


def test_compensation_survives_cancellation(oracle_lib):
    """A naive running sum loses the small terms here; the compensated one does not."""
    x = np.array([[0.0], [1e-3], [2e-3], [3e-3]])
    v = np.array([1e17, 1.0, -1e17, 1.0])
    y = oracle.mvm(x, v, 1, "l1", 1e12)
    K = oracle.kernel_matrix(x, 1, "l1", 1e12)
    for j in range(4):
        assert y[j] == math.fsum(K[j] * v)


# --------------------------------------------------------------------------
# Cholesky, positive definiteness, solve, GLS, predict
# --------------------------------------------------------------------------

def test_cholesky_and_solve_match_lapack(oracle_lib):
    p = workloads.random_problem(3, 300, 2, 3, "product", 0.2)
    A = oracle.kernel_matrix(p.x, 3, "product", p.ell, 1.0, sigma2=0.05)
    L = oracle.cholesky(A)
    assert np.max(np.abs(L - np.linalg.cholesky(A))) < 1e-12
    b = np.random.default_rng(1).standard_normal((300, 3))
    xs = oracle.cholesky_solve(L, b)
    ref = np.linalg.solve(A, b)
    assert np.max(np.abs(xs - ref)) / np.max(np.abs(ref)) < 1e-10


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("two_nu", NUS)
def test_product_form_is_positive_definite(oracle_lib, d, two_nu):
    p = workloads.random_problem(31 + d, 400, d, two_nu, "product", 0.3)
    A = oracle.kernel_matrix(p.x, two_nu, "product", p.ell, 1.0, sigma2=1e-8)
    oracle.cholesky(A)


def test_l1_form_is_indefinite_for_nu_three_halves_in_2d(oracle_lib):
    """Documented expectation: the L1 Matern-3/2 matrix has negative eigenvalues at the
    2-D, ell = 0.1 parameters (its sufficient PD condition in Appendix B fails)."""
    p = workloads.config2(n=1500)
    K = oracle.kernel_matrix(p.x, 3, "l1", 0.1)
    assert np.linalg.eigvalsh(K)[0] < -1e-3
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.cholesky(K + 0.01 * np.eye(K.shape[0]))
    Kp = oracle.kernel_matrix(p.x, 3, "product", 0.1)
    assert np.linalg.eigvalsh(Kp)[0] > -1e-10


def test_gp_solve_residual(oracle_lib):
    p = workloads.config2(n=1200)
    alpha = oracle.gp_solve(p.x, p.y, 3, "product", 0.1, 1.0, 0.01)
    r = oracle.mvm(p.x, alpha, 3, "product", 0.1) + 0.01 * alpha - p.y
    assert np.linalg.norm(r) / np.linalg.norm(p.y) < 1e-10


def test_gls_normal_equations_and_limits(oracle_lib):
    rng = np.random.default_rng(8)
    n, d = 400, 2
    x = rng.uniform(0, 1, size=(n, d))
    beta_true = np.array([0.7, -1.2, 2.0])
    y = oracle.design_matrix(x) @ beta_true + np.sin(6 * x[:, 0]) + 0.1 * rng.standard_normal(n)
    beta, alpha = oracle.gls(x, y, 3, "product", 0.2, 1.0, 0.05)
    H = oracle.design_matrix(x)
    # H^T alpha = 0: the GLS normal equations
    assert np.max(np.abs(H.T @ alpha)) < 1e-9 * np.linalg.norm(y)
    # alpha solves (K + s I) alpha = y - H beta
    r = oracle.mvm(x, alpha, 3, "product", 0.2) + 0.05 * alpha - (y - H @ beta)
    assert np.linalg.norm(r) < 1e-9 * np.linalg.norm(y)
    # vanishing outputscale: GLS -> OLS
    b0, _ = oracle.gls(x, y, 3, "product", 0.2, 1e-12, 0.05)
    assert np.max(np.abs(b0 - oracle.ols(x, y))) < 1e-9
    # exact affine data: GLS recovers beta, alpha = 0
    be, ae = oracle.gls(x, H @ beta_true, 3, "product", 0.2, 1.0, 0.05)
    assert np.max(np.abs(be - beta_true)) < 1e-9 and np.max(np.abs(ae)) < 1e-9


def test_predict_identity_at_training_points(oracle_lib):
    """At z = x: H beta + K alpha = y - sigma^2 alpha (eq. gp_mean with the GLS beta)."""
    rng = np.random.default_rng(12)
    n, d, s2n = 300, 3, 0.02
    x = rng.uniform(0, 1, size=(n, d))
    y = x @ np.array([1.0, -2.0, 0.5]) + np.cos(4 * x[:, 1]) + 0.1 * rng.standard_normal(n)
    beta, alpha = oracle.gls(x, y, 5, "product", 0.3, 1.0, s2n)
    mean = oracle.predict(x, alpha, x, 5, "product", 0.3, 1.0, beta=beta)
    assert np.max(np.abs(mean - (y - s2n * alpha))) < 1e-9
