"""GPU parity of the lengthscale-derivative product and the log marginal
likelihood with its gradient (Section 2.3 gradients, eq. gp_log_likelihood,
eq. gp_log_likelihood_derivative, Appendix A) against the dense oracle.

* The derivative product: every component's error relative to
  ((dK/dl)|v|)_j, and the normwise error, <= 1e-10 (every entry of dK/dl is
  non-negative, so that row sum is the natural scale).
* The likelihood: with the probes run to convergence, each estimated term
  equals the oracle's estimator on the same probes (dense solves) to the CG
  tolerance; the estimates lie within five standard errors of the exact
  gradient.
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
import workloads
from gpu_util import MVM_TOL, mvm_errors, say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def dl_case(x, v, two_nu, form, ell, s2=1.0, rows=None):
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, form, ell, s2))
    y = to_np(plan.mvm_dlengthscale(to_gpu(v)))
    plan.close()
    z = None if rows is None else x[rows]
    yref, yabs = oracle.mvm_dell(x, v, two_nu, form, ell, s2, z=z)
    if rows is not None:
        y = y[rows]
    return mvm_errors(y, yref, yabs)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("two_nu", [1, 3, 5])
@pytest.mark.parametrize("form", ["l1", "product"])
def test_dlengthscale_tiny_with_ties(oracle_lib, d, two_nu, form):
    for n in (1, 2, 3, 5, 8, 17, 33, 64):
        for ties in (False, True):
            p = workloads.random_problem(7000 + 1000 * d + 10 * two_nu + n + (500 if ties else 0), n, d,
                                         two_nu, form, 0.4, ties=ties)
            say("dl tiny d=%d nu=%d/2 %s n=%d ties=%s" % (d, two_nu, form, n, ties))
            comp, nrm = dl_case(p.x, p.v, two_nu, form, p.ell, s2=1.3)
            assert comp <= MVM_TOL and nrm <= MVM_TOL, (n, ties, comp, nrm)


# d = 1 has one form (the two coincide), so it is listed once
DL_TILE_CASES = [(d, n, form) for d, n in [(1, 5000), (2, 3000), (2, 5001), (3, 2500)]
                 for form in (["product"] if d == 1 else ["l1", "product"])]


@pytest.mark.parametrize("d,n,form", DL_TILE_CASES)
@pytest.mark.parametrize("two_nu", [1, 3, 5])
def test_dlengthscale_several_tiles(oracle_lib, d, n, two_nu, form):
    p = workloads.random_problem(8000 + n + two_nu, n, d, two_nu, form, 0.05 if d < 3 else 0.15)
    say("dl tiles d=%d n=%d nu=%d/2 %s" % (d, n, two_nu, form))
    comp, nrm = dl_case(p.x, p.v, two_nu, form, p.ell)
    say("  comp %.2e nrm %.2e" % (comp, nrm))
    assert comp <= MVM_TOL and nrm <= MVM_TOL


@pytest.mark.parametrize("nrhs", [2, 3, 5, 33])
def test_dlengthscale_columns(oracle_lib, nrhs):
    p = workloads.random_problem(9100 + nrhs, 1500, 2, 5, "product", 0.1, nrhs=nrhs)
    comp, nrm = dl_case(p.x, p.v, 5, "product", p.ell, s2=0.8)
    say("dl nrhs=%d comp %.2e nrm %.2e" % (nrhs, comp, nrm))
    assert comp <= MVM_TOL and nrm <= MVM_TOL


@pytest.mark.parametrize("d,n,two_nu,nrows", [(2, 100_000, 3, 150), (3, 100_000, 5, 40)])
def test_dlengthscale_full_size_sampled_rows(oracle_lib, d, n, two_nu, nrows):
    """The headline size (d = 2, N = 100k, nu = 3/2) and a d = 3 one, four columns,
    on sampled rows the oracle computes one by one."""
    rng = np.random.default_rng(9200 + d)
    x = rng.uniform(0, 1, (n, d))
    v = rng.standard_normal((n, 4))
    rows = rng.choice(n, nrows, replace=False)
    comp, nrm = dl_case(x, v, two_nu, "product", 0.1 if d == 2 else 0.2, rows=rows)
    say("dl full d=%d comp %.2e nrm %.2e" % (d, comp, nrm))
    assert comp <= MVM_TOL and nrm <= MVM_TOL


def _lml_problem(seed, n, d, two_nu, nprobes):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, d))
    y = np.sin(2 * np.pi * x[:, 0]) * np.cos(np.pi * x[:, -1]) + 0.1 * rng.standard_normal(n)
    Z = rng.choice([-1.0, 1.0], size=(n, nprobes))
    return x, y, Z


@pytest.mark.parametrize("d,two_nu", [(1, 1), (2, 3), (3, 5)])
def test_lml_terms_match_oracle_estimator(oracle_lib, d, two_nu):
    n, ell, s2, sig, l = 700, 0.2, 1.4, 0.05, 15
    x, y, Z = _lml_problem(9300 + d, n, d, two_nu, l)
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, "product", ell, s2))
    out, alpha = plan.lml(to_gpu(y), sig, to_gpu(Z), maxit=n, rtol=1e-11, want_alpha=True)
    plan.close()
    K = oracle.kernel_matrix(x, two_nu, "product", ell, s2)
    A = K + sig * np.eye(n)
    D = oracle.dkernel_matrix_dell(x, two_nu, "product", ell, s2)
    a = oracle.cholesky_solve(oracle.cholesky(A), y)
    t_inv = oracle.hutchinson_terms(A, np.eye(n), Z)
    t_dk = oracle.hutchinson_terms(A, D, Z)
    t_k = oracle.hutchinson_terms(A, K, Z)
    q_ld = oracle.quad_log_exact(A, Z)
    say("lml d=%d iters %d: quad %.10e / %.10e  logdet %.8e / %.8e  trdk %.8e / %.8e" %
        (d, out["iters"], out["quad"], y @ a, out["logdet"], q_ld.mean(), out["trace_dk_dlengthscale"],
         t_dk.mean()))
    assert out["status"] == "MM_OK" and out["converged"] == 1
    assert np.linalg.norm(to_np(alpha) - a) <= 1e-8 * np.linalg.norm(a)
    assert abs(out["quad"] - y @ a) <= 1e-9 * abs(y @ a)
    assert abs(out["logdet"] - q_ld.mean()) <= 1e-6 * abs(q_ld.mean())
    assert abs(out["trace_inv"] - t_inv.mean()) <= 1e-8 * abs(t_inv.mean())
    assert abs(out["trace_dk_dlengthscale"] - t_dk.mean()) <= 1e-8 * abs(t_dk.mean())
    # the gradient assembled from the same estimates (eq. gp_log_likelihood_derivative)
    g_ell = 0.5 * a @ D @ a - 0.5 * t_dk.mean()
    g_sig = 0.5 * a @ a - 0.5 * t_inv.mean()
    g_s2 = (0.5 * a @ K @ a - 0.5 * t_k.mean()) / s2
    for got, ref, scale in ((out["dlml_dlengthscale"], g_ell, 0.5 * a @ D @ a),
                            (out["dlml_dsigma2"], g_sig, 0.5 * a @ a),
                            (out["dlml_doutputscale2"], g_s2, 0.5 * a @ K @ a / s2)):
        assert abs(got - ref) <= 1e-7 * max(abs(ref), abs(scale))
    lml = -0.5 * out["quad"] - 0.5 * out["logdet"] - 0.5 * n * np.log(2 * np.pi)
    assert abs(out["lml"] - lml) <= 1e-12 * abs(lml)
    # the estimates against the exact values, within five standard errors
    ex_ell, ex_sig, ex_s2 = oracle.lml_grad_exact(x, y, two_nu, "product", ell, s2, sig)
    assert abs(out["dlml_dlengthscale"] - ex_ell) <= 5 * 0.5 * np.std(t_dk, ddof=1) / np.sqrt(l) + 1e-9
    assert abs(out["dlml_dsigma2"] - ex_sig) <= 5 * 0.5 * np.std(t_inv, ddof=1) / np.sqrt(l) + 1e-9
    assert abs(out["dlml_doutputscale2"] - ex_s2) <= 5 * 0.5 * np.std(t_k, ddof=1) / np.sqrt(l) / s2 + 1e-9
    ex_lml = oracle.lml_exact(x, y, two_nu, "product", ell, s2, sig)
    assert abs(out["lml"] - ex_lml) <= 5 * 0.5 * np.std(q_ld, ddof=1) / np.sqrt(l) + 1e-9


def test_lml_reports_nonconvergence_and_refuses_l1(oracle_lib):
    x, y, Z = _lml_problem(9400, 600, 2, 3, 7)
    plan = mm.Plan(to_gpu(x), mm.Kernel(3, "product", 0.2))
    out = plan.lml(to_gpu(y), 0.01, to_gpu(Z), maxit=3, rtol=1e-12, raise_on_error=False)
    assert out["status"] == "MM_ERR_NOCONV" and out["converged"] == 0 and out["iters"] == 3
    assert np.isfinite(out["lml"]) and np.isfinite(out["dlml_dlengthscale"])
    plan.close()
    plan = mm.Plan(to_gpu(x), mm.Kernel(3, "l1", 0.2))
    with pytest.raises(mm.MaternError) as e:
        plan.lml(to_gpu(y), 0.01, to_gpu(Z))
    assert e.value.status == mm.MM_ERR_NOTPD
    plan.close()


@pytest.mark.parametrize("d,two_nu,m", [(1, 1, 5), (2, 3, 40), (3, 5, 33)])
def test_posterior_variance_matches_oracle(oracle_lib, d, two_nu, m):
    """eq. gp_variance at prediction points spread over the domain, on training
    points and far away; 40 points take two blocks of solves."""
    rng = np.random.default_rng(9500 + d)
    n, ell, s2, sig = 900, 0.15, 1.3, 0.02
    x = rng.uniform(0, 1, (n, d))
    z = rng.uniform(0, 1, (m, d))
    z[0] = x[3]                       # on a training point
    z[-1] = 40.0                      # far from all of them
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, "product", ell, s2))
    var, info = plan.variance(to_gpu(z), sig, rtol=1e-12, maxit=n)
    plan.close()
    ref = oracle.posterior_variance(x, z, two_nu, "product", ell, s2, sig)
    err = np.max(np.abs(to_np(var) - ref))
    say("variance d=%d m=%d: iters %d max err %.2e" % (d, m, info["iters"], err))
    assert info["status"] == "MM_OK" and info["converged_cols"] == m
    assert err <= 1e-9 * s2
    assert abs(to_np(var)[-1] - s2) <= 1e-12
