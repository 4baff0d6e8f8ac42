"""Continuous-batching server and the many-problem runner.

Each served request must give what it gives alone (gp_cg_solve + gp_predict
on its own plan), bitwise, however the stream interleaves it with others; the
admission budget must hold at every tick and requests must overlap on the
device.  One request is also checked against the oracle's GLS and predictor.
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
from paper_2508_01864_amd import batched, serve
import workloads
from gpu_util import MVM_TOL, SOLVE_TOL, say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _requests(seed, count, n_lo, n_hi, gap):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        d = int(rng.integers(1, 4))
        two_nu = int(rng.choice([1, 3, 5]))
        ell = float(np.exp(rng.uniform(np.log(0.05), np.log(0.5))))
        s2 = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-1))))
        x = rng.uniform(0, 1, (n, d))
        beta = rng.standard_normal(d + 1)
        y = beta[0] + x @ beta[1:] + workloads.field_sin_cos(x) + np.sqrt(s2) * rng.standard_normal(n)
        z = rng.uniform(0, 1, (200, d))
        out.append(serve.Request(k, t, x, y, mm.Kernel(two_nu, workloads.solve_form(two_nu, d), ell), s2, z,
                                 rtol=1e-10, maxit=20000))
        t += float(rng.exponential(gap))
    return out


def _alone(r):
    plan = mm.Plan(to_gpu(r.x), r.kernel)
    alpha, beta, info = plan.cg_solve(to_gpu(r.y), r.sigma2, fixed_effects=True, rtol=r.rtol, maxit=r.maxit)
    mean = plan.predict(alpha, to_gpu(r.z), beta=beta)
    out = (to_np(alpha), beta, to_np(mean), info)
    plan.close()
    return out


def test_side_stream_admission_changes_nothing(oracle_lib):
    """Admissions built on the server's side stream while a chunk runs give the same
    bits as admissions built on the caller's stream between chunks."""
    reqs = _requests(15, 6, 300, 3000, 0.001)
    a = serve.Server(max_slots=4, chunk=8, side_stream=True).run(reqs)
    b = serve.Server(max_slots=4, chunk=8, side_stream=False).run(reqs)
    assert len(a) == len(b) == len(reqs)
    for ra, rb in zip(a, b):
        assert np.array_equal(to_np(ra.alpha), to_np(rb.alpha))
        assert np.array_equal(to_np(ra.mean), to_np(rb.mean))
        assert np.array_equal(ra.beta, rb.beta)


def test_served_equals_alone_with_admission_and_overlap(oracle_lib):
    reqs = _requests(5, 10, 300, 4000, 0.002)
    sizes = [serve.request_bytes(len(r.y), r.x.shape[1], len(r.z), r.kernel) for r in reqs]
    budget = sum(sorted(sizes)[-3:])          # room for about three requests at a time
    srv = serve.Server(budget_bytes=budget, max_slots=6, chunk=8)
    resps = srv.run(reqs)
    say("served: ticks %d rebuilds %d peak slots %d peak bytes %d / %d" %
        (srv.ticks, srv.rebuilds, srv.peak_slots, srv.peak_bytes, budget))
    assert len(resps) == len(reqs)
    assert srv.peak_bytes <= budget
    assert srv.peak_slots >= 2                # requests shared the device
    for r, q in zip(reqs, resps):
        a0, b0, m0, i0 = _alone(r)
        assert q.info["status"] == "MM_OK"
        assert q.info["iters"] == i0["iters"]
        assert np.array_equal(to_np(q.alpha), a0), "request %d" % r.rid
        assert np.array_equal(q.beta, b0)
        assert np.array_equal(to_np(q.mean), m0)
        assert q.done >= q.admitted >= q.arrival
    s = serve.summary(resps)
    assert s["p99_s"] >= s["p50_s"] > 0


def test_served_request_matches_oracle(oracle_lib):
    reqs = _requests(9, 3, 500, 1200, 0.0)
    resps = serve.Server(budget_bytes=1 << 34, chunk=16).run(reqs)
    for r, q in zip(reqs, resps):
        form = r.kernel.form
        bref, aref = oracle.gls(r.x, r.y, r.kernel.two_nu, form, r.kernel.lengthscale, 1.0, r.sigma2)
        a = to_np(q.alpha)
        assert np.linalg.norm(a - aref) / np.linalg.norm(aref) <= SOLVE_TOL
        assert np.max(np.abs(q.beta - bref)) <= SOLVE_TOL * max(1.0, np.max(np.abs(bref)))
        mref = oracle.predict(r.x, a, r.z, r.kernel.two_nu, form, r.kernel.lengthscale, 1.0, beta=q.beta)
        _, kabs = oracle.mvm(r.x, np.abs(a), r.kernel.two_nu, form, r.kernel.lengthscale, z=r.z, with_abs=True)
        scale = kabs + np.abs(oracle.design_matrix(r.z)) @ np.abs(q.beta)
        assert np.max(np.abs(to_np(q.mean) - mref) / scale) <= MVM_TOL


def test_plain_server_equals_alone(oracle_lib):
    reqs = _requests(13, 3, 300, 1500, 0.01)
    resps = serve.run_plain(reqs)
    for r, q in zip(reqs, resps):
        a0, b0, m0, _ = _alone(r)
        assert np.array_equal(to_np(q.alpha), a0)
        assert np.array_equal(to_np(q.mean), m0)


def test_solve_many_with_tuning_and_rebuilds_equals_alone(oracle_lib, tmp_path, monkeypatch):
    monkeypatch.setenv("MM_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs = workloads.config4(seed=404, count=12, n_lo=200, n_hi=5000)
    plans = [mm.Plan(to_gpu(p.x), mm.Kernel(p.two_nu, p.form, p.ell)) for p in probs]
    res = batched.solve_many(plans, [to_gpu(p.y) for p in probs], [p.sigma2 for p in probs],
                             rtol=1e-10, chunk=8, tune=True, rebuild_frac=0.1)
    assert (tmp_path / "tune.json").exists()
    for p, pl, r in zip(probs, plans, res):
        alpha, _, info = pl.cg_solve(to_gpu(p.y), p.sigma2, rtol=1e-10)
        assert r.info["iters"] == info["iters"]
        assert np.array_equal(to_np(r.alpha), to_np(alpha))
        pl.close()
