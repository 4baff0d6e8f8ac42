#!/usr/bin/env python3
"""Benchmark of the exact Matern kernel product and the GP solve built on it.

Workload: d = 2, N = 100,000, nu = 3/2, product form, lengthscale 0.1,
x ~ U[0,1]^2, y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.1^2), sigma^2 = 0.01
(synthetic, seeded).

One step is one pass of the whole hot path with the inputs already in HBM:
  plan build (sort, stored divide-and-conquer orders)  ->  one plain product
  y = K v  ->  conjugate-gradient solve of (K + sigma^2 I) with the linear
  fixed effects [1, x1, x2] (GLS), relative residual 1e-8  ->  posterior mean
  at 1000 new points.
`value` is the number of product point-columns (N x right-hand sides, summed
over every product of the step) per second of step wall time.

Also printed in the same JSON line:
  roofline      the dominant kernel, the divide-and-conquer sweep launch of a CG
                iteration (one launch covers every pass of the 4-column product):
                algorithmic bytes per launch (passes x N x (4 + 16 x 4)) over its
                average duration, measured with HIP events on its stream during
                the timed solves, against the 8 TB/s HBM peak; `traffic` is the
                measured HBM bytes per launch from the committed rocprofv3 counter
                summary, when that summary matches the current kernel source;
  mvm           the plain product alone at 1, 8 and 32 right-hand sides;
  batched       256 independent problems of uneven N, d, nu and lengthscale
                (N log-uniform in [1e3, 2e5], d in {1,2,3}, nu in {1/2,3/2,5/2}):
                one product each and a fixed number of CG iterations each, run
                batched (shared launches, HIP-graph replay, autotuned grids)
                and one problem at a time through the plain entry points, on
                the same inputs; results are checked bitwise equal;
  pcg           the same solve with the rank-100 pivoted Cholesky preconditioner
                against plain CG: iterations and time to solution;
  served        a bounded sample of the served GP-regression stream (fixed
                effects, Poisson arrivals at 0.9x the plain path's measured
                capacity): p50/p99 latency and solves/s of the continuous-
                batching server against first-come-first-served plain solves;
  cpu_baseline  the dense FP64 CPU oracle timed on a bounded sample of target
                rows of the same product (all host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 100_000
D = 2
TWO_NU = 3
ELL = 0.1
SIGMA2 = 0.01
RTOL = 1e-8
NPREDICT = 1000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def b_pass(n: int, cols: int) -> float:
    """Algorithmic bytes of one divide-and-conquer pass: 4-byte order index plus,
    per column, an 8-byte weight read and an 8-byte partial-sum write per point."""
    return float(n) * (4.0 + 16.0 * cols)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_main_d2_n100k_nu32_w4.txt")
SWEEP_SRC = os.path.join(ROOT, "paper_2508_01864_amd", "csrc", "sweep_core.h")


def recorded_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None when the kernel source has changed
    since the counters were taken (the summary records the SHA-256 of the
    kernels' source, sweep_core.h)."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(SWEEP_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.split("=", 1) for line in text.splitlines() if "=" in line and not line.startswith(" "))
    if fields.get("sweep_core_sha256", "").strip() != src:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(x, v, seconds: float):
    import oracle
    oracle.build(force=False)
    rows = 200
    t0 = time.perf_counter()
    oracle.mvm(x, v, TWO_NU, "product", ELL, z=x[:rows])
    dt = time.perf_counter() - t0
    rows = int(min(N, max(rows, rows * seconds / max(dt, 1e-6))))
    t0 = time.perf_counter()
    oracle.mvm(x, v, TWO_NU, "product", ELL, z=x[:rows])
    dt = time.perf_counter() - t0
    return {"value": rows / dt, "unit": "points/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "dense FP64 product K v for %d of the %d target rows (nrhs=1, %.1f s), "
                      "points/s = rows / time" % (rows, N, dt)}


def _events_ms(fn, reps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_pcg(mm, x, y, kern, rank, reps=2):
    """The headline solve (fixed effects, rtol 1e-8) with the rank-k pivoted
    Cholesky preconditioner, against plain CG: iterations and time to solution
    (plan and preconditioner build included), and the true residual."""
    import torch
    out = {"rank": rank}
    for label, use_pc in (("plain", False), ("preconditioned", True)):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = mm.Plan(x, kern)
            pc = mm.Precond(plan, max_rank=rank) if use_pc else None
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            alpha, beta, info = plan.cg_solve(y, SIGMA2, fixed_effects=True, rtol=RTOL, maxit=20000, precond=pc)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            Ka = plan.mvm(alpha, shift=SIGMA2)
            H = torch.cat([torch.ones(N, 1, dtype=torch.float64, device=x.device), x], dim=1)
            res = float(torch.linalg.norm(y - H @ torch.as_tensor(beta, device=x.device) - Ka) / torch.linalg.norm(y))
            if pc is not None:
                pc.close()
            plan.close()
            rec = {"iters": info["iters"], "setup_s": t1 - t0, "solve_s": t2 - t1, "total_s": t2 - t0,
                   "true_relres": res}
            if best is None or rec["total_s"] < best["total_s"]:
                best = rec
        out[label] = best
        log("%s: %d iterations, %.3f s" % (label, best["iters"], best["total_s"]))
    out["speedup"] = out["plain"]["total_s"] / out["preconditioned"]["total_s"]
    return out


def bench_gradient(mm, x, y, kern, probes, reps):
    """The headline configuration's lengthscale-derivative products (nrhs 1, 4
    and 32, against the plain product) and one evaluation of the log marginal
    likelihood with its gradient from `probes` Rademacher probes (CG to 1e-8,
    zero mean: the targets centred by their mean)."""
    import torch
    out = {"dlengthscale_mvm": {}}
    plan = mm.Plan(x, kern)
    for nrhs in (1, 4, 32):
        vv = torch.as_tensor(np.random.default_rng(70 + nrhs).standard_normal((nrhs, N)), device=x.device)
        yy = torch.empty_like(vv)
        for _ in range(2):
            plan.mvm_dlengthscale_raw(vv, yy, nrhs)
            plan.mvm_raw(vv, yy, nrhs)
        ms_d = _events_ms(lambda: plan.mvm_dlengthscale_raw(vv, yy, nrhs), reps)
        ms_k = _events_ms(lambda: plan.mvm_raw(vv, yy, nrhs), reps)
        out["dlengthscale_mvm"][str(nrhs)] = {"ms": round(ms_d, 4), "points_per_s": N * nrhs / (ms_d * 1e-3),
                                              "plain_ms": round(ms_k, 4)}
        log("dK/dl product nrhs=%d: %.3f ms (plain %.3f ms)" % (nrhs, ms_d, ms_k))
    Z = torch.as_tensor(np.random.default_rng(71).choice([-1.0, 1.0], size=(N, probes)), device=x.device)
    yc = y - y.mean()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.lml(yc, SIGMA2, Z, maxit=20000, rtol=RTOL, raise_on_error=False)
    torch.cuda.synchronize()
    res["seconds"] = time.perf_counter() - t0
    res["probes"] = probes
    out["lml"] = res
    log("lml with %d probes: %d iterations, %.2f s, L = %.6e, dL/dl = %.4e" %
        (probes, res["iters"], res["seconds"], res["lml"], res["dlml_dlengthscale"]))
    plan.close()
    return out


def bench_config3(dev, steps, rank):
    """d=3, N=500k, nu=5/2, lengthscale 0.3, x ~ N(0, I): one product with the 32
    Rademacher probes (product and L1 forms), the stochastic log-determinant from
    those probes (`steps` Lanczos steps), and one CG solve of the sin/cos
    targets (sigma2 0.01) preconditioned with the rank-`rank` pivoted Cholesky."""
    import torch
    import paper_2508_01864_amd as mm
    import workloads
    p = workloads.config3()
    n = p.n
    x = torch.as_tensor(p.x, device=dev)
    Z = torch.as_tensor(p.v, device=dev)          # (n, 32) Rademacher
    out = {"workload": "d=3 N=%d nu=5/2 ell=0.3 x~N(0,I3), 32 Rademacher probes" % n}
    for form in ("product", "l1"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = mm.Plan(x, mm.Kernel(5, form, 0.3))
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        Zc = Z.t().contiguous()
        Yc = torch.empty_like(Zc)
        plan.mvm_raw(Zc, Yc, 32)
        ms = _events_ms(lambda: plan.mvm_raw(Zc, Yc, 32), 2)
        out[form] = {"plan_build_s": tb, "mvm32_ms": ms, "points_per_s": n * 32 / (ms * 1e-3)}
        log("config 3 %s: 32-column product %.1f ms" % (form, ms))
        if form == "product":
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            est, quad, msteps = plan.logdet(0.01, Z, steps=steps, rtol=0.0)
            torch.cuda.synchronize()
            out["logdet"] = {"estimate": est, "steps": int(msteps.max()), "probes": 32,
                             "stderr": float(np.std(quad, ddof=1) / np.sqrt(len(quad))),
                             "seconds": time.perf_counter() - t0}
            log("config 3 log det ~ %.6e (%d steps)" % (est, int(msteps.max())))
            y = torch.as_tensor(p.y, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc = mm.Precond(plan, max_rank=rank)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            alpha, _, info = plan.cg_solve(y, 0.01, rtol=1e-8, maxit=4000, precond=pc, raise_on_error=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            out["pcg_solve"] = {"rank": rank, "precond_s": t1 - t0, "solve_s": t2 - t1, "iters": info["iters"],
                                "status": info["status"], "relres": info["relres_max"]}
            log("config 3 PCG: %d iterations, %.2f s" % (info["iters"], t2 - t1))
            pc.close()
        plan.close()
    return out


def bench_batched(dev, count, iters):
    """256 uneven problems: batched vs one-at-a-time, products and CG iterations."""
    import torch
    import paper_2508_01864_amd as mm
    from paper_2508_01864_amd import autotune, batched
    import workloads
    probs = workloads.config4(count=count)
    ntot = int(sum(p.n for p in probs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = [mm.Plan(torch.as_tensor(p.x, device=dev), mm.Kernel(p.two_nu, p.form, p.ell)) for p in probs]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    vcs = [torch.as_tensor(p.v, device=dev).view(1, -1) for p in probs]
    y_plain = [torch.empty_like(v) for v in vcs]
    y_batch = [torch.empty_like(v) for v in vcs]

    def plain_mvm():
        for pl, v, y in zip(plans, vcs, y_plain):
            pl.mvm_raw(v, y, 1)
    mb = mm.MvmBatch(plans, nrhs=1, use_graph=True)
    key = autotune.signature("mvm", [(p.n, p.d, p.kernel.two_nu, p.kernel.form, 1) for p in plans])
    sched = autotune.tune(mb, key, lambda: mb.run_raw(vcs, y_batch), reps=2)

    def batch_mvm():
        mb.run_raw(vcs, y_batch)
    plain_mvm()
    batch_mvm()
    ms_plain = _events_ms(plain_mvm, 3)
    ms_batch = _events_ms(batch_mvm, 5)
    torch.cuda.synchronize()
    same_mvm = all(torch.equal(a, b) for a, b in zip(y_plain, y_batch))
    mb.close()

    # CG: `iters` iterations of every problem (no convergence test counted)
    ys = [torch.as_tensor(p.y, device=dev) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alphas_plain = [pl.cg_solve(y, p.sigma2, rtol=1e-8, maxit=iters, raise_on_error=False)[0]
                    for pl, y, p in zip(plans, ys, probs)]
    torch.cuda.synchronize()
    cg_plain_s = time.perf_counter() - t0
    # tune once on a throwaway batch of the same shape (its iterations are not timed)
    warm = batched.solve_many(plans, ys, [p.sigma2 for p in probs], rtol=1e-8, maxit=40, chunk=8, tune=True)
    del warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batched.solve_many(plans, ys, [p.sigma2 for p in probs], rtol=1e-8, maxit=iters,
                             chunk=min(16, iters), tune=True, rebuild_frac=1.0)   # cached schedule
    torch.cuda.synchronize()
    cg_batch_s = time.perf_counter() - t0
    same_cg = all(torch.equal(a, r.alpha) for a, r in zip(alphas_plain, res))
    for pl in plans:
        pl.close()
    by_d = {str(d): int(sum(1 for p in probs if p.d == d)) for d in (1, 2, 3)}
    return {
        "workload": "%d problems, N log-uniform [1e3, 2e5] (total %d points), d/nu uniform, "
                    "ell log-uniform [0.05, 0.5], sigma2 0.01, product form for nu >= 3/2 in d >= 2" % (count, ntot),
        "dims": by_d, "total_points": ntot, "plan_build_s": build_s,
        "mvm_plain_ms": ms_plain, "mvm_batched_ms": ms_batch,
        "mvm_points_per_s_plain": ntot / (ms_plain * 1e-3),
        "mvm_points_per_s_batched": ntot / (ms_batch * 1e-3),
        "mvm_speedup": ms_plain / ms_batch, "mvm_bitwise_equal": bool(same_mvm),
        "mvm_schedule": list(sched),
        "cg_iters": iters, "cg_plain_s": cg_plain_s, "cg_batched_s": cg_batch_s,
        "cg_point_iters_per_s_plain": ntot * iters / cg_plain_s,
        "cg_point_iters_per_s_batched": ntot * iters / cg_batch_s,
        "cg_speedup": cg_plain_s / cg_batch_s, "cg_bitwise_equal": bool(same_cg),
    }


def bench_served(dev, count):
    """The served stream against plain first-come-first-served solves."""
    import torch
    import paper_2508_01864_amd as mm
    from paper_2508_01864_amd import serve
    import workloads
    probs = workloads.config5(count=count, rate=1.0)
    base = [p.arrival for p in probs]          # unit-rate Poisson arrival times
    reqs = [serve.Request(k, 0.0, p.x, p.y, mm.Kernel(p.two_nu, p.form, p.ell), p.sigma2, p.z,
                          rtol=1e-8, maxit=20000) for k, p in enumerate(probs)]
    # plain service times (all requests back to back) give the plain capacity
    def done(tag):
        return lambda r: log("%s: request %d (n=%d) done, %d iterations" % (tag, r.rid, len(reqs[r.rid].y),
                                                                          r.info.get("iters", -1)))

    plain0 = serve.run_plain(reqs, on_done=done("plain"))
    service = [r.done - r.admitted for r in plain0]
    cap = len(reqs) / sum(service)
    rate = 0.9 * cap
    for r, a in zip(reqs, base):
        r.arrival = a / rate
    # plain FIFO latencies for these arrivals from the measured service times
    free_at = 0.0
    plain = []
    for r, sv in zip(reqs, service):
        start = max(free_at, r.arrival)
        free_at = start + sv
        plain.append(serve.Response(r.rid, r.arrival, start, free_at, None, None, None, {}))
    srv = serve.Server(chunk=16)
    served = srv.run(reqs, on_done=done("served"))
    same = all(torch.equal(a.alpha, b.alpha) and torch.equal(a.mean, b.mean) for a, b in zip(served, plain0))
    sp, ss = serve.summary(plain), serve.summary(served)
    return {
        "workload": "first %d requests of the served stream: N log-uniform [5e3, 3e5], d/nu uniform, "
                    "sigma2 log-uniform [1e-3, 1e-1], affine trend + sin/cos field, fixed effects, "
                    "1000 predict points, rtol 1e-8; Poisson arrivals at 0.9x plain capacity" % count,
        "n": [len(r.y) for r in reqs], "d": [int(r.x.shape[1]) for r in reqs],
        "rate_per_s": rate, "plain_capacity_per_s": cap,
        "plain": sp, "served": ss, "served_bitwise_equal_alone": bool(same),
        "iters": [r.info["iters"] for r in served],
        "server": {"ticks": srv.ticks, "rebuilds": srv.rebuilds, "peak_slots": srv.peak_slots,
                   "peak_bytes": srv.peak_bytes, "budget_bytes": srv.budget},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mvm-reps", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mvm", action="store_true")
    ap.add_argument("--batched-count", type=int, default=256)
    ap.add_argument("--batched-iters", type=int, default=32)
    ap.add_argument("--served-count", type=int, default=4)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--config3", action="store_true",
                    help="also run the d=3 N=500k nu=5/2 section: one 32-probe product, the "
                         "stochastic log-determinant from those probes and one preconditioned solve")
    ap.add_argument("--logdet-steps", type=int, default=30)
    ap.add_argument("--lml-probes", type=int, default=31,
                    help="probes of the likelihood-gradient section (0: skip the section)")
    ap.add_argument("--pcg-rank", type=int, default=100,
                    help="rank of the pivoted Cholesky preconditioner of the extra PCG section (0: skip)")
    ap.add_argument("--maxit", type=int, default=20000,
                    help="CG iteration limit (below the default only for short profiling runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a device-to-device copy of this many MiB three times before the "
                         "steps (a known-size kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2508_01864_amd as mm
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = workloads.config2()
    rng = np.random.default_rng(20021)
    z_np = rng.uniform(0.0, 1.0, size=(NPREDICT, D))
    x = torch.as_tensor(p.x, device=dev)
    y = torch.as_tensor(p.y, device=dev)
    v = torch.as_tensor(p.v, device=dev)
    z = torch.as_tensor(z_np, device=dev)
    kern = mm.Kernel(TWO_NU, "product", ELL, 1.0)
    L = mm.levels(N)

    def step(profile: bool):
        plan = mm.Plan(x, kern)
        y1 = plan.mvm(v)
        if profile:                          # bracket the solve's sweep launches only
            plan.profile_enable(True)
        alpha, beta, info = plan.cg_solve(y, SIGMA2, fixed_effects=True, rtol=RTOL, maxit=args.maxit,
                                          raise_on_error=args.maxit >= 20000)
        prof = plan.profile_read() if profile else (0.0, 0, 0)
        if profile:
            plan.profile_enable(False)
        mean = plan.predict(alpha, z, beta=beta)
        plan.close()
        cols = 1 + 4 * info["iters"]        # plain product + CG columns (y, 1, x1, x2)
        pts = N * cols + (N + NPREDICT)      # + predict on the union of points
        # algorithmic bytes of the profiled launches: one per CG iteration, L passes, 4 columns
        sweep_bytes = info["iters"] * L * b_pass(N, 4)
        return pts, info, prof, sweep_bytes, (y1, alpha, beta, mean)

    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * 131072, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written per launch" % (args.calib_copy_mib, args.calib_copy_mib))
        del src, dst

    for w in range(args.warmup):
        log("warmup step %d" % w)
        step(False)
    torch.cuda.synchronize()

    log("timed steps: %d" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_pts = 0
    tot_ms = 0.0
    tot_launch = 0
    tot_bytes = 0.0
    iters = []
    last = None
    for s in range(args.steps):
        pts, info, prof, sb, last = step(True)
        tot_pts += pts
        tot_ms += prof[0]
        tot_launch += prof[1]
        tot_bytes += sb
        iters.append(info["iters"])
        log("step %d: CG iters %d relres %.2e" % (s, info["iters"], info["relres_max"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = tot_pts / elapsed
    avg_launch_ms = tot_ms / max(tot_launch, 1)
    # algorithmic bytes per launch (total over the launches / their number) over the
    # average launch duration
    achieved = (tot_bytes / max(tot_launch, 1)) / (avg_launch_ms * 1e-3) / 1e9 if tot_launch else 0.0

    # true residual of the last solve: ||y - H beta - (K + s I) alpha|| / ||y||
    _, alpha, beta, _ = last
    plan = mm.Plan(x, kern)
    Ka = plan.mvm(alpha, shift=SIGMA2)
    H = torch.cat([torch.ones(N, 1, dtype=torch.float64, device=dev), x], dim=1)
    bt = torch.as_tensor(beta, device=dev)
    true_res = float(torch.linalg.norm(y - H @ bt - Ka) / torch.linalg.norm(y))

    mvm_rows = {}
    if not args.no_mvm:
        for nrhs in (1, 8, 32):
            vv = torch.as_tensor(np.random.default_rng(7 + nrhs).standard_normal((nrhs, N)), device=dev)
            yy = torch.empty_like(vv)
            for _ in range(3):
                plan.mvm_raw(vv, yy, nrhs)
            plan.profile_enable(True)
            plan.profile_read(reset=True)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.mvm_reps):
                plan.mvm_raw(vv, yy, nrhs)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.mvm_reps
            sms, scnt, _ = plan.profile_read(reset=True)
            plan.profile_enable(False)
            sweep_ms = sms / max(scnt, 1)           # one launch covers all L passes
            mvm_rows[str(nrhs)] = {
                "ms": round(ms, 4), "points_per_s": N * nrhs / (ms * 1e-3),
                "sweep_ms": round(sweep_ms, 4),
                "sweep_gbs": L * b_pass(N, nrhs) / (sweep_ms * 1e-3) / 1e9,
            }
            log("mvm nrhs=%d: %.3f ms (%.3e points/s)" % (nrhs, ms, N * nrhs / (ms * 1e-3)))
    plan.close()

    pcg_out = None
    if args.pcg_rank > 0:
        log("preconditioned solve: rank %d" % args.pcg_rank)
        pcg_out = bench_pcg(mm, x, y, kern, args.pcg_rank)

    grad_out = None
    if args.lml_probes > 0:
        log("gradient: dK/dl products and the likelihood with %d probes" % args.lml_probes)
        grad_out = bench_gradient(mm, x, y, kern, args.lml_probes, args.mvm_reps)

    c3_out = None
    if args.config3:
        log("config 3: d=3 N=500k nu=5/2, 32 probes")
        c3_out = bench_config3(dev, args.logdet_steps, args.pcg_rank or 100)

    batched_out = None
    if not args.no_batched:
        log("batched: %d problems" % args.batched_count)
        batched_out = bench_batched(dev, args.batched_count, args.batched_iters)
    served_out = None
    if not args.no_served and args.served_count > 0:
        log("served: %d requests" % args.served_count)
        served_out = bench_served(dev, args.served_count)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(p.x, p.v, args.cpu_seconds)

    out = {
        "metric": "Matern MVM points/s (N x nrhs) d=2 N=100k nu=3/2",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "d=2 N=100000 nu=3/2 product ell=0.1 sigma2=0.01: plan build, "
                               "K v, CG+GLS to 1e-8, predict 1000 points",
                   "n": N, "d": D, "two_nu": TWO_NU, "form": "product", "lengthscale": ELL,
                   "sigma2": SIGMA2, "rtol": RTOL, "npredict": NPREDICT},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(),
                     "algorithmic_bytes_per_launch": L * b_pass(N, 4),
                     "kernel": "sweep_batch_kernel<d=2, nu=3/2, product, 4 columns> main launch of a CG "
                               "iteration (all %d divide-and-conquer passes per launch)" % L,
                     "avg_launch_ms": avg_launch_ms, "launches": tot_launch},
        "cpu_baseline": cpu,
        "cg_iters": iters,
        "true_relres": true_res,
        "mvm": mvm_rows,
        "pcg": pcg_out,
        "gradient": grad_out,
        "config3": c3_out,
        "batched": batched_out,
        "served": served_out,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
