#!/usr/bin/env python3
"""Benchmark of the exact Matern kernel product and the GP solve built on it.

Headline workload: d = 2, N = 100,000, nu = 3/2, product form, lengthscale 0.1,
x ~ U[0,1]^2 (synthetic, seeded), plan prebuilt, inputs resident in HBM.

One step is one call of matern_mvm, y = K v, on that plan with 32 right-hand
sides (the width of the multi-probe products).  `value` is N x nrhs / step
time (product point-columns per second) over the timed steps.

Also printed in the same JSON line:
  roofline      the dominant kernel, the main divide-and-conquer sweep launch of
                the headline product (one launch covers every pass): algorithmic
                bytes per launch (passes x N x (4 + 16 x 32)) over its average
                duration measured with HIP events on its stream during the timed
                steps, against the 8 TB/s HBM peak; `traffic` is the measured HBM
                bytes per launch from the committed rocprofv3 counter summary,
                when that summary matches the current kernel source;
  mvm           the median of one product (product and L1 forms) at 1, 8 and
                32 right-hand sides: points/s and the fraction of the HBM peak and
                of the measured copy bandwidth for the whole call against the
                level-streaming bytes N (8d + 16 nrhs + L (4 + 16 nrhs)), with the
                main sweep launch's own fraction beside it;
  plan_build_s  the plan build (sorts and stored orders), timed on its own;
  stream_copy   a device-to-device copy's measured bandwidth (read + write);
  solve         the configuration-2 GP regression: plan build, CG with the linear
                fixed effects (GLS) to relative residual 1e-8 and prediction at
                1000 points; the residual of the returned solution recomputed with
                the CPU oracle's dense product over every row;
  pcg           the same solve with the rank-100 pivoted Cholesky preconditioner;
  gradient      lengthscale-derivative products and the likelihood gradient;
  config3       d = 3, N = 500,000, nu = 5/2: the 32-probe product (both forms), the
                stochastic log-determinant and the single CG solve to rtol 1e-8;
  batched       256 independent problems of uneven N, d, nu and lengthscale,
                batched against one at a time, results checked bitwise equal;
  served        a bounded sample of the served GP-regression stream at three
                arrival rates against first-come-first-served plain solves;
  cpu_baseline  the dense FP64 CPU oracle timed on a bounded sample of target
                rows of the headline product (all host cores).
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_main_d2_n100k_nu32_w32.txt")
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


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, nrhs: int, seconds: float):
    """The oracle's dense product (each kernel entry evaluated once for all
    columns) on a bounded sample of target rows of the headline product."""
    import oracle
    oracle.build(force=False)
    v = np.random.default_rng(7 + nrhs).standard_normal((N, nrhs))
    rows, dt = 50, 0.0
    for _ in range(4):     # grow the sample until it takes most of `seconds`
        rows = int(min(N, max(rows, rows * seconds / max(dt, 1e-6)) if dt else rows))
        t0 = time.perf_counter()
        oracle.mvm(x, v, TWO_NU, "product", ELL, z=x[:rows], shared_kernel=True)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * seconds or rows == N:
            break
    return {"value": rows * nrhs / dt, "unit": "points/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": "dense FP64 product K v for %d of the %d target rows at nrhs=%d (%.1f s); "
                      "points/s = rows x nrhs / time" % (rows, N, nrhs, dt)}


def b_alg(n: int, d: int, nrhs: int, L: int) -> float:
    """Level-streaming algorithmic bytes of one product: x and v read, y written
    once, and per pass the 4-byte order index plus, per column, an 8-byte weight
    read and an 8-byte partial-sum write per point."""
    return float(n) * (8.0 * d + 16.0 * nrhs + L * (4.0 + 16.0 * nrhs))


def stream_copy_gbs(dev, mib: int = 1024, reps: int = 10) -> float:
    """Measured device-to-device copy bandwidth, bytes read + written per second."""
    import torch
    src = torch.ones(mib * 131072, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    return 2.0 * mib * 1048576 / (float(np.median(ts)) * 1e-3) / 1e9


def median_ms(fn, reps: int) -> float:
    """Median of `reps` single calls timed with HIP events on the current stream."""
    import torch
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def bench_mvm(mm, x, dev, reps: int, copy_gbs: float):
    """Median matern_mvm at 1, 8 and 32 columns, product and L1 forms, each on the
    schedule the autotuner picks for its width."""
    import torch
    from paper_2508_01864_amd import autotune
    L = mm.levels(N)
    out = {}
    for form in ("product", "l1"):
        plan = mm.Plan(x, mm.Kernel(TWO_NU, form, ELL))
        rows = {}
        for nrhs in (1, 8, 32):
            vv = torch.as_tensor(np.random.default_rng(7 + nrhs).standard_normal((nrhs, N)), device=dev)
            yy = torch.empty_like(vv)
            sched = autotune.tune_schedule(plan, nrhs, vectors=vv)
            for _ in range(3):
                plan.mvm_raw(vv, yy, nrhs)
            torch.cuda.synchronize()
            ms = median_ms(lambda: plan.mvm_raw(vv, yy, nrhs), reps)
            plan.profile_enable(True)
            plan.profile_read(reset=True)
            for _ in range(reps):
                plan.mvm_raw(vv, yy, nrhs)
            sms, scnt, _ = plan.profile_read(reset=True)
            plan.profile_enable(False)
            sweep_ms = sms / max(scnt, 1)
            ba = b_alg(N, D, nrhs, L)
            rows[str(nrhs)] = {
                "median_ms": round(ms, 4), "points_per_s": N * nrhs / (ms * 1e-3), "schedule": list(sched),
                "b_alg_bytes": ba, "gbs": ba / (ms * 1e-3) / 1e9,
                "frac_hbm_peak": ba / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "frac_copy_peak": ba / (ms * 1e-3) / 1e9 / copy_gbs,
                "main_sweep_ms": round(sweep_ms, 4),
                "main_sweep_frac_hbm_peak": L * b_pass(N, nrhs) / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            }
            log("mvm %s nrhs=%d: median %.4f ms, %.3e points/s, %.3f of HBM peak" %
                (form, nrhs, ms, N * nrhs / (ms * 1e-3), rows[str(nrhs)]["frac_hbm_peak"]))
        plan.close()
        out[form] = rows
    return out


def oracle_residual(x, y, alpha, beta, sigma2: float) -> float:
    """||y - H beta - (K + sigma2 I) alpha|| / ||y|| with the oracle's dense product."""
    import oracle
    oracle.build(force=False)
    ka = oracle.mvm(x, alpha, TWO_NU, "product", ELL)
    res = y - oracle.design_matrix(x) @ np.asarray(beta) - ka - sigma2 * alpha
    return float(np.linalg.norm(res) / np.linalg.norm(y))


def bench_solve(mm, p, dev, reps: int, maxit: int, check_oracle: bool):
    """Configuration 2's GP regression: plan, CG + GLS to 1e-8, predict 1000 points."""
    import torch
    x = torch.as_tensor(p.x, device=dev)
    y = torch.as_tensor(p.y, device=dev)
    z = torch.as_tensor(np.random.default_rng(20021).uniform(0.0, 1.0, size=(NPREDICT, D)), device=dev)
    kern = mm.Kernel(TWO_NU, "product", ELL, 1.0)
    from paper_2508_01864_amd import autotune
    tp = mm.Plan(x, kern)
    sched = autotune.tune_schedule(tp, 4)       # the solver's width (y, 1, x1, x2); cached for the plans below
    tp.close()
    best = None
    for r in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = mm.Plan(x, kern)
        autotune.tune_schedule(plan, 4)          # a cache hit: sets the tuned schedule
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        alpha, beta, info = plan.cg_solve(y, SIGMA2, fixed_effects=True, rtol=RTOL, maxit=maxit,
                                          raise_on_error=maxit >= 20000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        mean = plan.predict(alpha, z, beta=beta)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        plan.close()
        rec = {"plan_build_s": t1 - t0, "solve_s": t2 - t1, "predict_s": t3 - t2, "total_s": t3 - t0,
               "iters": info["iters"], "status": info["status"], "relres_recurrence": info["relres_max"],
               "true_relres_library": info["true_relres"],
               "per_iteration_ms": (t2 - t1) / max(info["iters"], 1) * 1e3}
        log("solve %d: %d iterations, %.3f s, library residual %.3e" % (r, info["iters"], t2 - t1,
                                                                        info["true_relres"]))
        if best is None or rec["total_s"] < best["total_s"]:
            best = rec
            best_out = (alpha, beta, mean)
    if check_oracle:
        t0 = time.perf_counter()
        best["true_relres_oracle"] = oracle_residual(p.x, p.y, best_out[0].cpu().numpy(), best_out[1], SIGMA2)
        log("oracle residual %.4e (%.1f s)" % (best["true_relres_oracle"], time.perf_counter() - t0))
    best["workload"] = ("d=2 N=%d nu=3/2 product ell=0.1 sigma2=0.01: plan build, CG + GLS (fixed effects "
                        "1, x1, x2) to 1e-8, predict %d points" % (N, NPREDICT))
    best["points_per_s"] = N * (1 + 4 * best["iters"]) / best["total_s"]
    best["schedule_width4"] = list(sched)
    return best


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
    (plan and preconditioner build included), and the library's recomputed residual."""
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
            if pc is not None:
                pc.close()
            plan.close()
            rec = {"iters": info["iters"], "setup_s": t1 - t0, "solve_s": t2 - t1, "total_s": t2 - t0,
                   "true_relres": info["true_relres"]}
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


def c3_solve(mm, plan, y, rank, maxit, sched, chunk=500):
    """The configuration-3 single solve: CG (preconditioned with the rank-`rank`
    pivoted Cholesky when rank > 0) on (K + 0.01 I) alpha = y to rtol 1e-8,
    advanced in chunks of `chunk` iterations with a progress line per chunk.  A
    column that converges by its recurrence has its residual recomputed with a
    fresh product (mm_solver_check); the solve ends when that residual meets
    rtol, or at maxit."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pc = mm.Precond(plan, max_rank=rank) if rank > 0 else None
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s = mm.Solver(plan, y, 0.01, rtol=1e-8, precond=pc)
    it = 0
    while it < maxit:
        k = min(chunk, maxit - it)
        s.iterate(k)
        it += k
        act, brk, info = s.poll()
        log("config 3 CG: %d iterations, recurrence residual %.3e, %.1f s" %
            (it, info["relres_max"], time.perf_counter() - t1))
        if act == 0:
            passed, _ = s.check(tighten=True)
            if passed:
                break
        if brk:
            break
    _, _, info = s.finish(raise_on_error=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.close()
    if pc is not None:
        pc.close()
    return {"method": "pcg rank %d" % rank if rank > 0 else "cg", "rtol": 1e-8, "schedule": list(sched),
            "precond_s": t1 - t0, "solve_s": t2 - t1, "iters": info["iters"], "maxit": maxit,
            "status": info["status"], "relres_recurrence": info["relres_max"],
            "true_relres": info["true_relres"], "per_iteration_ms": (t2 - t1) / max(info["iters"], 1) * 1e3,
            "polls_every": chunk}


def bench_config3(dev, steps, rank, maxit):
    """d=3, N=500k, nu=5/2, lengthscale 0.3, x ~ N(0, I): one product with the 32
    Rademacher probes (product and L1 forms, median of 3), the stochastic
    log-determinant from those probes (`steps` Lanczos steps), and one CG solve
    of the sin/cos targets (sigma2 0.01, rtol 1e-8, at most `maxit` iterations;
    preconditioned with the rank-`rank` pivoted Cholesky when rank > 0)."""
    import torch
    import paper_2508_01864_amd as mm
    from paper_2508_01864_amd import autotune
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
        sched = autotune.tune_schedule(plan, 32, reps=1, vectors=Zc)
        plan.mvm_raw(Zc, Yc, 32)
        ms = median_ms(lambda: plan.mvm_raw(Zc, Yc, 32), 3)
        Lp = mm.passes(n, 3)
        ba = float(n) * (8.0 * 3 + 16.0 * 32 + Lp * (4.0 + 16.0 * 32))
        out[form] = {"plan_build_s": tb, "mvm32_ms": ms, "points_per_s": n * 32 / (ms * 1e-3), "schedule": list(sched),
                     "b_alg_bytes": ba, "frac_hbm_peak": ba / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
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
            s1 = autotune.tune_schedule(plan, 1, reps=5)       # the single column's schedule
            out["cg_solve"] = c3_solve(mm, plan, y, rank, maxit, s1)
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


SERVED_N_HI = 30_000
SERVED_RANK = 64


def bench_served(dev, count, rates):
    """A bounded sample of the served stream against plain first-come-first-served
    solves, at several arrival rates (multiples of the plain path's measured
    capacity).  The sample is the first `count` requests of the configuration-5
    stream with N log-uniform in [5e3, 3e4] (instead of [5e3, 3e5]), each solved
    by rank-64 preconditioned CG on both paths."""
    import torch
    import paper_2508_01864_amd as mm
    from paper_2508_01864_amd import serve
    import workloads
    probs = workloads.config5(count=count, rate=1.0, n_hi=SERVED_N_HI)
    base = [p.arrival for p in probs]          # unit-rate Poisson arrival times
    reqs = [serve.Request(k, 0.0, p.x, p.y, mm.Kernel(p.two_nu, p.form, p.ell), p.sigma2, p.z,
                          rtol=1e-8, maxit=20000, precond_rank=SERVED_RANK) for k, p in enumerate(probs)]
    # plain service times (all requests back to back) give the plain capacity
    plain0 = serve.run_plain(reqs)
    service = [r.done - r.admitted for r in plain0]
    cap = len(reqs) / sum(service)
    log("served: plain capacity %.2f solves/s over %d requests" % (cap, len(reqs)))
    out = {
        "workload": "first %d requests of the served stream with N log-uniform [5e3, %d] (bounded sample; the "
                    "stream's own range is [5e3, 3e5]), d/nu uniform, sigma2 log-uniform [1e-3, 1e-1], affine "
                    "trend + sin/cos field, fixed effects, rank-%d pivoted Cholesky PCG to rtol 1e-8, 1000 "
                    "predict points; Poisson arrivals at the given multiples of the plain path's measured "
                    "capacity" % (count, SERVED_N_HI, SERVED_RANK),
        "requests": count, "n": [len(r.y) for r in reqs], "d": [int(r.x.shape[1]) for r in reqs],
        "plain_capacity_per_s": cap,
        "plain_latency_note": "plain-path latencies follow from the measured service times by the "
                              "first-come-first-served recursion on the same arrivals",
        "rates": {},
    }
    for mult in rates:
        rate = mult * cap
        for r, a in zip(reqs, base):
            r.arrival = a / rate
        free_at = 0.0
        plain = []
        for r, sv in zip(reqs, service):
            start = max(free_at, r.arrival)
            free_at = start + sv
            plain.append(serve.Response(r.rid, r.arrival, start, free_at, None, None, None, {}))
        srv = serve.Server(chunk=16)
        served = srv.run(reqs)
        same = all(torch.equal(a.alpha, b.alpha) and torch.equal(a.mean, b.mean) for a, b in zip(served, plain0))
        sp, ss = serve.summary(plain), serve.summary(served)
        log("served at %.1fx capacity: p50 %.3f s p99 %.3f s (plain %.3f / %.3f), %.2f vs %.2f solves/s" %
            (mult, ss["p50_s"], ss["p99_s"], sp["p50_s"], sp["p99_s"], ss["solves_per_s"], sp["solves_per_s"]))
        out["rates"]["%.1f" % mult] = {
            "rate_per_s": rate, "plain": sp, "served": ss, "served_bitwise_equal_alone": bool(same),
            "server": {"ticks": srv.ticks, "rebuilds": srv.rebuilds, "peak_slots": srv.peak_slots,
                       "peak_bytes": srv.peak_bytes, "budget_bytes": srv.budget}}
    out["iters"] = [r.info["iters"] for r in plain0]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--warmup-seconds", type=float, default=1.0,
                    help="keep warming up (untimed) until this much time has passed")
    ap.add_argument("--nrhs", type=int, default=32, help="right-hand sides of the headline product")
    ap.add_argument("--mvm-reps", type=int, default=21)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mvm", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-oracle-residual", action="store_true")
    ap.add_argument("--batched-count", type=int, default=256)
    ap.add_argument("--batched-iters", type=int, default=32)
    ap.add_argument("--served-count", type=int, default=32)
    ap.add_argument("--served-rates", type=str, default="0.5,0.9,1.2")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-config3", action="store_true")
    ap.add_argument("--logdet-steps", type=int, default=30)
    ap.add_argument("--lml-probes", type=int, default=31,
                    help="probes of the likelihood-gradient section (0: skip the section)")
    ap.add_argument("--pcg-rank", type=int, default=100,
                    help="rank of the pivoted Cholesky preconditioner of the extra PCG section (0: skip)")
    ap.add_argument("--c3-rank", type=int, default=0,
                    help="preconditioner rank of the configuration-3 solve (0: plain CG; rank 256 "
                         "saves no iterations on this kernel matrix)")
    ap.add_argument("--c3-maxit", type=int, default=8000)
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
    x = torch.as_tensor(p.x, device=dev)
    kern = mm.Kernel(TWO_NU, "product", ELL, 1.0)
    L = mm.levels(N)
    R = args.nrhs

    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * 131072, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written per launch" % (args.calib_copy_mib, args.calib_copy_mib))
        del src, dst

    # plan build, timed on its own (median of three)
    builds = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = mm.Plan(x, kern)
        torch.cuda.synchronize()
        builds.append(time.perf_counter() - t0)
        plan.close()
    plan_build_s = float(np.median(builds))
    log("plan build %.4f s" % plan_build_s)

    # the headline: one product with R columns per step, on the schedule the
    # autotuner picks for this width (tuning runs before the timed region)
    from paper_2508_01864_amd import autotune
    plan = mm.Plan(x, kern)
    vv = torch.as_tensor(np.random.default_rng(7 + R).standard_normal((R, N)), device=dev)
    yy = torch.empty_like(vv)
    head_sched = autotune.tune_schedule(plan, R, vectors=vv)
    log("headline schedule (columns per wave, run length, stored run carries): %s" % (head_sched,))
    # untimed warm-up: the W steps, continued until the GPU has run the product for
    # at least --warmup-seconds (its clocks settle; a schedule read from the tuning
    # cache skips the tuning runs that otherwise warm it)
    t0 = time.perf_counter()
    done = 0
    while done < args.warmup or time.perf_counter() - t0 < args.warmup_seconds:
        plan.mvm_raw(vv, yy, R)
        done += 1
        if done % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    log("warm-up: %d products in %.2f s; timed steps: %d" % (done, time.perf_counter() - t0, args.steps))
    plan.profile_enable(True)
    plan.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.mvm_raw(vv, yy, R)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sms, scnt, _ = plan.profile_read(reset=True)
    plan.profile_enable(False)
    plan.close()
    value = N * R * args.steps / elapsed
    avg_launch_ms = sms / max(scnt, 1)
    bytes_launch = L * b_pass(N, R)
    achieved = bytes_launch / (avg_launch_ms * 1e-3) / 1e9 if scnt else 0.0
    log("headline: %.4f ms per product, %.3e points/s; main sweep %.4f ms, %.0f GB/s" %
        (elapsed / args.steps * 1e3, value, avg_launch_ms, achieved))

    copy_gbs = stream_copy_gbs(dev)
    log("device copy: %.0f GB/s (read + write)" % copy_gbs)

    mvm_rows = None
    if not args.no_mvm:
        mvm_rows = bench_mvm(mm, x, dev, args.mvm_reps, copy_gbs)

    solve_out = None
    if not args.no_solve:
        solve_out = bench_solve(mm, p, dev, 2, args.maxit, not args.no_oracle_residual)

    pcg_out = None
    if args.pcg_rank > 0:
        log("preconditioned solve: rank %d" % args.pcg_rank)
        pcg_out = bench_pcg(mm, x, torch.as_tensor(p.y, device=dev), kern, args.pcg_rank)

    grad_out = None
    if args.lml_probes > 0:
        log("gradient: dK/dl products and the likelihood with %d probes" % args.lml_probes)
        grad_out = bench_gradient(mm, x, torch.as_tensor(p.y, device=dev), kern, args.lml_probes, args.mvm_reps)

    c3_out = None
    if not args.no_config3:
        log("config 3: d=3 N=500k nu=5/2, 32 probes")
        c3_out = bench_config3(dev, args.logdet_steps, args.c3_rank, args.c3_maxit)

    batched_out = None
    if not args.no_batched:
        log("batched: %d problems" % args.batched_count)
        batched_out = bench_batched(dev, args.batched_count, args.batched_iters)
    served_out = None
    if not args.no_served and args.served_count > 0:
        log("served: %d requests" % args.served_count)
        served_out = bench_served(dev, args.served_count, [float(r) for r in args.served_rates.split(",")])

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(p.x, R, args.cpu_seconds)

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
        "config": {"workload": "matern_mvm y = K v, d=2 N=100000 nu=3/2 product form ell=0.1, "
                               "x ~ U[0,1]^2, %d right-hand sides, plan prebuilt" % R,
                   "n": N, "d": D, "two_nu": TWO_NU, "form": "product", "lengthscale": ELL, "nrhs": R,
                   "schedule": {"columns_per_wave": head_sched[0], "run_length": head_sched[1],
                                "stored_run_carries": autotune.stores_run_carries(D, autotune.product_width(R),
                                                                                  *head_sched),
                                "chosen_by": "autotune.tune_schedule"}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(),
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "kernel": "main divide-and-conquer sweep launch of the headline product "
                               "(d=2, nu=3/2, product, %d columns; all %d passes per launch)" % (R, L),
                     "avg_launch_ms": avg_launch_ms, "launches": scnt,
                     "whole_product_frac": b_alg(N, D, R, L) / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS},
        "cpu_baseline": cpu,
        "plan_build_s": plan_build_s,
        "stream_copy_gbs": copy_gbs,
        "mvm": mvm_rows,
        "solve": solve_out,
        "pcg": pcg_out,
        "gradient": grad_out,
        "config3": c3_out,
        "batched": batched_out,
        "served": served_out,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
