"""Serving GP regressions with continuous batching.

Requests (points x, targets y, noise sigma^2, kernel, prediction points z)
arrive over time.  The server keeps every admitted request's stored sorting
outputs (its plan) and conjugate-gradient state resident on the GPU and
advances all of them together: each tick runs ``chunk`` iterations of one
:class:`SolverBatch` over the admitted requests (their kernel products share
launches), then polls.  Finished requests leave (their GLS estimate and
posterior mean at z are computed, their memory is released) and waiting
requests are admitted in arrival order as slots and device memory free up.
A request admitted while a chunk is in flight has its plan, preconditioner
and solver created on a side stream, beside that chunk; it joins the batch
when the chunk's poll returns.
Admission is by device footprint: the plan, the solver, the optional
pivoted Cholesky preconditioner and the temporary prediction plan of a
request are bounded on the host before anything is allocated, and a request is admitted only while the sum over admitted
requests stays within the memory budget.

Every request's result equals what gp_cg_solve + gp_predict give for it alone
(bitwise): a solver's arithmetic does not depend on its batch-mates.

Time.  ``run`` uses a clock that follows the wall clock while the GPU has
work, and jumps forward to the next arrival when the server is idle instead
of sleeping, so a run's latencies are those of a real-time server without
its idle waits.  ``run_plain`` serves the same stream one request at a time
(first come, first served, gp_cg_solve then gp_predict) for comparison.
"""
from __future__ import annotations

import collections
import os
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import (Kernel, Plan, Precond, Solver, SolverBatch, autotune, footprint_bytes,
               solver_footprint_bytes)
from .batched import batch_key


@dataclass
class Request:
    rid: int
    arrival: float            # seconds from the start of the stream
    x: np.ndarray             # (n, d)
    y: np.ndarray             # (n,)
    kernel: Kernel
    sigma2: float
    z: np.ndarray             # (m, d) prediction points
    rtol: float = 1e-8
    maxit: int = 20000
    precond_rank: int = 0     # rank of the pivoted Cholesky preconditioner (0: plain CG)


@dataclass
class Response:
    rid: int
    arrival: float
    admitted: float
    done: float
    alpha: object             # device tensor (n,)
    beta: np.ndarray
    mean: object              # device tensor (m,)
    info: dict

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def request_bytes(n: int, d: int, m: int, kernel: Kernel, precond_rank: int = 0) -> int:
    """Device-memory bound of one request: its plan, its solver (fixed
    effects), its input copies, the temporary plan of the prediction and its
    preconditioner (the n x rank factor, the preconditioned solver's vectors and
    the Woodbury factors)."""
    b = footprint_bytes(n, d, 1, kernel) + solver_footprint_bytes(n, d, True, kernel)
    b += 8 * (n * (d + 1) + m * (d + 1))
    b += footprint_bytes(n + m, d, 1, kernel) + 8 * (n + m) * (d + 2)
    if precond_rank > 0:
        k = min(precond_rank, n)
        b += 8 * n * k + 8 * (2 * n * 8 + 1024 * 8 * (2 + 2 * k) + 4 * k * k) + (1 << 20)
    return b


def default_budget() -> int:
    """Admission budget in bytes: $MM_SERVE_HBM_BYTES, else 3/4 of the free
    device memory."""
    env = os.environ.get("MM_SERVE_HBM_BYTES")
    if env:
        return int(float(env))
    import torch
    free, _ = torch.cuda.mem_get_info()
    return int(free * 3 // 4)


def percentile(vals, q) -> float:
    return float(np.percentile(np.asarray(vals, dtype=np.float64), q)) if len(vals) else float("nan")


def summary(resps: List[Response]) -> dict:
    lat = [r.latency for r in resps]
    span = max(r.done for r in resps) - min(r.arrival for r in resps) if resps else 0.0
    return {"requests": len(resps), "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "mean_s": float(np.mean(lat)) if lat else float("nan"),
            "solves_per_s": len(resps) / span if span > 0 else float("nan"), "span_s": span}


class _Live:
    """An admitted request: its inputs, plan, preconditioner and solver, all
    created on ``stream`` (the server's side stream), so that their creation
    kernels run beside the iterations already in flight on the batch's own
    stream."""

    def __init__(self, req: Request, device, admitted: float, stream=None):
        import torch
        self.req = req
        self.admitted = admitted
        with torch.cuda.stream(stream) if stream is not None else _null():
            self.x = torch.as_tensor(req.x, device=device)
            self.y = torch.as_tensor(req.y, device=device)
            self.z = torch.as_tensor(req.z, device=device)
            self.plan = Plan(self.x, req.kernel, stream=stream)
            self.pc = Precond(self.plan, max_rank=req.precond_rank, stream=stream) if req.precond_rank > 0 else None
            self.solver = Solver(self.plan, self.y, req.sigma2, fixed_effects=True, rtol=req.rtol,
                                 stream=stream, precond=self.pc)
        self.iters = 0
        self.bytes = request_bytes(len(req.y), req.x.shape[1], len(req.z), req.kernel, req.precond_rank)

    def close(self):
        self.solver.close()
        if self.pc is not None:
            self.pc.close()
        self.plan.close()


class _null:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False


class Server:
    def __init__(self, budget_bytes: Optional[int] = None, max_slots: int = 64, chunk: int = 16,
                 use_graph: bool = True, tune: bool = True, device=None, side_stream: bool = True):
        import torch
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        # admissions build on their own stream (default priority) while the batch iterates
        self.side = torch.cuda.Stream(device=self.device) if side_stream else None
        self.budget = int(budget_bytes) if budget_bytes is not None else default_budget()
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.use_graph = use_graph
        self.tune = tune
        self.rebuilds = 0
        self.ticks = 0
        self.peak_bytes = 0
        self.peak_slots = 0

    def run(self, requests: List[Request], on_done=None) -> List[Response]:
        """Serve the stream; on_done(response) is called as each request finishes."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        live: Dict[int, _Live] = {}
        out: List[Response] = []
        used = 0
        batch: Optional[SolverBatch] = None
        members: List[int] = []
        wall0 = time.perf_counter()
        skipped = 0.0

        def now() -> float:
            return time.perf_counter() - wall0 + skipped

        def admit(room: int):
            """Admit queued requests in arrival order while slots and memory allow."""
            nonlocal used
            got = []
            while queue and len(live) + len(got) < min(room, self.max_slots):
                r = queue[0]
                need = request_bytes(len(r.y), r.x.shape[1], len(r.z), r.kernel, r.precond_rank)
                if need > self.budget:
                    raise RuntimeError("request %d needs %d bytes, more than the whole budget %d"
                                       % (r.rid, need, self.budget))
                if used + need > self.budget:
                    break
                queue.popleft()
                got.append(_Live(r, self.device, now(), stream=self.side))
                used += need
            return got

        new: List[_Live] = []
        try:
            while pending or queue or live:
                t = now()
                while pending and pending[0].arrival <= t:
                    queue.append(pending.popleft())
                if not live:
                    for lv in admit(self.max_slots):
                        live[lv.req.rid] = lv
                    self.peak_bytes = max(self.peak_bytes, used)
                    self.peak_slots = max(self.peak_slots, len(live))
                    if not live:
                        # idle: jump to the next arrival
                        if pending:
                            skipped += max(0.0, pending[0].arrival - now())
                        continue
                if batch is None:
                    members = sorted(live)
                    batch = SolverBatch([live[i].solver for i in members], use_graph=self.use_graph)
                    self.rebuilds += 1
                    if self.tune:
                        # schedules tuned earlier for a batch of this shape; no timing runs here
                        sched = autotune.cached(batch_key([live[i].plan for i in members], True))
                        if sched:
                            batch.set_schedule(*sched)
                k = min([self.chunk] + [live[i].req.maxit - live[i].iters for i in members])
                k = max(k, 1)
                if self.side is not None:
                    # creation, check and restart work of the solvers was queued on the side
                    # stream; the batch runs on its own stream, ordered after this point
                    self.side.synchronize()
                batch.iterate(k)
                # requests that arrived meanwhile are admitted (plans built on the side
                # stream) while the chunk runs; they join the batch at its next rebuild
                new = admit(self.max_slots)
                status = batch.poll()
                self.ticks += 1
                finished = []
                for i, st in zip(members, status):
                    live[i].iters += k
                    if st == 0 and live[i].iters < live[i].req.maxit:
                        # converged by the recurrence: the recomputed residual decides
                        passed, _ = live[i].solver.check(tighten=True)
                        if not passed:
                            continue
                    if st <= 0 or live[i].iters >= live[i].req.maxit:
                        finished.append(i)
                if finished or new:
                    batch.close()
                    batch = None
                for i in finished:
                    lv = live.pop(i)
                    alpha, beta, info = lv.solver.finish(raise_on_error=False)
                    mean = lv.plan.predict(alpha, lv.z, beta=beta)
                    lv.close()
                    out.append(Response(i, lv.req.arrival, lv.admitted, now(), alpha, beta, mean, info))
                    used -= lv.bytes
                    if on_done is not None:
                        on_done(out[-1])
                for lv in new:
                    live[lv.req.rid] = lv
                new = []
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_slots = max(self.peak_slots, len(live))
        finally:
            if batch is not None:
                batch.close()
            for lv in list(live.values()) + [lv for lv in new if lv.req.rid not in live]:
                lv.close()
        return sorted(out, key=lambda r: r.rid)


def run_plain(requests: List[Request], device=None, on_done=None) -> List[Response]:
    """Serve the stream one request at a time in arrival order (the plain
    path): plan, gp_cg_solve with fixed effects, gp_predict.  Service times are
    measured; a request starts when it has arrived and the previous one is
    done, as in a real-time first-come-first-served server."""
    import torch
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = []
    free_at = 0.0
    for r in sorted(requests, key=lambda q: q.arrival):
        start = max(free_at, r.arrival)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = torch.as_tensor(r.x, device=dev)
        y = torch.as_tensor(r.y, device=dev)
        z = torch.as_tensor(r.z, device=dev)
        plan = Plan(x, r.kernel)
        pc = Precond(plan, max_rank=r.precond_rank) if r.precond_rank > 0 else None
        alpha, beta, info = plan.cg_solve(y, r.sigma2, fixed_effects=True, rtol=r.rtol, maxit=r.maxit,
                                          raise_on_error=False, precond=pc)
        mean = plan.predict(alpha, z, beta=beta)
        torch.cuda.synchronize()
        if pc is not None:
            pc.close()
        plan.close()
        service = time.perf_counter() - t0
        free_at = start + service
        out.append(Response(r.rid, r.arrival, start, free_at, alpha, beta, mean, info))
        if on_done is not None:
            on_done(out[-1])
    return out
