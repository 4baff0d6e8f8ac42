"""Many independent GP problems solved together.

``solve_many`` advances the conjugate-gradient solvers of many problems
(uneven n, d, nu, lengthscale, noise) in shared launches: each iteration of a
:class:`SolverBatch` runs every problem's kernel product in one launch per
kernel configuration and sweep phase, and every CG vector update in one launch
per step, replayed from a HIP graph.  Solvers that converge are dropped from
the batch once they make up a set fraction of its work, so finished problems
stop costing launches.  A problem's iterates do not depend on its batch-mates:
the result equals gp_cg_solve on that problem alone, bit for bit (a solver
that converges by its recurrence has its residual recomputed and, if that
misses rtol, restarts with tighter tolerances, exactly as gp_cg_solve does).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

from . import Plan, Solver, SolverBatch, passes, autotune


@dataclass
class SolveResult:
    alpha: object
    beta: object
    info: dict
    iters_batched: int = 0         # batch iterations the solver took part in
    done_at_s: float = 0.0         # seconds from the start of solve_many


def work_units(n: int, d: int, width: int) -> int:
    """Relative cost of one product: points x passes x columns."""
    return max(n, 1) * max(passes(n, d), 1) * width


def solver_width(d: int, fixed_effects: bool) -> int:
    ncols = d + 2 if fixed_effects else 1
    w = 1
    base = 1 if ncols < 2 else (2 if ncols < 4 else 4)
    while w < max(ncols, base):
        w <<= 1
    return w


def batch_key(plans: List[Plan], fixed_effects: bool) -> str:
    return autotune.signature("solver", [(p.n, p.d, p.kernel.two_nu, p.kernel.form,
                                          solver_width(p.d, fixed_effects)) for p in plans])


def solve_many(plans: List[Plan], ys, sigma2s, fixed_effects: bool = False, rtol: float = 1e-8,
               maxit: int = 20000, chunk: int = 16, use_graph: bool = True, tune: bool = True,
               rebuild_frac: float = 0.25) -> List[SolveResult]:
    """Solve (K_k + sigma2_k I) alpha_k = y_k - H_k beta_k for every problem k.

    ``chunk`` iterations run between polls; ``rebuild_frac`` is the share of
    the batch's work that finished solvers must reach before the batch is
    rebuilt without them."""
    t0 = time.perf_counter()
    solvers = [Solver(p, y, s2, fixed_effects=fixed_effects, rtol=rtol)
               for p, y, s2 in zip(plans, ys, sigma2s)]
    works = [work_units(p.n, p.d, solver_width(p.d, fixed_effects)) for p in plans]
    active = list(range(len(solvers)))
    finished = [False] * len(solvers)
    taken = [0] * len(solvers)
    done_at = [0.0] * len(solvers)
    batch: Optional[SolverBatch] = None
    members: List[int] = []
    try:
        while active:
            if batch is None:
                members = list(active)
                batch = SolverBatch([solvers[i] for i in members], use_graph=use_graph)
                if tune and min(taken[i] for i in members) + 32 <= maxit:
                    steps = [0]

                    def one_step(b=batch):
                        b.iterate(1)
                        steps[0] += 1
                    autotune.tune(batch, batch_key([plans[i] for i in members], fixed_effects), one_step, reps=1)
                    for i in members:       # tuning iterations are real iterations
                        taken[i] += steps[0]
            k = min(chunk, maxit - min(taken[i] for i in members))
            if k <= 0:
                break
            batch.iterate(k)
            status = batch.poll()
            now = time.perf_counter() - t0
            for i, st in zip(members, status):
                taken[i] += k
                if finished[i]:
                    continue
                if st == 0 and taken[i] < maxit:
                    # converged by the recurrence: recompute the residual; a miss
                    # restarts the solver with tighter tolerances (it stays active)
                    passed, _ = solvers[i].check(tighten=True)
                    if not passed:
                        continue
                if st <= 0 or taken[i] >= maxit:
                    finished[i] = True
                    done_at[i] = now
            active = [i for i in members if not finished[i]]
            done_work = sum(works[i] for i in members if finished[i])
            if active and done_work >= rebuild_frac * sum(works[i] for i in members):
                batch.close()
                batch = None
            elif not active:
                break
    finally:
        if batch is not None:
            batch.close()
    out = []
    for i, s in enumerate(solvers):
        alpha, beta, info = s.finish(raise_on_error=False)
        out.append(SolveResult(alpha, beta, info, taken[i], done_at[i]))
        s.close()
    return out
