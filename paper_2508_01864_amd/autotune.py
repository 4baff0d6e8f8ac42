"""Launch-schedule autotuner for batched products and solver batches.

A batch runs persistent grids whose size is a free parameter: the workgroups
per compute unit of the carry-scan launches and the grid of the vector-update
(or gather/scatter) launches.  (The sweep launches run one workgroup per work
item and take no grid parameter.)  Results never depend on them (every work item runs
the same arithmetic), so tuning only changes speed.  The tuner times each
candidate with HIP events on the caller's stream, keeps the fastest, and
caches the choice in a JSON file keyed by the batch's shape (its kernel
classes, column widths and size buckets).

The cache file is ``$MM_TUNE_CACHE`` if set, else ``_tune_cache.json`` next to
this module.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_WG_PER_CU = (1, 4, 16)
SIDE_GRID = (512, 2048, 8192)
DEFAULT = (16, 2048)


def cache_path() -> str:
    return os.environ.get("MM_TUNE_CACHE", os.path.join(_HERE, "_tune_cache.json"))


def _load() -> Dict[str, list]:
    try:
        with open(cache_path()) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(key: str, value: Tuple[int, int], timings: Dict[str, float]):
    data = _load()
    data[key] = {"schedule": list(value), "ms": timings}
    tmp = cache_path() + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path())


def signature(kind: str, members: Iterable[Tuple[int, int, int, str, int]]) -> str:
    """Cache key of a batch: kind ('solver' or 'mvm'), the sorted set of
    (d, two_nu, form, width) classes, and log2 buckets of the problem count
    and of the total number of points."""
    members = list(members)
    classes = sorted(set((d, t, f, w) for (_, d, t, f, w) in members))
    ntot = sum(m[0] for m in members)
    return "%s|k%d|N%d|%s" % (kind, int(round(math.log2(max(len(members), 1)))),
                              int(round(math.log2(max(ntot, 1)))),
                              ";".join("d%d.nu%d.%s.w%d" % c for c in classes))


def cached(key: str):
    """The cached schedule of a batch shape, or None."""
    hit = _load().get(key)
    return tuple(int(v) for v in hit["schedule"]) if hit else None


def _time(step: Callable[[], None], reps: int) -> float:
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(batch, key: str, step: Callable[[], None], reps: int = 2,
         sweep_candidates: Sequence[int] = SWEEP_WG_PER_CU,
         side_candidates: Sequence[int] = SIDE_GRID, use_cache: bool = True) -> Tuple[int, int]:
    """Pick (carry-scan workgroups per CU, side grid) for ``batch`` (an
    MvmBatch or SolverBatch: anything with ``set_schedule``) by timing ``step``
    (one or a few batch launches).  The carry parameter is tuned first with the
    default side grid, then the side grid with the chosen carry parameter."""
    if use_cache:
        hit = _load().get(key)
        if hit:
            sched = tuple(int(v) for v in hit["schedule"])
            batch.set_schedule(*sched)
            return sched
    timings: Dict[str, float] = {}
    best_wg, best_t = DEFAULT[0], float("inf")
    batch.set_schedule(DEFAULT[0], DEFAULT[1])
    step()  # graph capture and first touch outside the timings
    for wg in sweep_candidates:
        batch.set_schedule(wg, DEFAULT[1])
        step()
        t = _time(step, reps)
        timings["wg%d/g%d" % (wg, DEFAULT[1])] = t
        if t < best_t:
            best_wg, best_t = wg, t
    best_g = DEFAULT[1]
    for g in side_candidates:
        if g == DEFAULT[1]:
            continue
        batch.set_schedule(best_wg, g)
        step()
        t = _time(step, reps)
        timings["wg%d/g%d" % (best_wg, g)] = t
        if t < best_t:
            best_g, best_t = g, t
    batch.set_schedule(best_wg, best_g)
    if use_cache:
        _store(key, (best_wg, best_g), timings)
    return best_wg, best_g


# ---------------------------------------------------------------------------
# Scan schedules of a plan's products (mm_plan_set_schedule): the column block
# of a wavefront, the run length of a lane (hence the tile length) and whether
# the tile-aggregate pre-pass stores the runs' within-tile carries.  They change
# the launch shapes and the order in which tiles join, never the exact result
# (only its rounding), and they are chosen per (d, nu, form, size bucket,
# width) by timing the product at that width.
# ---------------------------------------------------------------------------
BASE_SCHEDULES = ((1, 4), (2, 8), (4, 16), (4, 32), (32, 128))
TUNED_SCHEDULES = ((1, 8), (1, 16), (4, 8), (8, 16), (8, 32), (16, 32), (16, 64), (32, 64))


def rhs_block(nrhs: int) -> int:
    """The library's default column block for nrhs right-hand sides."""
    return 32 if nrhs >= 32 else (4 if nrhs >= 4 else (2 if nrhs >= 2 else 1))


def product_width(nrhs: int) -> int:
    """Padded width of a product with nrhs right-hand sides (matern_mvm's rule)."""
    r = rhs_block(nrhs)
    return (nrhs + r - 1) // r * r


def schedule_candidates(d: int, two_nu: int, form: str, width: int) -> List[Tuple[int, int, int]]:
    """(wb, e, runex) schedules compiled for the kernel class at this width."""
    tuned = form == "product" and ((d == 2 and two_nu == 3) or (d == 3 and two_nu == 5))
    pairs = list(BASE_SCHEDULES) + (list(TUNED_SCHEDULES) if tuned else [])
    out = []
    for wb, e in pairs:
        if width % wb:
            continue
        stores = d <= 2 and wb >= 2 and e <= 32   # the pre-pass can store run carries
        for rx in ((1, 0) if stores else (1,)):
            out.append((wb, e, rx))
    return out


def stores_run_carries(d: int, width: int, wb: int, e: int, runex) -> bool:
    """Whether a product at padded width `width` on schedule (wb, e, runex)
    stores the runs' within-tile carries in its pre-pass: d <= 2, at least 2
    columns per wave and runs of 8 to 32 (the lane keeps its run's sums in
    registers)."""
    return bool(runex) and d <= 2 and wb >= 2 and 4 < e <= 32


def schedule_key(n: int, d: int, two_nu: int, form: str, width: int) -> str:
    return "sched|d%d.nu%d.%s|N%d|w%d" % (d, two_nu, form, int(round(math.log2(max(n, 1)))), width)


def _median_ms(step: Callable[[], None], reps: int) -> float:
    import torch
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune_schedule(plan, nrhs: int, reps: int = 5, use_cache: bool = True, vectors=None):
    """Pick the scan schedule of ``plan``'s products at nrhs right-hand sides
    (its padded width) by timing matern_mvm under each compiled candidate,
    set it on the plan, and return (wb, e, runex).  Cached by
    (d, nu, form, log2 n, width)."""
    import torch
    import numpy as np
    width = product_width(nrhs)
    k = plan.kernel
    key = schedule_key(plan.n, plan.d, k.two_nu, k.form, width)
    if use_cache:
        hit = _load().get(key)
        if hit:
            sc = tuple(int(v) for v in hit["schedule"])
            plan.set_schedule(width, *sc)
            return sc
    dev = torch.device("cuda", torch.cuda.current_device())
    if vectors is None:
        vc = torch.as_tensor(np.random.default_rng(0).standard_normal((nrhs, plan.n)), device=dev)
    else:
        vc = vectors
    yc = torch.empty_like(vc)
    timings: Dict[str, float] = {}
    best, best_t = None, float("inf")
    for wb, e, rx in schedule_candidates(plan.d, k.two_nu, k.form, width):
        plan.set_schedule(width, wb, e, bool(rx))
        plan.mvm_raw(vc, yc, nrhs)          # first touch of the workspaces outside the timing
        t = _median_ms(lambda: plan.mvm_raw(vc, yc, nrhs), reps)
        timings["wb%d/e%d/rx%d" % (wb, e, rx)] = t
        if t < best_t:
            best, best_t = (wb, e, rx), t
    plan.set_schedule(width, *best)
    if use_cache:
        _store(key, best, timings)
    return best
