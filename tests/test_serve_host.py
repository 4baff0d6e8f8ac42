"""Host-side logic of the server and the autotuner cache (no GPU)."""
import json

import numpy as np

import paper_2508_01864_amd as mm
from paper_2508_01864_amd import autotune, serve
from paper_2508_01864_amd.batched import solver_width


def test_request_bytes_grow_with_size_and_dimension():
    k = mm.Kernel(3, "product", 0.1)
    b = [serve.request_bytes(n, 2, 1000, k) for n in (5_000, 50_000, 300_000)]
    assert 0 < b[0] < b[1] < b[2]
    assert serve.request_bytes(50_000, 3, 1000, k) > b[1]
    # a request's bound covers at least its plan and its CG vectors
    assert b[1] >= mm.footprint_bytes(50_000, 2, 1, k) + 6 * 50_000 * 4 * 8


def test_solver_footprint_host_only():
    k = mm.Kernel(5, "product", 0.2)
    assert mm.solver_footprint_bytes(0, 2, True, k) == 0
    assert mm.solver_footprint_bytes(10, 4, True, k) == 0
    a = mm.solver_footprint_bytes(100_000, 2, False, k)
    b = mm.solver_footprint_bytes(100_000, 2, True, k)
    assert 0 < a < b


def test_solver_width_matches_library_rule():
    assert [solver_width(d, False) for d in (1, 2, 3)] == [1, 1, 1]
    assert [solver_width(d, True) for d in (1, 2, 3)] == [4, 4, 8]


def test_summary_percentiles():
    rs = [serve.Response(i, float(i), float(i), float(i) + lat, None, None, None, {})
          for i, lat in enumerate([1.0, 2.0, 3.0, 4.0, 100.0])]
    s = serve.summary(rs)
    assert s["p50_s"] == 3.0
    assert 4.0 < s["p99_s"] <= 100.0
    assert abs(s["span_s"] - 104.0) < 1e-12
    assert abs(s["solves_per_s"] - 5 / 104.0) < 1e-12


def test_autotune_signature_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("MM_TUNE_CACHE", str(tmp_path / "c.json"))
    key = autotune.signature("solver", [(1000, 2, 3, "product", 4), (3000, 3, 5, "product", 8)])
    assert key.startswith("solver|") and "d2.nu3.product.w4" in key and "d3.nu5.product.w8" in key
    assert autotune.cached(key) is None

    class Fake:
        def __init__(self):
            self.sched = None

        def set_schedule(self, a, b):
            self.sched = (a, b)

    autotune._store(key, (4, 512), {"x": 1.0})
    f = Fake()
    assert autotune.tune(f, key, lambda: None) == (4, 512)
    assert f.sched == (4, 512)
    assert json.load(open(tmp_path / "c.json"))[key]["schedule"] == [4, 512]
