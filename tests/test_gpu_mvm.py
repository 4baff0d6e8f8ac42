"""GPU parity of the exact Matern product against the dense FP64 oracle.

Every case runs the HIP path through the C ABI (via the ctypes binding) and
compares with oracle.mvm on the same seeded inputs.  Tolerance: the error of
every component relative to (K|v|)_j, and the normwise relative error, are
both <= 1e-10.
"""
import numpy as np
import pytest

import oracle
import paper_2508_01864_amd as mm
import workloads
from gpu_util import MVM_TOL, mvm_errors, say, to_gpu, to_np

pytestmark = pytest.mark.gpu
NUS = (1, 3, 5)


def run_case(x, v, two_nu, form, ell, s2=1.0, rows=None, shift=0.0, nrhs_tag=""):
    plan = mm.Plan(to_gpu(x), mm.Kernel(two_nu, form, ell, s2))
    y = to_np(plan.mvm(to_gpu(v), shift=shift))
    plan.close()
    if rows is None:
        yref, yabs = oracle.mvm(x, v, two_nu, form, ell, s2, with_abs=True)
    else:
        yref, yabs = oracle.mvm(x, v, two_nu, form, ell, s2, z=x[rows], with_abs=True,
                                shared_kernel=True)
        y = y[rows]
    yref = yref + shift * (v if rows is None else v[rows])
    yabs = yabs + abs(shift) * np.abs(v if rows is None else v[rows])
    return mvm_errors(y, yref, yabs)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("two_nu", NUS)
@pytest.mark.parametrize("form", ["l1", "product"])
def test_brute_force_tiny_with_ties(oracle_lib, d, two_nu, form):
    """N = 1..64, random and tied coordinates (duplicated points, shared values)."""
    worst = 0.0
    for n in (1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 31, 33, 64):
        for ties in (False, True):
            p = workloads.random_problem(1000 * d + 10 * two_nu + n + (500 if ties else 0), n, d,
                                         two_nu, form, 0.4, ties=ties)
            say("tiny d=%d nu=%d/2 %s n=%d ties=%s" % (d, two_nu, form, n, ties))
            comp, nrm = run_case(p.x, p.v, two_nu, form, p.ell, s2=1.3)
            worst = max(worst, comp)
            assert comp <= MVM_TOL and nrm <= MVM_TOL, (n, ties, comp, nrm)
    say("worst", worst)


def test_config1_full(oracle_lib):
    """d=1, N=2000, nu=1/2, ell=0.5 (benchmark configuration 1), full oracle."""
    p = workloads.config1()
    comp, nrm = run_case(p.x, p.v, 1, "l1", 0.5)
    say("config1", comp, nrm)
    assert comp <= MVM_TOL and nrm <= MVM_TOL


# d = 1 has one form (the two coincide), so it is listed once
TILE_CASES = [(d, n, form) for d, n in [(1, 5000), (2, 3000), (2, 5001), (3, 2500)]
              for form in (["product"] if d == 1 else ["l1", "product"])]


@pytest.mark.parametrize("d,n,form", TILE_CASES)
@pytest.mark.parametrize("two_nu", NUS)
def test_several_tiles_ragged(oracle_lib, d, n, two_nu, form):
    """Sizes spanning several 1024-position tiles, segments wider than a tile,
    and a ragged last tile; full oracle."""
    p = workloads.random_problem(77 + n + d + two_nu, n, d, two_nu, form, 0.15)
    say("tiles d=%d n=%d nu=%d/2 %s" % (d, n, two_nu, form))
    comp, nrm = run_case(p.x, p.v, two_nu, form, p.ell)
    assert comp <= MVM_TOL and nrm <= MVM_TOL, (comp, nrm)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("ell", [1e-3, 1e3])
def test_extreme_lengthscales(oracle_lib, d, ell):
    """ell = 1e-3 (global exp weights would overflow) and 1e3 (kernel ~ 1 everywhere)."""
    for two_nu in NUS:
        p = workloads.random_problem(31 + d, 1500, d, two_nu, "product", ell)
        say("ell=%g d=%d nu=%d/2" % (ell, d, two_nu))
        comp, nrm = run_case(p.x, p.v, two_nu, "product", ell)
        assert comp <= MVM_TOL and nrm <= MVM_TOL, (two_nu, comp, nrm)


@pytest.mark.parametrize("d", [2, 3])
def test_gaussian_points_l1_and_product(oracle_lib, d):
    for form in ("l1", "product"):
        p = workloads.random_problem(5 + d, 3000, d, 5, form, 0.3, dist="normal")
        say("normal d=%d %s" % (d, form))
        comp, nrm = run_case(p.x, p.v, 5, form, 0.3, s2=2.5)
        assert comp <= MVM_TOL and nrm <= MVM_TOL, (form, comp, nrm)


@pytest.mark.parametrize("nrhs", [2, 5, 12, 31])
@pytest.mark.parametrize("d,two_nu,form", [(1, 5, "product"), (2, 1, "product"), (2, 5, "product"),
                                           (2, 3, "l1")])
def test_stored_run_carry_widths(oracle_lib, nrhs, d, two_nu, form):
    """Column counts on both sides of the stored within-tile run carries (d <= 2):
    2 and 5 columns (blocks of 2 and 4, tiles of 256), 12 (tiles of 512 in d = 2) and 31
    (padded to 32 columns in blocks of 4) use them.  3001 points: 12 or 6 tiles and
    several passes whose segments span tiles."""
    p = workloads.random_problem(600 + nrhs + 10 * d + two_nu, 3001, d, two_nu, form, 0.1, nrhs=nrhs)
    say("stored run carries: nrhs=%d d=%d nu=%d/2 %s" % (nrhs, d, two_nu, form))
    comp, nrm = run_case(p.x, p.v, two_nu, form, 0.1)
    assert comp <= MVM_TOL and nrm <= MVM_TOL, (comp, nrm)


@pytest.mark.parametrize("nrhs", [2, 3, 8, 33])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_multiple_right_hand_sides(oracle_lib, nrhs, d):
    p = workloads.random_problem(400 + nrhs + d, 2100, d, 3, "product", 0.2, nrhs=nrhs)
    say("nrhs=%d d=%d" % (nrhs, d))
    comp, nrm = run_case(p.x, p.v, 3, "product", 0.2, shift=0.01)
    assert comp <= MVM_TOL and nrm <= MVM_TOL, (comp, nrm)


def test_deterministic_and_reusable_plan(oracle_lib):
    p = workloads.random_problem(9, 20000, 2, 3, "product", 0.1, nrhs=4)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.1))
    v = to_gpu(p.v)
    a = to_np(plan.mvm(v))
    b = to_np(plan.mvm(v))
    assert np.array_equal(a, b)
    # kernel change on the same stored structure
    plan.set_kernel(mm.Kernel(5, "l1", 0.2, 1.5))
    c = to_np(plan.mvm(v))
    rows = np.arange(0, 20000, 97)
    yref, yabs = oracle.mvm(p.x, p.v, 5, "l1", 0.2, 1.5, z=p.x[rows], with_abs=True,
                            shared_kernel=True)
    comp, nrm = mvm_errors(c[rows], yref, yabs)
    assert comp <= MVM_TOL and nrm <= MVM_TOL
    plan.close()


def test_config2_full_size_sampled(oracle_lib):
    """d=2, N=100000, nu=3/2, ell=0.1 (configuration 2), both forms, 5000 oracle rows."""
    for form in ("product", "l1"):
        p = workloads.config2(form=form, nrhs=1)
        rows = np.arange(5000)
        say("config2 %s" % form)
        comp, nrm = run_case(p.x, p.v, 3, form, 0.1, rows=rows)
        say("config2", form, comp, nrm)
        assert comp <= MVM_TOL and nrm <= MVM_TOL


def test_several_pass_groups_with_stored_run_carries(oracle_lib):
    """d=2, N = 2^21 + 3, 16 columns: the per-pass partial results exceed their
    budget, so the product runs its 22 passes in groups of 3 (tiles of 512, the
    runs' within-tile carries stored per group); 48 sampled rows."""
    rng = np.random.default_rng(9900)
    n = (1 << 21) + 3
    x = rng.uniform(0.0, 1.0, (n, 2))
    v = rng.standard_normal((n, 16))
    rows = rng.choice(n, 48, replace=False)
    say("several pass groups: n=%d nrhs=16" % n)
    comp, nrm = run_case(x, v, 3, "product", 0.05, rows=rows)
    say("several pass groups", comp, nrm)
    assert comp <= MVM_TOL and nrm <= MVM_TOL


@pytest.mark.parametrize("nrhs", [1, 8, 32])
def test_config2_rhs_widths(oracle_lib, nrhs):
    p = workloads.config2(nrhs=nrhs)
    rows = np.arange(0, 100_000, 211)
    say("config2 nrhs=%d" % nrhs)
    comp, nrm = run_case(p.x, p.v, 3, "product", 0.1, rows=rows)
    assert comp <= MVM_TOL and nrm <= MVM_TOL


def test_config3_full_size_sampled(oracle_lib):
    """d=3, N=500000, nu=5/2, ell=0.3, x ~ N(0, I3), 32 Rademacher columns, both forms;
    oracle on 300 sampled rows x 32 columns."""
    for form in ("product", "l1"):
        p = workloads.config3(form=form)
        rows = np.random.default_rng(3).choice(p.n, 300, replace=False)
        say("config3 %s" % form)
        comp, nrm = run_case(p.x, p.probes, 5, form, 0.3, rows=rows)
        say("config3", form, comp, nrm)
        assert comp <= MVM_TOL and nrm <= MVM_TOL


@pytest.mark.parametrize("nrhs", [100, 256])
@pytest.mark.parametrize("d,two_nu", [(2, 3), (3, 5)])
def test_widest_products(oracle_lib, nrhs, d, two_nu):
    """The widest products: 100 columns (padded to 128, four 32-column blocks) and the
    limit of 256; 1500 points, several tiles; oracle on 60 sampled rows."""
    p = workloads.random_problem(700 + nrhs + d, 1500, d, two_nu, "product", 0.15, nrhs=nrhs)
    rows = np.random.default_rng(701 + nrhs).choice(1500, 60, replace=False)
    say("widest product nrhs=%d d=%d nu=%d/2" % (nrhs, d, two_nu))
    comp, nrm = run_case(p.x, p.v, two_nu, "product", 0.15, rows=rows, shift=0.02)
    say("  comp %.2e nrm %.2e" % (comp, nrm))
    assert comp <= MVM_TOL and nrm <= MVM_TOL


def test_width_beyond_the_limit_is_refused(oracle_lib):
    p = workloads.random_problem(799, 200, 2, 3, "product", 0.2, nrhs=257)
    plan = mm.Plan(to_gpu(p.x), mm.Kernel(3, "product", 0.2))
    with pytest.raises(mm.MaternError) as e:
        plan.mvm(to_gpu(p.v))
    assert e.value.status == mm.MM_ERR_ARG
    plan.close()
