"""Host-side checks of the C-ABI library (no GPU needed, no compute calls).

The shared library must load, export every function that include/maternmvm.h
declares, and reject invalid arguments on the host before touching a device.
"""
import ctypes
import os
import re

import pytest

import paper_2508_01864_amd as mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maternmvm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"typedef[^;]*;", "", text)          # function-pointer and struct typedefs
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return", "sizeof")))


def test_library_loads_and_exports_every_declared_symbol():
    L = mm.lib()  # loads after torch so that one HIP runtime serves both
    names = declared_functions()
    assert len(names) >= 14, names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, "not exported: %s" % missing
    # the binding declares a signature for each of them
    assert set(names) <= set(mm._SIGS), set(names) - set(mm._SIGS)


def test_version_and_status_strings():
    assert "gfx950" in mm.version()
    for st, name in mm.STATUS_NAMES.items():
        assert mm.lib().mm_status_str(st).decode() == name


def test_footprint_is_host_only_and_sane():
    k = mm.Kernel(3, "product", 0.1)
    b2 = mm.footprint_bytes(100_000, 2, 1, k)
    b3 = mm.footprint_bytes(100_000, 3, 1, k)
    assert 0 < b2 < b3
    # structure: at least L int32 orders of n for d = 2
    assert b2 >= 17 * 100_000 * 4
    assert mm.footprint_bytes(100_000, 2, 32, k) > b2
    assert mm.footprint_bytes(0, 2, 1, k) == 0
    assert mm.footprint_bytes(10, 4, 1, k) == 0
    assert mm.footprint_bytes(10, 2, 1, mm.Kernel(4, "product", 0.1)) == 0
    assert mm.footprint_bytes(10, 2, 1, mm.Kernel(3, "product", -1.0)) == 0


def _create(n, d, ldx, k, xptr=1):
    h = ctypes.c_void_p()
    kk = k.c()
    st = mm.lib().mm_plan_create(ctypes.c_void_p(xptr), n, d, ldx, ctypes.byref(kk), None,
                                 ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("n,d,ldx,k,what", [
    (0, 2, 1, mm.Kernel(3, "product", 0.1), "n must be"),
    (10, 0, 10, mm.Kernel(3, "product", 0.1), "d must be"),
    (10, 4, 10, mm.Kernel(3, "product", 0.1), "d must be"),
    (10, 2, 5, mm.Kernel(3, "product", 0.1), "ldx"),
    (10, 2, 10, mm.Kernel(2, "product", 0.1), "two_nu"),
    (10, 2, 10, mm.Kernel(3, "product", 0.0), "lengthscale"),
    (10, 2, 10, mm.Kernel(3, "product", float("nan")), "lengthscale"),
    (10, 2, 10, mm.Kernel(3, "product", 0.1, 0.0), "outputscale2"),
])
def test_plan_create_rejects_bad_arguments_on_host(n, d, ldx, k, what):
    st, h = _create(n, d, ldx, k)
    assert st == mm.MM_ERR_ARG
    assert not h.value
    assert what in mm.last_error()


def test_null_pointers_rejected_on_host():
    st, _ = _create(10, 2, 10, mm.Kernel(3, "product", 0.1), xptr=0)
    assert st == mm.MM_ERR_ARG and "x is NULL" in mm.last_error()
    L = mm.lib()
    assert L.matern_mvm(None, None, 1, None, 1, 1, 0.0, None) == mm.MM_ERR_ARG
    assert L.gp_cg_solve(None, None, 0.1, 0, 1e-8, 10, None, None, None, None) == mm.MM_ERR_ARG
    assert L.gp_predict(None, None, None, None, 1, 1, None, None) == mm.MM_ERR_ARG
    assert L.matern_mvm_dlengthscale(None, None, 1, None, 1, 1, None) == mm.MM_ERR_ARG
    assert L.gp_lml(None, None, 0.1, None, 1, 1, 10, 1e-8, None, None, None) == mm.MM_ERR_ARG
    assert L.mm_plan_destroy(None) == mm.MM_OK
    assert L.mm_plan_profile_enable(None, 1) == mm.MM_ERR_ARG
    kk = mm.Kernel(3, "product", 0.1).c()
    assert L.mm_plan_set_kernel(None, ctypes.byref(kk), None) == mm.MM_ERR_ARG


def test_solver_entry_points_reject_null_handles_on_host():
    L = mm.lib()
    h = ctypes.c_void_p()
    assert L.mm_solver_create(None, None, 0.1, 0, 1e-8, None, ctypes.byref(h)) == mm.MM_ERR_ARG
    assert not h.value
    assert L.mm_solver_iterate(None, 1, None) == mm.MM_ERR_ARG
    assert L.mm_solver_poll(None, None, None, None, None) == mm.MM_ERR_ARG
    assert L.mm_solver_finish(None, None, None, None, None) == mm.MM_ERR_ARG
    assert L.mm_solver_check(None, 1, None, None, None) == mm.MM_ERR_ARG
    assert L.mm_solver_destroy(None) == mm.MM_OK
    assert L.mm_solver_batch_create(None, 0, 1, ctypes.byref(h)) == mm.MM_ERR_ARG
    assert L.mm_solver_batch_iterate(None, 1, None) == mm.MM_ERR_ARG
    assert L.mm_solver_batch_set_schedule(None, 1, 1) == mm.MM_ERR_ARG
    assert L.mm_solver_batch_poll(None, None, None) == mm.MM_ERR_ARG
    assert L.mm_solver_batch_destroy(None) == mm.MM_OK


def test_set_allocator_argument_rules_on_host():
    L = mm.lib()
    fn = ctypes.cast(mm._ALLOC_FN(lambda n, s, c: None), ctypes.c_void_p)
    assert L.mm_set_allocator(fn, None, None) == mm.MM_ERR_ARG
    assert "both" in mm.last_error()
    assert L.mm_set_allocator(None, None, None) == mm.MM_OK
