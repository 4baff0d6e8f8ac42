"""The oracle's pins must catch plausible mistakes.

Each case compiles a copy of ``oracle/oracle.c`` with one planted mistake (on
the CPU, into a temporary directory), swaps it in for the real library and
checks that at least one of a fixed set of pins fails.  The real library is
restored afterwards.
"""
import ctypes
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import decomposition as dec
import workloads

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "dropped_quadratic_term": ("(5.0 / 3.0) * r * r", "(5.0 / 6.0) * r * r"),
    "wrong_rate_3_2": ("double s3 = sqrt(3.0);", "double s3 = sqrt(2.0);"),
    "l1_as_max_norm": ("l1 += fabs(a[k * sa] - b[k * sb]);",
                       "l1 = fmax(l1, fabs(a[k * sa] - b[k * sb]));"),
    "product_missing_dimension": ("for (int k = 0; k < d; ++k)\n            prod *=",
                                  "for (int k = 1; k < d; ++k)\n            prod *="),
    "no_compensation": ("y[(int64_t)r * ldy + j] = sum + comp;", "y[(int64_t)r * ldy + j] = sum;"),
    "cholesky_no_sqrt": ("double lkk = sqrt(dkk);", "double lkk = dkk;"),
    "lost_diagonal_shift": ("kv += diag;", "kv += 0.0;"),
}


def _pins():
    """A fixed subset of the oracle pins; returns the list of failures."""
    fails = []
    r = np.linspace(1e-3, 5.0, 50)
    for two_nu in (1, 3, 5):
        nu = two_nu / 2
        t = np.sqrt(2 * nu) * r
        ref = t ** nu / (2 ** (nu - 1) * sp.gamma(nu)) * sp.kv(nu, t)
        if np.max(np.abs(oracle.profile(two_nu, r) - ref)) > 1e-13:
            fails.append("bessel%d" % two_nu)
    for d in (2, 3):
        for two_nu in (3, 5):
            for form in ("l1", "product"):
                p = workloads.random_problem(50 + d, 60, d, two_nu, form, 0.6)
                dense, s = oracle.mvm(p.x, p.v, two_nu, form, p.ell, with_abs=True)
                fn = (lambda: dec.matern_l1(p.x, p.v, two_nu, p.ell)) if form == "l1" else \
                     (lambda: dec.prop2_product(p.x, p.v, two_nu, p.ell))
                if np.max(np.abs(fn() - dense) / s) > 1e-11:
                    fails.append("decomp-%s-%d-%d" % (form, two_nu, d))
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, size=(200, 2))
    v = rng.standard_normal(200) * 10.0 ** rng.uniform(-8, 8, size=200)
    K = oracle.kernel_matrix(x, 3, "product", 0.4)
    y = oracle.mvm(x, v, 3, "product", 0.4)
    for j in range(0, 200, 23):
        ex = math.fsum(K[j] * v)
        if abs(y[j] - ex) > 2.5e-16 * abs(ex) + 1e-30:
            fails.append("fsum")
            break
    A = oracle.kernel_matrix(x, 3, "product", 0.2, sigma2=0.05)
    try:
        L = oracle.cholesky(A)
        if np.max(np.abs(L - np.linalg.cholesky(A))) > 1e-12:
            fails.append("chol")
    except oracle.NotPositiveDefinite:
        fails.append("chol-raise")
    if abs(A[3, 3] - 1.05) > 1e-15:
        fails.append("diag")
    return fails


def test_real_oracle_passes_pins(oracle_lib):
    assert _pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_lib, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: %s" % name
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "mut.c")
        so = os.path.join(td, "libmut.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
                               "-o", so, c, "-lm"])
        real = oracle.lib()
        mut = ctypes.CDLL(so)
        for fn in ("oracle_matern_profile", "oracle_profile_array", "oracle_kernel", "oracle_mvm",
                   "oracle_mvm_multi", "oracle_kernel_matrix", "oracle_cholesky",
                   "oracle_cholesky_solve", "oracle_num_threads"):
            getattr(mut, fn).argtypes = getattr(real, fn).argtypes
            getattr(mut, fn).restype = getattr(real, fn).restype
        oracle._lib = mut
        try:
            fails = _pins()
        finally:
            oracle._lib = real
    assert fails, "planted mistake %s was not caught by any pin" % name
