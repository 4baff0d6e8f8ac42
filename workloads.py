"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it holds none of the method's
arithmetic.  Every generator uses ``numpy.random.default_rng(seed)`` (PCG64)
and draws in a fixed order: points first, then vectors / noise, then probes.

The shapes follow the paper's simulated workloads (x uniform on [0,1]^d,
d <= 3, N in the tens to hundreds of thousands; Section 3.1) and the five
benchmark configurations:

1. d=1, N=2000, nu=1/2, ell=0.5, x ~ U[0,1], v ~ N(0,1)
2. d=2, N=100000, nu=3/2, ell=0.1, x ~ U[0,1]^2,
   y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.1^2), sigma^2 = 0.01
3. d=3, N=500000, nu=5/2, ell=0.3, x ~ N(0, I_3), 32 Rademacher probes,
   CG right-hand side as in 2, sigma^2 = 0.01
4. 256 independent problems of log-uniform N in [1e3, 2e5], uneven d, nu, ell
5. a Poisson stream of GP regression requests with an affine trend

The paper's real 2-D temperature dataset (Section 3.2) is not available; the
request stream of configuration 5 stands in for its shape.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class Problem:
    """One GP problem: points, kernel, right-hand side(s) and noise."""
    x: np.ndarray                 # (n, d) float64
    two_nu: int
    form: str                     # "l1" or "product"
    ell: float
    s2: float = 1.0
    sigma2: float = 0.0
    v: Optional[np.ndarray] = None      # MVM input (n,) or (n, nrhs)
    y: Optional[np.ndarray] = None      # regression targets (n,)
    probes: Optional[np.ndarray] = None  # (n, k) Rademacher
    z: Optional[np.ndarray] = None      # prediction points (m, d)
    beta: Optional[np.ndarray] = None   # true affine trend used to draw y
    seed: int = 0
    arrival: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def d(self) -> int:
        return self.x.shape[1]


def solve_form(two_nu: int, d: int) -> str:
    """Form used for solves: product whenever the L1 form is not positive definite."""
    return "product" if (two_nu >= 3 and d >= 2) else "l1"


def field_sin_cos(x: np.ndarray) -> np.ndarray:
    """sin(2 pi x1) * cos(2 pi x2) * cos(2 pi x3) over the coordinates present."""
    f = np.sin(TWO_PI * x[:, 0])
    for k in range(1, x.shape[1]):
        f = f * np.cos(TWO_PI * x[:, k])
    return f


def config1(seed: int = 1001, n: int = 2000) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 1))
    v = rng.standard_normal(n)
    return Problem(x=x, two_nu=1, form="l1", ell=0.5, v=v, seed=seed)


def config2(seed: int = 1002, n: int = 100_000, nrhs: int = 1, form: str = "product") -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 2))
    y = np.sin(TWO_PI * x[:, 0]) * np.cos(TWO_PI * x[:, 1]) + 0.1 * rng.standard_normal(n)
    v = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return Problem(x=x, two_nu=3, form=form, ell=0.1, sigma2=0.01, v=v, y=y, seed=seed)


def config3(seed: int = 1003, n: int = 500_000, nprobes: int = 32, form: str = "product") -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    y = np.sin(TWO_PI * x[:, 0]) * np.cos(TWO_PI * x[:, 1]) + 0.1 * rng.standard_normal(n)
    probes = rng.integers(0, 2, size=(n, nprobes)).astype(np.float64) * 2.0 - 1.0
    return Problem(x=x, two_nu=5, form=form, ell=0.3, sigma2=0.01, v=probes, y=y,
                   probes=probes, seed=seed)


def config4(seed: int = 1004, count: int = 256, n_lo: float = 1e3, n_hi: float = 2e5) -> List[Problem]:
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(np.int64)
    ds = rng.integers(1, 4, size=count)
    nus = rng.choice(np.array([1, 3, 5]), size=count)
    ells = np.exp(rng.uniform(np.log(0.05), np.log(0.5), size=count))
    probs = []
    for k in range(count):
        x = rng.uniform(0.0, 1.0, size=(int(ns[k]), int(ds[k])))
        v = rng.standard_normal(int(ns[k]))
        probs.append(Problem(x=x, two_nu=int(nus[k]), form=solve_form(int(nus[k]), int(ds[k])),
                             ell=float(ells[k]), sigma2=0.01, v=v, y=v, seed=seed * 1000 + k))
    return probs


def config5(seed: int = 1005, count: int = 200, n_lo: float = 5e3, n_hi: float = 3e5,
            rate: float = 1.0, npredict: int = 1000) -> List[Problem]:
    """GP regression requests with an affine trend h(x)^T beta plus a sin/cos field
    plus N(0, sigma^2) noise, arriving as a Poisson stream of the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(np.int64)
    ds = rng.integers(1, 4, size=count)
    nus = rng.choice(np.array([1, 3, 5]), size=count)
    sig2 = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=count))
    ells = np.exp(rng.uniform(np.log(0.05), np.log(0.5), size=count))
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(count):
        n, d = int(ns[k]), int(ds[k])
        x = rng.uniform(0.0, 1.0, size=(n, d))
        beta = rng.standard_normal(d + 1)
        trend = beta[0] + x @ beta[1:]
        y = trend + field_sin_cos(x) + np.sqrt(sig2[k]) * rng.standard_normal(n)
        z = rng.uniform(0.0, 1.0, size=(npredict, d))
        reqs.append(Problem(x=x, two_nu=int(nus[k]), form=solve_form(int(nus[k]), d),
                            ell=float(ells[k]), sigma2=float(sig2[k]), y=y, z=z, beta=beta,
                            seed=seed * 1000 + k, arrival=float(arrivals[k])))
    return reqs


def random_problem(seed: int, n: int, d: int, two_nu: int, form: str, ell: float,
                   nrhs: int = 1, dist: str = "uniform", ties: bool = False) -> Problem:
    """A small random MVM problem; ``ties`` snaps coordinates to a coarse grid so
    that equal coordinates and duplicated points occur."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        x = rng.uniform(0.0, 1.0, size=(n, d))
    else:
        x = rng.standard_normal((n, d))
    if ties:
        x = np.round(x * 4.0) / 4.0
    v = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return Problem(x=x, two_nu=two_nu, form=form, ell=ell, v=v, seed=seed)
