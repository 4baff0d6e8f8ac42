"""The paper's weighted-ECDF decomposition of the Matern kernel sum, evaluated
by brute-force masked sums.

TEST INFRASTRUCTURE ONLY (an independent cross-check of the dense oracle and
of the tie conventions on small inputs; O(2^d P N^2) work).

Everything here follows Section 2 of the paper in its own notation:

* ``ecdf``            the weighted multivariate ECDF F(delta z, delta; delta x, w)
                      of eq. ECDFdelta, with the generalised inequality <=_c
                      meaning <= for c >= 0 and < for c < 0.
* ``phi_table``       the univariate separable factors phi_{1,p}, phi_{2,p} of
                      Assumption 1 (eq. k12_decomposition_phi, k32_decomposition_phi,
                      k52_decomposition_phi).
* ``prop1_l1``        Proposition 1 (eq. L1_decomposition, L1_weights).
* ``prop2_product``   Proposition 2 (eq. product_decomposition, product_weights).
* ``matern_l1``       the L1 Matern examples (eq. matern_12_decomposition,
                      matern_32_decomposition, matern_52_decomposition with the
                      weights of eq. matern_weights).
* ``matern_product_32``  the product Matern-3/2 example (eq.
                      matern_product_32_decomposition with eq.
                      matern_product_weights_0 / _1 / _vector).  The printed
                      pi weights are read as products over the coordinates with
                      theta_k = 1 (for pi^(0)) and theta_k = 0 (for pi^(1)); a
                      literal reading of the printed product of theta_k factors
                      would vanish unless every theta_k is 1.

The scaled kernel sigma_s^2 k(u / ell) (eq. scaled_kernel) is obtained by
applying the unscaled identities to x / ell and z / ell.
"""
from __future__ import annotations

import itertools

import numpy as np


def _pts(x):
    x = np.asarray(x, dtype=np.float64)
    return x[:, None] if x.ndim == 1 else x


def ecdf(dz: np.ndarray, delta, dx: np.ndarray, w: np.ndarray) -> np.ndarray:
    """F(delta z, delta; delta x, w) for every target row of ``dz`` (eq. ECDFdelta).

    dz: (m, d) already multiplied by delta; dx: (n, d) likewise; w: (n,) or (n, r).
    The indicator is prod_k 1{dx_k <=_{delta_k} dz_k}.
    """
    m, d = dz.shape
    mask = np.ones((m, dx.shape[0]), dtype=bool)
    for k in range(d):
        a = dx[None, :, k]
        b = dz[:, None, k]
        mask &= (a <= b) if delta[k] >= 0 else (a < b)
    return mask.astype(np.float64) @ w


def phi_table(two_nu: int):
    """(phi_1, phi_2) lists for Assumption 1 (k(u - v) = sum_p phi_1p(u) phi_2p(v), u >= v)."""
    if two_nu == 1:          # eq. k12_decomposition_phi
        return ([lambda u: np.exp(-u)], [lambda v: np.exp(v)])
    if two_nu == 3:          # eq. k32_decomposition_phi
        s = np.sqrt(3.0)
        return ([lambda u: (1.0 + s * u) * np.exp(-s * u), lambda u: -s * np.exp(-s * u)],
                [lambda v: np.exp(s * v), lambda v: v * np.exp(s * v)])
    if two_nu == 5:          # eq. k52_decomposition_phi
        s = np.sqrt(5.0)
        return ([lambda u: (1.0 + s * u + 5.0 / 3.0 * u * u) * np.exp(-s * u),
                 lambda u: -(s + 10.0 / 3.0 * u) * np.exp(-s * u),
                 lambda u: 5.0 / 3.0 * np.exp(-s * u)],
                [lambda v: np.exp(s * v),
                 lambda v: v * np.exp(s * v),
                 lambda v: v * v * np.exp(s * v)])
    raise ValueError("two_nu must be 1, 3 or 5")


def _orthants(d):
    return [np.array(t, dtype=np.float64) for t in itertools.product((-1.0, 1.0), repeat=d)]


def prop1_l1(x, v, two_nu: int, ell: float, s2: float = 1.0, z=None) -> np.ndarray:
    """Proposition 1: sum_delta sum_p phi_1p(delta.z) F(delta z, delta; delta x, w_p),
    with w_{i,p} = v_i phi_2p(delta.x_i) (eq. L1_decomposition, L1_weights)."""
    x = _pts(x) / ell
    z = x if z is None else _pts(z) / ell
    phi1, phi2 = phi_table(two_nu)
    out = 0.0
    for delta in _orthants(x.shape[1]):
        dz, dx = z * delta, x * delta
        sz, sx = dz.sum(axis=1), dx.sum(axis=1)
        for p in range(len(phi1)):
            w = np.asarray(v, dtype=np.float64) * (phi2[p](sx) if np.ndim(v) == 1
                                                   else phi2[p](sx)[:, None])
            F = ecdf(dz, delta, dx, w)
            out = out + (phi1[p](sz) if F.ndim == 1 else phi1[p](sz)[:, None]) * F
    return s2 * out


def prop2_product(x, v, two_nu: int, ell: float, s2: float = 1.0, z=None) -> np.ndarray:
    """Proposition 2: sum_theta sum_delta (prod_k phi_1,theta_k(delta_k z_k))
    F(delta z, delta; delta x, w) with w_i = v_i prod_k phi_2,theta_k(delta_k x_ki)
    (eq. product_decomposition, product_weights)."""
    x = _pts(x) / ell
    z = x if z is None else _pts(z) / ell
    d = x.shape[1]
    phi1, phi2 = phi_table(two_nu)
    P = len(phi1)
    v = np.asarray(v, dtype=np.float64)
    out = 0.0
    for theta in itertools.product(range(P), repeat=d):
        for delta in _orthants(d):
            dz, dx = z * delta, x * delta
            c1 = np.ones(z.shape[0])
            c2 = np.ones(x.shape[0])
            for k in range(d):
                c1 = c1 * phi1[theta[k]](dz[:, k])
                c2 = c2 * phi2[theta[k]](dx[:, k])
            w = v * (c2 if v.ndim == 1 else c2[:, None])
            F = ecdf(dz, delta, dx, w)
            out = out + (c1 if F.ndim == 1 else c1[:, None]) * F
    return s2 * out


def matern_weights(v, dxsum, p: int, two_nu: int, ell: float):
    """w_i^(p) = v_i (delta.x_i)^p exp(sqrt(2 nu)/ell delta.x_i) (eq. matern_weights)."""
    a = np.sqrt(float(two_nu)) / ell
    g = dxsum ** p * np.exp(a * dxsum)
    v = np.asarray(v, dtype=np.float64)
    return v * (g if v.ndim == 1 else g[:, None])


def matern_l1(x, v, two_nu: int, ell: float, s2: float = 1.0, z=None) -> np.ndarray:
    """L1 Matern kernel sums via eq. matern_12_decomposition (2nu=1),
    matern_32_decomposition (2nu=3) and matern_52_decomposition (2nu=5)."""
    x = _pts(x)
    z = x if z is None else _pts(z)
    a = np.sqrt(float(two_nu)) / ell
    out = 0.0
    for delta in _orthants(x.shape[1]):
        dz, dx = z * delta, x * delta
        sz, sx = dz.sum(axis=1), dx.sum(axis=1)
        F = [ecdf(dz, delta, dx, matern_weights(v, sx, p, two_nu, ell)) for p in range(3)]
        e = np.exp(-a * sz)
        if two_nu == 1:
            c = [e, 0.0 * e, 0.0 * e]
        elif two_nu == 3:
            c = [e * (1.0 + a * sz), -a * e, 0.0 * e]
        else:
            b = 5.0 / (3.0 * ell * ell)
            c = [e * (1.0 + a * sz + b * sz * sz), -e * (a + 2.0 * b * sz), b * e]
        for p in range(3):
            cp = c[p] if F[p].ndim == 1 else c[p][:, None]
            out = out + cp * F[p]
    return s2 * out


def matern_product_32(x, v, ell: float, s2: float = 1.0, z=None) -> np.ndarray:
    """Product Matern-3/2 kernel sums via eq. matern_product_32_decomposition."""
    x = _pts(x)
    z = x if z is None else _pts(z)
    d = x.shape[1]
    a = np.sqrt(3.0) / ell
    v = np.asarray(v, dtype=np.float64)
    out = 0.0
    for theta in itertools.product((0, 1), repeat=d):
        for delta in _orthants(d):
            dz, dx = z * delta, x * delta
            pi0 = np.ones(z.shape[0])      # eq. matern_product_weights_0 (theta_k = 1 terms)
            pi1 = np.ones(x.shape[0])      # eq. matern_product_weights_1 (theta_k = 0 terms)
            for k in range(d):
                if theta[k] == 1:
                    pi0 = pi0 * (1.0 + a * dz[:, k])
                else:
                    pi1 = pi1 * (-a * dx[:, k])
            g = pi1 * np.exp(a * dx.sum(axis=1))   # eq. matern_product_weights_vector
            w = v * (g if v.ndim == 1 else g[:, None])
            F = ecdf(dz, delta, dx, w)
            c = pi0 * np.exp(-a * dz.sum(axis=1))
            out = out + (c if F.ndim == 1 else c[:, None]) * F
    return s2 * out
