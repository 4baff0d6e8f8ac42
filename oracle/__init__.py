"""Plain CPU oracle for the exact Matern kernel MVM and the direct GP solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline of the benchmark import this package.  It shares no code with the
HIP library in ``paper_2508_01864_amd`` and never imports it.

Contents (each function cites the passage it follows):

* ``mvm``            dense FP64 y_j = sum_i K(z_j, x_i) v_i (Section 2, eq. Ky)
                     with Neumaier-compensated rows, in C (``oracle.c``).
* ``kernel_matrix``  dense K (eq. covariance_matrix), optionally + sigma^2 I.
* ``cholesky`` / ``cholesky_solve``  textbook Cholesky of K + sigma^2 I and
                     the direct solve of eq. gp_mean_system.
* ``gls``            generalised least squares fixed effects (Section 3.2,
                     the beta_GLS formula) with H = [1, x_1 .. x_d].
* ``predict``        posterior mean h(z)^T beta + k_z^T alpha (eq. gp_mean,
                     eq. gp_mean_2).
* ``cg_lanczos`` / ``lanczos_tridiagonal`` / ``logquad_from_cg``  CG
                     coefficients, the Lanczos matrix built from them and the
                     quadrature ||z||^2 e_1^T log(T) e_1 of the stochastic
                     log-determinant (Appendix A, Algorithm 2 and eq.
                     approximationLogDet); ``quad_log_exact``, ``logdet_exact``
                     the dense quantities they estimate.
* ``pivoted_cholesky`` / ``woodbury_apply``  the rank-k pivoted Cholesky
                     preconditioner P = L L^T + sigma^2 I and its inverse by
                     the Woodbury identity (Appendix A, 'Preconditioning').
* ``dprofile_dell`` / ``dkernel_matrix_dell`` / ``mvm_dell``  the lengthscale
                     derivative of the kernel (the gradients of the Section
                     2.3 examples; the product rule for the product form).
* ``lml_exact`` / ``lml_grad_exact`` / ``hutchinson_terms``  the log marginal
                     likelihood and its gradient (eq. gp_log_likelihood, eq.
                     gp_log_likelihood_derivative) by dense algebra, and the
                     terms of the stochastic trace estimator (Appendix A).
* ``posterior_variance``  the posterior variance of eq. gp_variance by Cholesky.
* ``decomposition``  (sub-module) the paper's weighted-ECDF decomposition
                     evaluated by brute-force masked sums (Props. 1-2 and the
                     Matern examples of Section 2.3); used only to pin the
                     dense oracle and the tie conventions on small inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FORM_L1 = 0
FORM_PRODUCT = 1
FORMS = {"l1": FORM_L1, "product": FORM_PRODUCT, FORM_L1: FORM_L1, FORM_PRODUCT: FORM_PRODUCT}

_lib = None


class NotPositiveDefinite(RuntimeError):
    """Raised when the Cholesky factorisation meets a non-positive pivot."""


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc and OpenMP.

    Generic x86-64-v3 code (AVX2 + FMA) so the library runs on any recent
    host, and no fast-math (it would undo the compensated summation).
    """
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        P = ctypes.c_void_p
        L.oracle_matern_profile.argtypes = [i32, dbl]
        L.oracle_matern_profile.restype = dbl
        L.oracle_profile_array.argtypes = [i32, i64, P, P]
        L.oracle_profile_array.restype = i32
        L.oracle_kernel.argtypes = [i32, P, P, i32, i32, dbl, dbl]
        L.oracle_kernel.restype = dbl
        mvm_args = [i64, i32, P, i64, i64, P, i64, i32, i32, dbl, dbl, P, i64, i32, P, i64, P]
        L.oracle_mvm.argtypes = mvm_args
        L.oracle_mvm.restype = i32
        L.oracle_mvm_multi.argtypes = mvm_args
        L.oracle_mvm_multi.restype = i32
        L.oracle_kernel_matrix.argtypes = [i64, i32, P, i64, i64, P, i64, i32, i32, dbl, dbl,
                                           dbl, i32, P, i64]
        L.oracle_kernel_matrix.restype = i32
        L.oracle_cholesky.argtypes = [i64, P, i64]
        L.oracle_cholesky.restype = i32
        L.oracle_cholesky_solve.argtypes = [i64, P, i64, P, i64, i32]
        L.oracle_cholesky_solve.restype = i32
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = i32
        _lib = L
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(lib().oracle_num_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _points(x) -> np.ndarray:
    """Points as a Fortran-ordered (n, d) float64 array (column k = coordinate k)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    return np.asfortranarray(x)


def profile(two_nu: int, r) -> np.ndarray:
    """Matern profile k_nu(r) (Appendix C, eq. matern_1_2 / 3_2 / 5_2)."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
    out = np.empty_like(r)
    lib().oracle_profile_array(int(two_nu), r.size, _ptr(r), _ptr(out))
    return out


def kernel(a, b, two_nu: int, form, ell: float, s2: float = 1.0) -> float:
    """Scalar K(a, b) for two d-vectors (eq. L1_kernel / product_kernel, scaled)."""
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(a, dtype=np.float64)))
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(b, dtype=np.float64)))
    return float(lib().oracle_kernel(a.size, _ptr(a), _ptr(b), int(two_nu), FORMS[form],
                                     float(ell), float(s2)))


def mvm(x, v, two_nu: int, form, ell: float, s2: float = 1.0, z=None,
        with_abs: bool = False, shared_kernel: bool = False):
    """Dense y = K(Z, X) v with compensated row sums (Section 2, eq. Ky / kde).

    x: (n, d) sources; v: (n,) or (n, nrhs); z: (m, d) targets (default x).
    Returns y (same trailing shape as v) and, if ``with_abs``, sum_i |K_ji v_i|.
    ``shared_kernel`` evaluates each kernel entry once for all right-hand sides
    (same arithmetic per column; faster at many columns).
    """
    x = _points(x)
    n, d = x.shape
    zz = x if z is None else _points(z)
    if zz.shape[1] != d:
        raise ValueError("z must have the same dimension as x")
    m = zz.shape[0]
    v = np.asarray(v, dtype=np.float64)
    vec = v.ndim == 1
    V = np.asfortranarray(v[:, None] if vec else v)
    if V.shape[0] != n:
        raise ValueError("v must have n rows")
    nrhs = V.shape[1]
    Y = np.zeros((m, nrhs), dtype=np.float64, order="F")
    A = np.zeros((m, nrhs), dtype=np.float64, order="F")
    fn = lib().oracle_mvm_multi if shared_kernel else lib().oracle_mvm
    rc = fn(n, d, _ptr(x), max(n, 1), m, _ptr(zz), max(m, 1), int(two_nu), FORMS[form],
            float(ell), float(s2), _ptr(V), max(n, 1), nrhs, _ptr(Y), max(m, 1), _ptr(A))
    if rc != 0:
        raise ValueError("oracle_mvm rejected its arguments")
    if vec:
        Y, A = Y[:, 0], A[:, 0]
    return (Y, A) if with_abs else Y


def kernel_matrix(x, two_nu: int, form, ell: float, s2: float = 1.0, z=None,
                  sigma2: float = 0.0) -> np.ndarray:
    """Dense K(Z, X) (eq. covariance_matrix); with z=None adds sigma2 on the diagonal."""
    x = _points(x)
    n, d = x.shape
    zz = x if z is None else _points(z)
    m = zz.shape[0]
    K = np.empty((m, n), dtype=np.float64, order="F")
    rc = lib().oracle_kernel_matrix(n, d, _ptr(x), max(n, 1), m, _ptr(zz), max(m, 1),
                                    int(two_nu), FORMS[form], float(ell), float(s2),
                                    float(sigma2), 1 if z is None else 0, _ptr(K), max(m, 1))
    if rc != 0:
        raise ValueError("oracle_kernel_matrix rejected its arguments")
    return K


def cholesky(a: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a symmetric positive definite matrix."""
    L = np.array(a, dtype=np.float64, order="F", copy=True)
    n = L.shape[0]
    rc = lib().oracle_cholesky(n, _ptr(L), max(n, 1))
    if rc != 0:
        raise NotPositiveDefinite("non-positive pivot at column %d" % (rc - 1))
    return np.tril(L)


def cholesky_solve(L: np.ndarray, b) -> np.ndarray:
    """Solve L L^T x = b by forward then back substitution."""
    L = np.asfortranarray(L, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    B = np.array(b[:, None] if vec else b, dtype=np.float64, order="F", copy=True)
    n, nrhs = B.shape
    lib().oracle_cholesky_solve(n, _ptr(L), max(n, 1), _ptr(B), max(n, 1), nrhs)
    return B[:, 0] if vec else B


def gp_solve(x, y, two_nu: int, form, ell: float, s2: float, sigma2: float) -> np.ndarray:
    """Direct alpha = (K + sigma^2 I)^{-1} y (eq. gp_mean_system) by Cholesky."""
    A = kernel_matrix(x, two_nu, form, ell, s2, sigma2=sigma2)
    return cholesky_solve(cholesky(A), y)


def design_matrix(x) -> np.ndarray:
    """Affine fixed-effects basis H = [1, x_1, ..., x_d] (eq. BetaLin; Section 3.2)."""
    x = _points(x)
    return np.column_stack([np.ones(x.shape[0]), x])


def gls(x, y, two_nu: int, form, ell: float, s2: float, sigma2: float):
    """Generalised least squares fixed effects (Section 3.2, beta_GLS).

    beta = (H^T A^{-1} H)^{-1} H^T A^{-1} y with A = K + sigma^2 I, then the
    centred solve alpha = A^{-1} (y - H beta) (the translation of Section 1).
    Returns (beta, alpha).
    """
    H = design_matrix(x)
    A = kernel_matrix(x, two_nu, form, ell, s2, sigma2=sigma2)
    L = cholesky(A)
    AiH = cholesky_solve(L, H)
    Aiy = cholesky_solve(L, np.asarray(y, dtype=np.float64))
    G = H.T @ AiH
    beta = np.linalg.solve(G, H.T @ Aiy)
    alpha = Aiy - AiH @ beta
    return beta, alpha


def ols(x, y) -> np.ndarray:
    """Ordinary least squares beta = (H^T H)^{-1} H^T y (Algorithm 1, first step)."""
    H = design_matrix(x)
    return np.linalg.solve(H.T @ H, H.T @ np.asarray(y, dtype=np.float64))


def predict(x, alpha, z, two_nu: int, form, ell: float, s2: float, beta=None) -> np.ndarray:
    """Posterior mean k_z^T alpha + h(z)^T beta (eq. gp_mean, eq. gp_mean_2)."""
    mean = mvm(x, alpha, two_nu, form, ell, s2, z=z)
    if beta is not None:
        mean = mean + design_matrix(z) @ np.asarray(beta, dtype=np.float64)
    return mean


def posterior_variance(x, z, two_nu: int, form, ell: float, s2: float, sigma2: float) -> np.ndarray:
    """Posterior variance of the latent function (eq. gp_variance):
    K(z, z) - k_z^T (K + sigma^2 I)^{-1} k_z with K(z, z) = s2, by Cholesky."""
    A = kernel_matrix(x, two_nu, form, ell, s2, sigma2=sigma2)
    Kxz = kernel_matrix(z, two_nu, form, ell, s2, z=x)      # K(X, Z): n x m
    U = cholesky_solve(cholesky(A), Kxz)
    return s2 - np.einsum("ij,ij->j", Kxz, U)


def pivoted_cholesky(x, two_nu: int, form, ell: float, s2: float, max_rank: int, tol: float = 0.0):
    """Rank-k pivoted Cholesky of K (the preconditioner of Appendix A,
    'Preconditioning': P = L L^T + sigma^2 I with L L^T the pivoted Cholesky
    decomposition of K, after Harbrecht, Peters and Schneider).

    Greedy on the residual diagonal d = diag(K - L L^T): step m takes the
    pivot p = argmax d (the smallest index among equal values), sets
    L[:, m] = (K[:, p] - L[:, :m] L[p, :m]^T) / sqrt(d_p) and removes
    L[:, m]^2 from d (negative round-off clamped to zero).  Stops after
    max_rank columns, when d_p <= 0, or when the residual trace sum(d) is at
    most tol * trace(K).

    Returns (L of shape (n, rank), pivots, residual trace)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n = x.shape[0]
    K = kernel_matrix(x, two_nu, form, ell, s2)
    d = np.diag(K).copy()
    trace0 = float(d.sum())
    L = np.zeros((n, max_rank))
    piv = []
    for m in range(max_rank):
        if float(d.sum()) <= tol * trace0:
            break
        p = int(np.argmax(d))
        dp = float(d[p])
        if not dp > 0.0:
            break
        col = (K[:, p] - L[:, :m] @ L[p, :m]) / np.sqrt(dp)
        col[p] = np.sqrt(dp)
        L[:, m] = col
        d = np.maximum(d - col * col, 0.0)
        d[p] = 0.0
        piv.append(p)
    r = len(piv)
    return L[:, :r], np.array(piv, dtype=np.int64), float(d.sum())


def woodbury_apply(L, sigma2: float, r):
    """P^{-1} r for P = L L^T + sigma^2 I by the Woodbury identity
    (Appendix A, 'Preconditioning'):
    P^{-1} r = r / sigma^2 - L (I_k + L^T L / sigma^2)^{-1} L^T r / sigma^4."""
    L = np.asarray(L, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    k = L.shape[1]
    M = np.eye(k) + (L.T @ L) / sigma2
    return r / sigma2 - L @ np.linalg.solve(M, L.T @ r) / (sigma2 * sigma2)


def cg_lanczos(A, b, steps: int, rtol: float = 0.0):
    """Conjugate gradients on dense A with a null start, recording the step
    sizes alpha_k and ratios beta_k (Appendix A, Algorithm 2 without
    preconditioner).  Like the algorithm, it returns when the residual meets
    the tolerance; beta is recorded only for iterations that continue.
    Returns (alphas, betas) as arrays."""
    A = np.asarray(A, dtype=np.float64)
    r = np.asarray(b, dtype=np.float64).copy()
    x = np.zeros_like(r)
    p = r.copy()
    rr = float(r @ r)
    bnorm = np.sqrt(rr)
    alphas, betas = [], []
    for _ in range(steps):
        Ap = A @ p
        alpha = rr / float(p @ Ap)
        alphas.append(alpha)
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        if np.sqrt(rr_new) <= rtol * bnorm:
            break
        beta = rr_new / rr
        betas.append(beta)
        p = r + beta * p
        rr = rr_new
    return np.array(alphas), np.array(betas)


def pcg_lanczos(A, b, Pinv, steps: int, rtol: float = 0.0):
    """Preconditioned conjugate gradients on dense A with a null start
    (Appendix A, Algorithm 2 with the preconditioner solve s_P = Pinv),
    recording alpha_k = r_k^T z_k / p_k^T A p_k and
    beta_k = r_{k+1}^T z_{k+1} / r_k^T z_k.  These define the Lanczos matrix of
    P^{-1/2} A P^{-1/2} started from P^{-1/2} b.  Stops like cg_lanczos on the
    unpreconditioned residual.  Returns (alphas, betas, b^T P^{-1} b)."""
    A = np.asarray(A, dtype=np.float64)
    r = np.asarray(b, dtype=np.float64).copy()
    x = np.zeros_like(r)
    z = Pinv(r)
    p = z.copy()
    rz = float(r @ z)
    rz0 = rz
    bnorm = float(np.sqrt(r @ r))
    alphas, betas = [], []
    for _ in range(steps):
        Ap = A @ p
        alpha = rz / float(p @ Ap)
        alphas.append(alpha)
        x += alpha * p
        r -= alpha * Ap
        if np.sqrt(float(r @ r)) <= rtol * bnorm:
            break
        z = Pinv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    return np.array(alphas), np.array(betas), rz0


def logdet_lowrank_plus_noise(L, sigma2: float) -> float:
    """log det(L L^T + sigma^2 I_n) = n log sigma^2 + log det(I_k + L^T L / sigma^2)
    (Sylvester's determinant identity), the second term by this module's Cholesky."""
    L = np.asarray(L, dtype=np.float64)
    n, k = L.shape
    M = np.eye(k) + (L.T @ L) / sigma2
    return float(n * np.log(sigma2) + 2.0 * np.sum(np.log(np.diag(cholesky(M)))))


def logdet_pc_estimate(A, L, sigma2: float, G1, G2, steps: int, rtol: float = 0.0):
    """Preconditioned stochastic log-determinant (Appendix A, the preconditioned
    variant of eq. approximationLogDet): probes z_i = L g1_i + sigma g2_i are
    N(0, P) draws for P = L L^T + sigma^2 I; each gives the quadrature
    (z_i^T P^{-1} z_i) e_1^T log(T_i) e_1 from PCG with s_P = P^{-1}, an unbiased
    term of log det(P^{-1/2} A P^{-1/2}); the estimate adds log det P.
    Returns (estimate, per-probe quadratures)."""
    G1 = np.asarray(G1, dtype=np.float64)
    G2 = np.asarray(G2, dtype=np.float64)
    if G1.ndim == 1:
        G1, G2 = G1[:, None], G2[:, None]
    Z = np.asarray(L, dtype=np.float64) @ G1 + np.sqrt(sigma2) * G2
    quads = []
    for i in range(Z.shape[1]):
        al, be, rz0 = pcg_lanczos(A, Z[:, i], lambda r: woodbury_apply(L, sigma2, r), steps, rtol)
        # T is built from the iterations that continued (one per beta); a solve
        # that ends in its first step leaves the 1 x 1 matrix [1 / alpha_0]
        quads.append(logquad_from_cg(al, be, rz0) if len(be) else rz0 * float(np.log(1.0 / al[0])))
    quads = np.array(quads)
    return logdet_lowrank_plus_noise(L, sigma2) + float(np.mean(quads)), quads


def lanczos_tridiagonal(alphas, betas):
    """The Lanczos tridiagonal matrix from CG coefficients (Algorithm 2):
    T[k,k] = 1/alpha_k + beta_{k-1}/alpha_{k-1} (beta_0/alpha_0 = 0) and
    T[k,k+1] = T[k+1,k] = sqrt(beta_k)/alpha_k, of size m = len(betas)
    (the iterations that continued)."""
    m = len(betas)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    return T


def logquad_from_cg(alphas, betas, znorm2: float) -> float:
    """||z||^2 e_1^T log(T) e_1 (eq. approximationLogDet with the exact norm of
    the probe in place of sqrt(N))."""
    T = lanczos_tridiagonal(alphas, betas)
    w, Q = np.linalg.eigh(T)
    return float(znorm2 * np.sum(Q[0, :] ** 2 * np.log(w)))


def quad_log_exact(A, Z) -> np.ndarray:
    """z_i^T log(A) z_i for each column of Z, by the dense eigendecomposition."""
    w, Q = np.linalg.eigh(np.asarray(A, dtype=np.float64))
    P = Q.T @ np.asarray(Z, dtype=np.float64)
    if P.ndim == 1:
        P = P[:, None]
    return (np.log(w)[:, None] * P * P).sum(axis=0)


def logdet_exact(A) -> float:
    """log det A = 2 sum log diag(chol(A)) (textbook Cholesky of this module)."""
    return float(2.0 * np.sum(np.log(np.diag(cholesky(np.asarray(A, dtype=np.float64))))))


def dprofile_dell(two_nu: int, r, ell: float) -> np.ndarray:
    """d/d ell of k_nu(r / ell) for the scaled Matern profiles (the lengthscale
    gradients printed with the L1 examples of Section 2.3):
    nu = 1/2: r / ell^2 exp(-r / ell);
    nu = 3/2: 3 r^2 / ell^3 exp(-sqrt(3) r / ell);
    nu = 5/2: 5/3 (r^2 / ell^3 + sqrt(5) r^3 / ell^4) exp(-sqrt(5) r / ell)."""
    r = np.asarray(r, dtype=np.float64)
    if two_nu == 1:
        return r / ell ** 2 * np.exp(-r / ell)
    if two_nu == 3:
        return 3.0 * r ** 2 / ell ** 3 * np.exp(-np.sqrt(3.0) * r / ell)
    if two_nu == 5:
        return 5.0 / 3.0 * (r ** 2 / ell ** 3 + np.sqrt(5.0) * r ** 3 / ell ** 4) * np.exp(-np.sqrt(5.0) * r / ell)
    raise ValueError("two_nu must be 1, 3 or 5")


def dkernel_matrix_dell(x, two_nu: int, form, ell: float, s2: float = 1.0, z=None) -> np.ndarray:
    """Dense d K(Z, X) / d ell (Z defaults to X).  L1 form: s2 times the
    profile derivative of the L1 distance.  Product form (eq. product_kernel):
    the derivative of a product, s2 sum_j dk(|u_j|)/d ell prod_{k != j}
    k(|u_k| / ell), with the one-dimensional profiles of ``profile``."""
    x = _points(x)
    zz = x if z is None else _points(z)
    U = np.abs(zz[:, None, :] - x[None, :, :])          # (m, n, d)
    if FORMS[form] == FORM_L1:
        return s2 * dprofile_dell(two_nu, U.sum(axis=2), ell)
    d = x.shape[1]
    F = np.stack([profile(two_nu, U[:, :, k] / ell) for k in range(d)], axis=2)
    G = np.stack([dprofile_dell(two_nu, U[:, :, k], ell) for k in range(d)], axis=2)
    out = np.zeros(U.shape[:2])
    for j in range(d):
        term = G[:, :, j].copy()
        for k in range(d):
            if k != j:
                term = term * F[:, :, k]
        out += term
    return s2 * out


def mvm_dell(x, v, two_nu: int, form, ell: float, s2: float = 1.0, z=None):
    """Dense y = (dK(Z, X)/d ell) v and its absolute counterpart (dK/d ell)|v|
    (every entry of dK/d ell is non-negative)."""
    D = dkernel_matrix_dell(x, two_nu, form, ell, s2, z=z)
    v = np.asarray(v, dtype=np.float64)
    return D @ v, D @ np.abs(v)


def lml_exact(x, y, two_nu: int, form, ell: float, s2: float, sigma2: float) -> float:
    """Log marginal likelihood with zero mean (eq. gp_log_likelihood):
    -1/2 y^T A^{-1} y - 1/2 log det A - n/2 log(2 pi), A = K + sigma2 I, by
    the textbook Cholesky of this module."""
    A = kernel_matrix(x, two_nu, form, ell, s2, sigma2=sigma2)
    L = cholesky(A)
    y = np.asarray(y, dtype=np.float64)
    alpha = cholesky_solve(L, y)
    n = len(y)
    return float(-0.5 * y @ alpha - np.sum(np.log(np.diag(L))) - 0.5 * n * np.log(2.0 * np.pi))


def lml_grad_exact(x, y, two_nu: int, form, ell: float, s2: float, sigma2: float):
    """Gradient of ``lml_exact`` (eq. gp_log_likelihood_derivative),
    1/2 alpha^T dA alpha - 1/2 tr(A^{-1} dA), for the lengthscale
    (dA = dK/d ell), the noise variance (dA = I) and the output scale s2
    (dA = K / s2), with the dense inverse.  Returns (d_ell, d_sigma2, d_s2)."""
    K = kernel_matrix(x, two_nu, form, ell, s2)
    A = K + sigma2 * np.eye(K.shape[0])
    L = cholesky(A)
    Ainv = cholesky_solve(L, np.eye(K.shape[0]))
    alpha = Ainv @ np.asarray(y, dtype=np.float64)
    D = dkernel_matrix_dell(x, two_nu, form, ell, s2)
    g_ell = 0.5 * alpha @ D @ alpha - 0.5 * np.sum(Ainv * D.T)
    g_sig = 0.5 * alpha @ alpha - 0.5 * np.trace(Ainv)
    g_s2 = (0.5 * alpha @ K @ alpha - 0.5 * np.sum(Ainv * K.T)) / s2
    return float(g_ell), float(g_sig), float(g_s2)


def hutchinson_terms(A, M, Z) -> np.ndarray:
    """z_i^T A^{-1} M z_i for each probe column of Z (the terms of the
    stochastic trace estimator of Appendix A, 'Stochastic trace estimation'),
    with a dense solve."""
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    U = cholesky_solve(cholesky(np.asarray(A, dtype=np.float64)), Z)
    return np.einsum("ij,ij->j", U, np.asarray(M, dtype=np.float64) @ Z)
