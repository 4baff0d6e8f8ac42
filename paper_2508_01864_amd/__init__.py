"""Exact fast Matern kernel products on AMD Instinct MI355X (gfx950).

Thin ctypes binding of ``libmaternmvm.so`` (C ABI in ``include/maternmvm.h``).
It only marshals arguments: every step of the product, the solve and the
prediction runs in the library's HIP kernels.  PyTorch supplies device memory
and the current stream.  Importing works without a GPU; using a plan needs the
built library and a GPU, and fails loudly otherwise.

    >>> import torch, paper_2508_01864_amd as mm
    >>> x = torch.rand(100_000, 2, dtype=torch.float64, device="cuda")
    >>> plan = mm.Plan(x, mm.Kernel(two_nu=3, form="product", lengthscale=0.1))
    >>> y = plan.mvm(torch.randn(100_000, dtype=torch.float64, device="cuda"))
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmaternmvm.so")

MM_OK = 0
MM_ERR_ARG = 1
MM_ERR_NOMEM = 2
MM_ERR_HIP = 3
MM_ERR_NOTPD = 4
MM_ERR_BREAKDOWN = 5
MM_ERR_NOCONV = 6
STATUS_NAMES = {0: "MM_OK", 1: "MM_ERR_ARG", 2: "MM_ERR_NOMEM", 3: "MM_ERR_HIP",
                4: "MM_ERR_NOTPD", 5: "MM_ERR_BREAKDOWN", 6: "MM_ERR_NOCONV"}

FORM_L1 = 0
FORM_PRODUCT = 1
_FORMS = {"l1": FORM_L1, "product": FORM_PRODUCT, FORM_L1: FORM_L1, FORM_PRODUCT: FORM_PRODUCT}


class MaternError(RuntimeError):
    """A library call returned a non-OK status."""

    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class _MMKernel(ctypes.Structure):
    _fields_ = [("two_nu", ctypes.c_int32), ("form", ctypes.c_int32),
                ("lengthscale", ctypes.c_double), ("outputscale2", ctypes.c_double)]


class _MMSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("relres_max", ctypes.c_double),
                ("converged_cols", ctypes.c_int32), ("true_relres", ctypes.c_double)]


class _MMLmlInfo(ctypes.Structure):
    _fields_ = [("lml", ctypes.c_double), ("quad", ctypes.c_double), ("logdet", ctypes.c_double),
                ("dlml_dlengthscale", ctypes.c_double), ("dlml_dsigma2", ctypes.c_double),
                ("dlml_doutputscale2", ctypes.c_double), ("trace_dk_dlengthscale", ctypes.c_double),
                ("trace_inv", ctypes.c_double), ("relres_max", ctypes.c_double),
                ("iters", ctypes.c_int32), ("converged", ctypes.c_int32)]


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "mm_version": (ctypes.c_char_p, []),
    "mm_set_allocator": (ctypes.c_int, [_P, _P, _P]),
    "mm_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "mm_last_error": (ctypes.c_char_p, []),
    "mm_plan_footprint_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(_MMKernel)]),
    "mm_plan_create": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.POINTER(_MMKernel), _P, ctypes.POINTER(_P)]),
    "mm_plan_set_schedule": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "mm_plan_get_schedule": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "mm_plan_set_kernel": (ctypes.c_int, [_P, ctypes.POINTER(_MMKernel), _P]),
    "mm_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(_MMKernel)]),
    "mm_plan_destroy": (ctypes.c_int, [_P]),
    "matern_mvm": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_double, _P]),
    "matern_mvm_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_double, _P]),
    "matern_mvm_dlengthscale": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32, _P]),
    "gp_lml": (ctypes.c_int, [_P, _P, ctypes.c_double, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_double, ctypes.POINTER(_MMLmlInfo), _P, _P]),
    "gp_variance": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_int32, _P, ctypes.POINTER(_MMSolveInfo), _P]),
    "gp_cg_solve": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(_MMSolveInfo), _P]),
    "gp_cg_solve_multi": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, _P, ctypes.c_int64,
                                         ctypes.POINTER(_MMSolveInfo), _P]),
    "gp_predict": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double), _P, ctypes.c_int64,
                                  ctypes.c_int64, _P, _P]),
    "mm_precond_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, _P, ctypes.POINTER(_P)]),
    "mm_precond_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "mm_precond_factor": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), _P]),
    "mm_precond_destroy": (ctypes.c_int, [_P]),
    "mm_solver_create_pc": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_double, _P, _P,
                                           ctypes.POINTER(_P)]),
    "gp_pcg_solve": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P,
                                    _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_MMSolveInfo), _P]),
    "gp_logdet": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int32), _P]),
    "mm_lanczos_logquad": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "mm_solver_footprint_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.POINTER(_MMKernel)]),
    "mm_solver_create": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_double, _P,
                                        ctypes.POINTER(_P)]),
    "mm_solver_iterate": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "mm_solver_poll": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(_MMSolveInfo), _P]),
    "mm_solver_check": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double), _P]),
    "mm_solver_finish": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_MMSolveInfo), _P]),
    "mm_solver_destroy": (ctypes.c_int, [_P]),
    "mm_solver_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(_P)]),
    "mm_solver_batch_set_schedule": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "mm_solver_batch_iterate": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "mm_solver_batch_poll": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
    "mm_solver_batch_destroy": (ctypes.c_int, [_P]),
    "mm_mvm_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(_P)]),
    "mm_mvm_batch_set_schedule": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "mm_mvm_batch_run": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64), ctypes.c_double, _P]),
    "mm_mvm_batch_destroy": (ctypes.c_int, [_P]),
    "gp_logdet_pc": (ctypes.c_int, [_P, ctypes.c_double, _P, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double), _P]),
    "mm_plan_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "mm_plan_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
}

_lib = None


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted(set(line.split()[-1] for line in f if "libamdhip64" in line))
    except OSError:
        return []


def lib():
    """The loaded library; raises if it has not been built (no fallback exists).

    PyTorch is imported first so that the library binds to the HIP runtime
    PyTorch already uses: device memory and stream handles then belong to one
    runtime (a second copy of the runtime in the process would not see
    PyTorch's streams and may fail to open the device)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmaternmvm.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2508_01864_amd.build); there is no fallback path")
        import torch  # noqa: F401  (loads PyTorch's HIP runtime before the library)
        L = ctypes.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError("two HIP runtimes are loaded (%s); load libmaternmvm through this "
                               "module after importing torch" % ", ".join(rts))
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def version() -> str:
    return lib().mm_version().decode()


def last_error() -> str:
    return lib().mm_last_error().decode()


def _check(st: int):
    if st != MM_OK:
        raise MaternError(st, last_error())


@dataclass
class Kernel:
    """Scaled Matern kernel outputscale2 * k_nu(r / lengthscale), nu = two_nu / 2."""
    two_nu: int = 3
    form: str = "product"
    lengthscale: float = 0.1
    outputscale2: float = 1.0

    def c(self) -> _MMKernel:
        return _MMKernel(int(self.two_nu), _FORMS[self.form], float(self.lengthscale),
                         float(self.outputscale2))


def footprint_bytes(n: int, d: int, nrhs: int, kernel: Kernel) -> int:
    """Upper bound of a plan's device memory (host-only; 0 for invalid arguments)."""
    k = kernel.c()
    return int(lib().mm_plan_footprint_bytes(int(n), int(d), int(nrhs), ctypes.byref(k)))


def solver_footprint_bytes(n: int, d: int, fixed_effects: bool, kernel: Kernel) -> int:
    """Upper bound of one solver's device memory, plan excluded (host-only)."""
    k = kernel.c()
    return int(lib().mm_solver_footprint_bytes(int(n), int(d), 1 if fixed_effects else 0, ctypes.byref(k)))


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _colmajor(t, n: int):
    """(n,) or (n, k) float64 CUDA tensor -> contiguous (k, n) tensor (column-major n x k)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError("expected float64")
    if t.shape[0] != n:
        raise ValueError("leading dimension must be %d (got %d)" % (n, t.shape[0]))
    if t.dim() == 1:
        return t.contiguous().view(1, n)
    return t.t().contiguous()


class Plan:
    """Stored sorting outputs of a point set plus the kernel (mm_plan)."""

    def __init__(self, x, kernel: Kernel, stream=None):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64:
            raise TypeError("x must be a float64 CUDA tensor of shape (n, d)")
        if x.dim() == 1:
            x = x.view(-1, 1)
        self.n, self.d = int(x.shape[0]), int(x.shape[1])
        self.kernel = kernel
        self._x = x.t().contiguous()      # column-major n x d, ldx = n
        self._h = ctypes.c_void_p()
        k = kernel.c()
        self._stream = stream
        _check(lib().mm_plan_create(ctypes.c_void_p(self._x.data_ptr()), self.n, self.d, self.n,
                                    ctypes.byref(k), _stream_ptr(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().mm_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, width: int, wb: int, e: int = 0, runex: bool = True):
        """Scan schedule of this plan's products at padded width `width`
        (mm_plan_set_schedule): wb columns per wave, runs of e positions."""
        _check(lib().mm_plan_set_schedule(self._h, int(width), int(wb), int(e), 1 if runex else 0))

    def schedule(self, width: int):
        """(wb, e, runex) in effect at padded width `width`."""
        wb, e, rx = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mm_plan_get_schedule(self._h, int(width), ctypes.byref(wb), ctypes.byref(e), ctypes.byref(rx)))
        return wb.value, e.value, bool(rx.value)

    def set_kernel(self, kernel: Kernel):
        k = kernel.c()
        _check(lib().mm_plan_set_kernel(self._h, ctypes.byref(k), _stream_ptr(self._stream)))
        self.kernel = kernel

    def mvm(self, v, shift: float = 0.0, out=None):
        """y = (K + shift I) v for v of shape (n,) or (n, nrhs)."""
        torch = _torch()
        vc = _colmajor(v, self.n)
        nrhs = vc.shape[0]
        yc = out if out is not None else torch.empty_like(vc)
        _check(lib().matern_mvm(self._h, ctypes.c_void_p(vc.data_ptr()), self.n,
                                ctypes.c_void_p(yc.data_ptr()), self.n, nrhs, float(shift),
                                _stream_ptr(self._stream)))
        return yc.view(-1) if v.dim() == 1 else yc.t()

    def mvm_noalloc_raw(self, vc, yc, nrhs: int, shift: float = 0.0):
        """matern_mvm_noalloc on preallocated column-major buffers (nrhs, n): the
        product without any device allocation (work buffers in the library's
        fixed scratch array)."""
        _check(lib().matern_mvm_noalloc(self._h, ctypes.c_void_p(vc.data_ptr()), self.n,
                                        ctypes.c_void_p(yc.data_ptr()), self.n, int(nrhs), float(shift),
                                        _stream_ptr(self._stream)))

    def mvm_dlengthscale(self, v, out=None):
        """y = (dK/d lengthscale) v for v of shape (n,) or (n, nrhs)."""
        torch = _torch()
        vc = _colmajor(v, self.n)
        nrhs = vc.shape[0]
        yc = out if out is not None else torch.empty_like(vc)
        _check(lib().matern_mvm_dlengthscale(self._h, ctypes.c_void_p(vc.data_ptr()), self.n,
                                             ctypes.c_void_p(yc.data_ptr()), self.n, nrhs,
                                             _stream_ptr(self._stream)))
        return yc.view(-1) if v.dim() == 1 else yc.t()

    def mvm_dlengthscale_raw(self, vc, yc, nrhs: int):
        """Derivative product on preallocated column-major buffers (nrhs, n)."""
        _check(lib().matern_mvm_dlengthscale(self._h, ctypes.c_void_p(vc.data_ptr()), self.n,
                                             ctypes.c_void_p(yc.data_ptr()), self.n, int(nrhs),
                                             _stream_ptr(self._stream)))

    def lml(self, y, sigma2: float, probes, maxit: int = 20000, rtol: float = 1e-8,
            raise_on_error: bool = True, want_alpha: bool = False):
        """Log marginal likelihood (zero mean) and its gradient in the lengthscale,
        the noise variance and the output scale, with the stochastic log-determinant
        and trace estimates from the probe columns (n, l), l <= 63.  Returns a dict
        (and alpha = A^{-1} y when want_alpha)."""
        torch = _torch()
        yc = _colmajor(y, self.n).view(-1)
        Zc = _colmajor(probes, self.n)
        k = Zc.shape[0]
        info = _MMLmlInfo()
        alpha = torch.empty_like(yc) if want_alpha else None
        st = lib().gp_lml(self._h, ctypes.c_void_p(yc.data_ptr()), float(sigma2), ctypes.c_void_p(Zc.data_ptr()),
                          self.n, k, int(maxit), float(rtol), ctypes.byref(info),
                          ctypes.c_void_p(alpha.data_ptr()) if want_alpha else None, _stream_ptr(self._stream))
        msg = last_error()
        if st != MM_OK and raise_on_error:
            raise MaternError(st, msg)
        out = {name: getattr(info, name) for name, _ in _MMLmlInfo._fields_}
        out["status"] = STATUS_NAMES[st]
        return (out, alpha) if want_alpha else out

    def mvm_raw(self, vc, yc, nrhs: int, shift: float = 0.0):
        """Product on preallocated column-major buffers (no copies): vc, yc of shape (nrhs, n)."""
        _check(lib().matern_mvm(self._h, ctypes.c_void_p(vc.data_ptr()), self.n,
                                ctypes.c_void_p(yc.data_ptr()), self.n, int(nrhs), float(shift),
                                _stream_ptr(self._stream)))

    def cg_solve(self, y, sigma2: float, fixed_effects: bool = False, rtol: float = 1e-8,
                 maxit: int = 20000, raise_on_error: bool = True, precond=None):
        """alpha = (K + sigma2 I)^{-1} (y - H beta) with the GLS beta when fixed_effects,
        optionally preconditioned by a :class:`Precond` of this plan.
        Returns (alpha, beta or None, info dict with iters / converged_cols / relres_max / status)."""
        torch = _torch()
        yc = _colmajor(y, self.n).view(-1)
        alpha = torch.empty_like(yc)
        beta = (ctypes.c_double * (self.d + 1))()
        info = _MMSolveInfo()
        if precond is None:
            st = lib().gp_cg_solve(self._h, ctypes.c_void_p(yc.data_ptr()), float(sigma2),
                                   1 if fixed_effects else 0, float(rtol), int(maxit),
                                   ctypes.c_void_p(alpha.data_ptr()),
                                   beta if fixed_effects else None, ctypes.byref(info),
                                   _stream_ptr(self._stream))
        else:
            st = lib().gp_pcg_solve(self._h, ctypes.c_void_p(yc.data_ptr()), float(sigma2),
                                    1 if fixed_effects else 0, float(rtol), int(maxit), precond.handle,
                                    ctypes.c_void_p(alpha.data_ptr()),
                                    beta if fixed_effects else None, ctypes.byref(info),
                                    _stream_ptr(self._stream))
        msg = last_error()
        if st != MM_OK and raise_on_error:
            raise MaternError(st, msg)
        out = _info_dict(info, st)
        return alpha, (np.array(beta[:]) if fixed_effects else None), out

    def cg_solve_multi(self, B, sigma2: float, rtol: float = 1e-8, maxit: int = 20000,
                       raise_on_error: bool = True):
        """X = (K + sigma2 I)^{-1} B for B of shape (n, k)."""
        torch = _torch()
        Bc = _colmajor(B, self.n)
        k = Bc.shape[0]
        Xc = torch.empty_like(Bc)
        info = _MMSolveInfo()
        st = lib().gp_cg_solve_multi(self._h, ctypes.c_void_p(Bc.data_ptr()), self.n, k,
                                     float(sigma2), float(rtol), int(maxit),
                                     ctypes.c_void_p(Xc.data_ptr()), self.n, ctypes.byref(info),
                                     _stream_ptr(self._stream))
        msg = last_error()
        if st != MM_OK and raise_on_error:
            raise MaternError(st, msg)
        out = _info_dict(info, st)
        return (Xc.view(-1) if B.dim() == 1 else Xc.t()), out

    def predict(self, alpha, z, beta=None):
        """Posterior mean sum_i alpha_i K(z, x_i) + h(z)^T beta at z of shape (m, d)."""
        torch = _torch()
        ac = _colmajor(alpha, self.n).view(-1)
        if z.dim() == 1:
            z = z.view(-1, 1)
        m = int(z.shape[0])
        zc = z.t().contiguous()
        mean = torch.empty(m, dtype=torch.float64, device=z.device)
        bp = None
        if beta is not None:
            bb = np.asarray(beta, dtype=np.float64)
            bp = (ctypes.c_double * len(bb))(*bb.tolist())
        _check(lib().gp_predict(self._h, ctypes.c_void_p(ac.data_ptr()), bp,
                                ctypes.c_void_p(zc.data_ptr()), m, m,
                                ctypes.c_void_p(mean.data_ptr()), _stream_ptr(self._stream)))
        return mean

    def variance(self, z, sigma2: float, rtol: float = 1e-10, maxit: int = 20000, raise_on_error: bool = True):
        """Posterior variance of the latent function at z of shape (m, d)
        (eq. gp_variance).  Returns (var, info dict)."""
        torch = _torch()
        if z.dim() == 1:
            z = z.view(-1, 1)
        m = int(z.shape[0])
        zc = z.t().contiguous()
        var = torch.empty(m, dtype=torch.float64, device=z.device)
        info = _MMSolveInfo()
        st = lib().gp_variance(self._h, float(sigma2), ctypes.c_void_p(zc.data_ptr()), m, m, float(rtol), int(maxit),
                               ctypes.c_void_p(var.data_ptr()), ctypes.byref(info), _stream_ptr(self._stream))
        msg = last_error()
        if st != MM_OK and raise_on_error:
            raise MaternError(st, msg)
        return var, _info_dict(info, st)

    def logdet(self, sigma2: float, probes, steps: int = 200, rtol: float = 0.0):
        """Stochastic log det(K + sigma2 I) from CG-Lanczos quadratures of the probe
        columns (n, l).  Returns (estimate, per-probe terms, Lanczos sizes)."""
        Zc = _colmajor(probes, self.n)
        k = Zc.shape[0]
        est = ctypes.c_double()
        quad = (ctypes.c_double * k)()
        steps_out = (ctypes.c_int32 * k)()
        _check(lib().gp_logdet(self._h, float(sigma2), ctypes.c_void_p(Zc.data_ptr()), self.n, k, int(steps),
                               float(rtol), ctypes.byref(est), quad, steps_out, _stream_ptr(self._stream)))
        return est.value, np.array(quad[:]), np.array(steps_out[:])

    def logdet_pc(self, sigma2: float, precond, G1, G2, steps: int = 200, rtol: float = 0.0):
        """Preconditioned stochastic log det(K + sigma2 I) (gp_logdet_pc): probes
        L g1 + sigma g2 from standard normal G1 (rank, l) and G2 (n, l).
        Returns (estimate, per-probe terms, Lanczos sizes, log det P)."""
        G2c = _colmajor(G2, self.n)
        k = G2c.shape[0]
        rank = precond.info()[0]
        G1c = None
        if rank > 0:
            G1c = G1.t().contiguous() if G1.dim() == 2 else G1.contiguous().view(1, -1)
            if G1c.shape != (k, rank):
                raise ValueError("G1 must have shape (rank, nprobes) = (%d, %d)" % (rank, k))
        est = ctypes.c_double()
        ldp = ctypes.c_double()
        quad = (ctypes.c_double * k)()
        steps_out = (ctypes.c_int32 * k)()
        _check(lib().gp_logdet_pc(self._h, float(sigma2), precond.handle,
                                  ctypes.c_void_p(G1c.data_ptr()) if G1c is not None else None, max(rank, 1),
                                  ctypes.c_void_p(G2c.data_ptr()), self.n, k, int(steps), float(rtol),
                                  ctypes.byref(est), quad, steps_out, ctypes.byref(ldp), _stream_ptr(self._stream)))
        return est.value, np.array(quad[:]), np.array(steps_out[:]), ldp.value

    def profile_enable(self, on: bool = True):
        _check(lib().mm_plan_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        """(summed milliseconds, launches, passes covered) of the bracketed sweep launches."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        npass = ctypes.c_int64()
        _check(lib().mm_plan_profile_read(self._h, ctypes.byref(ms), ctypes.byref(cnt),
                                          ctypes.byref(npass), 1 if reset else 0))
        return ms.value, cnt.value, npass.value


def _info_dict(info: _MMSolveInfo, st: int) -> dict:
    return {"iters": info.iters, "converged_cols": info.converged_cols,
            "relres_max": info.relres_max, "true_relres": info.true_relres, "status": STATUS_NAMES[st]}


class Solver:
    """Conjugate-gradient GP solve split into steps (mm_solver): create, iterate,
    poll, finish.  gp_cg_solve runs the same kernels, so results agree bitwise."""

    def __init__(self, plan: Plan, y, sigma2: float, fixed_effects: bool = False,
                 rtol: float = 1e-8, stream=None, precond=None):
        self.plan = plan
        self.precond = precond
        self.fixed_effects = bool(fixed_effects)
        self._stream = stream
        self._y = _colmajor(y, plan.n).view(-1)   # read by the creation kernels
        self._h = ctypes.c_void_p()
        _check(lib().mm_solver_create_pc(plan.handle, ctypes.c_void_p(self._y.data_ptr()), float(sigma2),
                                         1 if fixed_effects else 0, float(rtol),
                                         precond.handle if precond is not None else None,
                                         _stream_ptr(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def iterate(self, iters: int):
        _check(lib().mm_solver_iterate(self._h, int(iters), _stream_ptr(self._stream)))

    def poll(self):
        """(active columns, breakdown flag, info dict)."""
        act = ctypes.c_int32()
        brk = ctypes.c_int32()
        info = _MMSolveInfo()
        _check(lib().mm_solver_poll(self._h, ctypes.byref(act), ctypes.byref(brk), ctypes.byref(info),
                                    _stream_ptr(self._stream)))
        return act.value, brk.value, _info_dict(info, MM_OK)

    def check(self, tighten: bool = True):
        """Recompute the residual of the current iterate with a fresh product and
        restart from it (mm_solver_check).  Returns (passed, true relative
        residual); when it misses rtol and tighten is set, the column tolerances
        shrink and further iterations continue the solve."""
        ok = ctypes.c_int32()
        rel = ctypes.c_double()
        _check(lib().mm_solver_check(self._h, 1 if tighten else 0, ctypes.byref(ok), ctypes.byref(rel),
                                     _stream_ptr(self._stream)))
        return bool(ok.value), rel.value

    def finish(self, raise_on_error: bool = True):
        """(alpha, beta or None, info) from the current iterate."""
        torch = _torch()
        alpha = torch.empty(self.plan.n, dtype=torch.float64, device=self._y.device)
        beta = (ctypes.c_double * (self.plan.d + 1))()
        info = _MMSolveInfo()
        st = lib().mm_solver_finish(self._h, ctypes.c_void_p(alpha.data_ptr()),
                                    beta if self.fixed_effects else None, ctypes.byref(info),
                                    _stream_ptr(self._stream))
        msg = last_error()
        if st not in (MM_OK, MM_ERR_NOCONV, MM_ERR_BREAKDOWN) or (st != MM_OK and raise_on_error):
            raise MaternError(st, msg)
        return alpha, (np.array(beta[:]) if self.fixed_effects else None), _info_dict(info, st)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mm_solver_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SolverBatch:
    """Joint iteration of several solvers (mm_solver_batch): one launch per kernel
    configuration and phase per iteration, optionally replayed from a HIP graph."""

    def __init__(self, solvers, use_graph: bool = True, stream=None):
        self.solvers = list(solvers)
        self._stream = stream
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.handle.value for s in self.solvers])
        self._h = ctypes.c_void_p()
        _check(lib().mm_solver_batch_create(arr, len(self.solvers), 1 if use_graph else 0,
                                            ctypes.byref(self._h)))

    def set_schedule(self, sweep_wg_per_cu: int, cg_grid: int):
        _check(lib().mm_solver_batch_set_schedule(self._h, int(sweep_wg_per_cu), int(cg_grid)))

    def iterate(self, iters: int):
        _check(lib().mm_solver_batch_iterate(self._h, int(iters), _stream_ptr(self._stream)))

    def poll(self):
        """Active columns per solver after the last iteration (-1 = breakdown)."""
        out = (ctypes.c_int32 * len(self.solvers))()
        _check(lib().mm_solver_batch_poll(self._h, out, _stream_ptr(self._stream)))
        return list(out)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mm_solver_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Precond:
    """Rank-k pivoted Cholesky preconditioner P = L L^T + sigma^2 I of a plan (mm_precond)."""

    def __init__(self, plan: Plan, max_rank: int = 100, tol: float = 0.0, stream=None):
        self.plan = plan
        self._stream = stream
        self._h = ctypes.c_void_p()
        _check(lib().mm_precond_create(plan.handle, int(max_rank), float(tol), _stream_ptr(stream),
                                       ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def info(self):
        """(rank, residual trace, trace of K)."""
        r = ctypes.c_int32()
        tr = ctypes.c_double()
        t0 = ctypes.c_double()
        _check(lib().mm_precond_info(self._h, ctypes.byref(r), ctypes.byref(tr), ctypes.byref(t0)))
        return r.value, tr.value, t0.value

    def factor(self):
        """(L as an (n, rank) float64 CUDA tensor with rows in the caller's point order,
        the pivots' caller indices in column order)."""
        torch = _torch()
        rank = self.info()[0]
        out = torch.zeros((rank, self.plan.n), dtype=torch.float64, device="cuda")
        piv = (ctypes.c_int32 * max(rank, 1))()
        if rank > 0:
            _check(lib().mm_precond_factor(self._h, ctypes.c_void_p(out.data_ptr()), self.plan.n, piv,
                                           _stream_ptr(self._stream)))
        return out.t(), np.array(piv[:rank], dtype=np.int64)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().mm_precond_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MvmBatch:
    """Batched products y_k = (K_k + shift I) v_k over many plans (mm_mvm_batch)."""

    def __init__(self, plans, nrhs: int = 1, use_graph: bool = True, stream=None):
        self.plans = list(plans)
        self.nrhs = int(nrhs)
        self._stream = stream
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self._h = ctypes.c_void_p()
        _check(lib().mm_mvm_batch_create(arr, len(self.plans), self.nrhs, 1 if use_graph else 0,
                                         ctypes.byref(self._h)))

    def set_schedule(self, sweep_wg_per_cu: int, grid: int):
        _check(lib().mm_mvm_batch_set_schedule(self._h, int(sweep_wg_per_cu), int(grid)))

    def run_raw(self, vcs, ycs, shift: float = 0.0):
        """vcs, ycs: lists of contiguous (nrhs, n_k) float64 CUDA tensors (column-major n_k x nrhs)."""
        k = len(self.plans)
        vp = (ctypes.c_void_p * k)(*[t.data_ptr() for t in vcs])
        yp = (ctypes.c_void_p * k)(*[t.data_ptr() for t in ycs])
        ld = (ctypes.c_int64 * k)(*[p.n for p in self.plans])
        _check(lib().mm_mvm_batch_run(self._h, vp, ld, yp, ld, float(shift), _stream_ptr(self._stream)))

    def run(self, vs, shift: float = 0.0):
        """vs: list of (n_k,) or (n_k, nrhs) tensors; returns the list of products."""
        vcs = [_colmajor(v, p.n) for v, p in zip(vs, self.plans)]
        ycs = [_torch().empty_like(vc) for vc in vcs]
        self.run_raw(vcs, ycs, shift)
        return [yc.view(-1) if v.dim() == 1 else yc.t() for v, yc in zip(vs, ycs)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mm_mvm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
# Every callback pair ever registered, kept for the life of the process: a
# buffer returns to the allocator that provided it, so a plan, solver or batch
# created under one pair still calls that pair's free thunk after a switch.
_allocator_refs = []


def use_torch_allocator(on: bool = True):
    """Route every device buffer of the library through torch's caching
    allocator (mm_set_allocator), or back to hipMalloc with on=False.  Objects
    created before a switch keep freeing through the allocator that gave them
    their buffers (its callbacks are never released).  Call while no library
    objects are being created or destroyed."""
    if not on:
        _check(lib().mm_set_allocator(None, None, None))
        return
    torch = _torch()

    def _alloc(nbytes, stream, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
        except Exception:
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    refs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _allocator_refs.append(refs)
    _check(lib().mm_set_allocator(ctypes.cast(refs[0], ctypes.c_void_p), ctypes.cast(refs[1], ctypes.c_void_p),
                                  None))


def lanczos_logquad(alpha, beta) -> float:
    """e_1^T log(T) e_1 of the Lanczos matrix of CG coefficients (host computation)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    m = len(a)
    out = ctypes.c_double()
    bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(b) else None
    _check(lib().mm_lanczos_logquad(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), bp, m, ctypes.byref(out)))
    return out.value


def levels(n: int) -> int:
    """ceil(log2 n): number of divide-and-conquer levels of a point set of size n."""
    L = 0
    while (1 << L) < n:
        L += 1
    return L


def passes(n: int, d: int) -> int:
    """Number of divide-and-conquer passes: 1 (d=1), L (d=2), L(L+1)/2 (d=3)."""
    if n < 2:
        return 0
    L = levels(n)
    return 1 if d == 1 else (L if d == 2 else L * (L + 1) // 2)
