"""Hyperparameter estimation by gradient ascent on the log marginal likelihood.

Section 3 fits the lengthscale and the output scale with ADAM (Kingma & Ba)
on eq. gp_log_likelihood, whose gradient is eq.
gp_log_likelihood_derivative, and Algorithm 1 wraps that ascent in an
alternation with a closed-form update of the noise level (after Sigrist) and
the generalised least squares fixed effects.  This module is orchestration
only: every product, solve, log-determinant and trace estimate runs in the
HIP library (``Plan.lml``, ``Plan.cg_solve``); the optimiser itself updates
three scalars on the host.

Readings (the paper leaves them open):

* The ascent runs on (log lengthscale, log output scale) so that both stay
  positive; the learning rate falls linearly from ``lr0`` to ``lr1`` over
  ``max_iter`` iterations (0.005 -> 0.0005 over 20000 in Section 3).
* One likelihood evaluation per iteration: it is taken at the new (output
  scale, lengthscale) with the previous noise level, so its quadratic form
  y^T (K + sigma^2 I)^{-1} y gives the noise update
  sigma^2 <- sigma^2 * quad / N (the profile update of Algorithm 1 written
  for K + sigma^2 I = sigma^2 (K~ + I)) and its gradient drives the next step.
* The stop tests are those of Section 3: the gradient norm (in the raw
  parameters) below ``grad_tol``, or a parameter change below ``param_tol``
  over ``window`` iterations.
* ``algorithm1`` returns the GLS coefficients at the fitted parameters (one
  more GLS solve after the last round).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import Kernel, Plan


class Adam:
    """ADAM ascent on a parameter vector (Kingma & Ba, Algorithm 1 of their
    paper, with the bias corrections)."""

    def __init__(self, theta, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.theta = np.asarray(theta, dtype=np.float64).copy()
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.beta1, self.beta2, self.eps = beta1, beta2, eps

    def step(self, grad, lr: float) -> np.ndarray:
        """theta <- theta + lr * mhat / (sqrt(vhat) + eps): one ascent step."""
        g = np.asarray(grad, dtype=np.float64)
        self.t += 1
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * g
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * g * g
        mhat = self.m / (1.0 - self.beta1 ** self.t)
        vhat = self.v / (1.0 - self.beta2 ** self.t)
        self.theta = self.theta + lr * mhat / (np.sqrt(vhat) + self.eps)
        return self.theta


def learning_rate(j: int, max_iter: int, lr0: float, lr1: float) -> float:
    """Linear decay from lr0 (iteration 0) to lr1 (iteration max_iter)."""
    f = min(max(j / max(max_iter, 1), 0.0), 1.0)
    return lr0 + (lr1 - lr0) * f


@dataclass
class AscentResult:
    lengthscale: float
    outputscale2: float
    sigma2: float
    iters: int
    stopped: str                      # "grad", "param", "max_iter"
    history: List[dict] = field(default_factory=list)


def gradient_ascent(plan: Plan, y, sigma2: float, probes, *, lr0: float = 0.005, lr1: float = 0.0005,
                    max_iter: int = 20000, grad_tol: float = 1e-3, param_tol: float = 1e-4,
                    window: int = 100, rtol: float = 1e-5, maxit: int = 20000,
                    update_sigma: bool = True) -> AscentResult:
    """ADAM on (lengthscale, output scale) of the plan's kernel for the
    centred targets y (device tensor), with the noise update of Algorithm 1
    when update_sigma.  The plan's kernel is updated in place."""
    k0 = plan.kernel
    two_nu, form = k0.two_nu, k0.form
    ell, s2 = float(k0.lengthscale), float(k0.outputscale2)
    n = plan.n
    opt = Adam([math.log(ell), 0.5 * math.log(s2)])       # log l, log varsigma
    hist: List[dict] = []
    recent: List[np.ndarray] = []
    stopped = "max_iter"
    j = 0
    for j in range(1, max_iter + 1):
        out = plan.lml(y, sigma2, probes, maxit=maxit, rtol=rtol, raise_on_error=False)
        if out["status"] not in ("MM_OK", "MM_ERR_NOCONV"):
            raise RuntimeError("likelihood evaluation failed: %s" % out["status"])
        # the quadratic form at the current (varsigma, l) and the previous sigma2
        if update_sigma and j > 1:
            sigma2 = sigma2 * out["quad"] / n
        g_ell = out["dlml_dlengthscale"]
        g_vs = out["dlml_doutputscale2"] * 2.0 * math.sqrt(s2)      # dL/dvarsigma
        grad_norm = math.hypot(g_ell, g_vs)
        hist.append({"iter": j, "lml": out["lml"], "lengthscale": ell, "outputscale2": s2, "sigma2": sigma2,
                     "grad_norm": grad_norm, "cg_iters": out["iters"]})
        if grad_norm < grad_tol:
            stopped = "grad"
            break
        # chain rule to the log parameters, then one ascent step
        theta = opt.step([g_ell * ell, g_vs * math.sqrt(s2)], learning_rate(j - 1, max_iter, lr0, lr1))
        ell, s2 = math.exp(theta[0]), math.exp(2.0 * theta[1])
        plan.set_kernel(Kernel(two_nu, form, ell, s2))
        recent.append(np.array([ell, s2]))
        if len(recent) > window:
            recent.pop(0)
            if np.linalg.norm(recent[-1] - recent[0]) < param_tol:
                stopped = "param"
                break
    return AscentResult(ell, s2, sigma2, j, stopped, hist)


@dataclass
class FitResult:
    lengthscale: float
    outputscale2: float
    sigma2: float
    beta: np.ndarray
    rounds: int
    ascents: List[AscentResult]


def algorithm1(x, y, kernel: Kernel, sigma2: float, probes, *, eps_beta: float = 1e-3, max_rounds: int = 10,
               **ascent_kw) -> FitResult:
    """Algorithm 1: OLS-centred ascent, then rounds of GLS fixed effects
    (running average of the GLS coefficients), re-centring and ascent until
    successive GLS coefficients differ by less than eps_beta.  x, y, probes
    are device tensors; H = [1, x_1 .. x_d]."""
    import torch
    n, d = x.shape
    H = torch.cat([torch.ones(n, 1, dtype=torch.float64, device=x.device), x], dim=1)
    Hn = H.cpu().numpy()
    yn = y.cpu().numpy()
    beta_ols = np.linalg.lstsq(Hn, yn, rcond=None)[0]
    plan = Plan(x, kernel)
    ascents = []
    try:
        yc = y - H @ torch.as_tensor(beta_ols, device=x.device)
        res = gradient_ascent(plan, yc, sigma2, probes, **ascent_kw)
        ascents.append(res)
        sigma2 = res.sigma2
        beta_avg = np.zeros(d + 1)
        beta_old = beta_ols
        beta_gls = beta_ols
        rounds = 0
        for i in range(1, max_rounds + 1):
            rounds = i
            _, beta_gls, _ = plan.cg_solve(y, sigma2, fixed_effects=True, rtol=ascent_kw.get("rtol", 1e-5),
                                           maxit=ascent_kw.get("maxit", 20000), raise_on_error=False)
            beta_avg = (i - 1) / i * beta_avg + beta_gls / i
            yc = y - H @ torch.as_tensor(beta_avg, device=x.device)
            res = gradient_ascent(plan, yc, sigma2, probes, **ascent_kw)
            ascents.append(res)
            sigma2 = res.sigma2
            change = float(np.linalg.norm(beta_gls - beta_old))
            beta_old = beta_gls
            if change < eps_beta:
                break
        # the GLS coefficients at the fitted parameters (the last round's are
        # within eps_beta of them once the rounds have converged)
        _, beta_fit, _ = plan.cg_solve(y, sigma2, fixed_effects=True, rtol=ascent_kw.get("rtol", 1e-5),
                                       maxit=ascent_kw.get("maxit", 20000), raise_on_error=False)
        k = plan.kernel
        return FitResult(k.lengthscale, k.outputscale2, sigma2, np.asarray(beta_fit), rounds, ascents)
    finally:
        plan.close()
