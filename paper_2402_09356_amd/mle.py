"""Maximum-likelihood estimation of the Matern parameters (host driver).

Nelder-Mead (Nelder & Mead 1965, with the standard coefficients of Lagarias,
Reeds, Wright & Wright 1998: reflection 1, expansion 2, contraction 1/2,
shrink 1/2) over log theta, so the search respects theta > 0.  Every
objective value is one l(theta) evaluation through the GPU library
(generation, compression, TLR Cholesky, solve); a failed factorisation
(l = -inf) is an infinitely bad point.  The fit stops when the spread of l
over the simplex falls below `ftol` (the paper's optimisation tolerance,
Section 5.1.1, is 1e-9) or after `max_evals` evaluations.

The simplex method itself is deterministic host code; `nelder_mead` takes any
objective and is tested on the CPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class NMResult:
    x: np.ndarray
    f: float
    evals: int
    iterations: int
    converged: bool
    history: list = field(default_factory=list)


def nelder_mead(fun, x0, step=0.1, ftol=1e-9, max_evals=1000) -> NMResult:
    """Minimise fun from x0; initial simplex x0 + step * e_i."""
    x0 = np.asarray(x0, dtype=np.float64)
    dim = x0.size
    simplex = [x0.copy()] + [x0 + step * np.eye(dim)[i] for i in range(dim)]
    values = []
    evals = 0
    history = []

    def f(x):
        nonlocal evals
        evals += 1
        v = float(fun(x))
        if not math.isfinite(v):
            v = math.inf
        history.append((x.copy(), v))
        return v

    values = [f(x) for x in simplex]
    it = 0
    converged = False
    while evals < max_evals:
        order = np.argsort(values, kind="stable")
        simplex = [simplex[i] for i in order]
        values = [values[i] for i in order]
        if math.isfinite(values[-1]) and values[-1] - values[0] <= ftol:
            converged = True
            break
        it += 1
        centroid = np.mean(simplex[:-1], axis=0)
        worst = simplex[-1]
        xr = centroid + (centroid - worst)
        fr = f(xr)
        if values[0] <= fr < values[-2]:
            simplex[-1], values[-1] = xr, fr
            continue
        if fr < values[0]:
            xe = centroid + 2.0 * (centroid - worst)
            fe = f(xe)
            if fe < fr:
                simplex[-1], values[-1] = xe, fe
            else:
                simplex[-1], values[-1] = xr, fr
            continue
        if fr < values[-1]:  # outside contraction
            xc = centroid + 0.5 * (xr - centroid)
            fc = f(xc)
            if fc <= fr:
                simplex[-1], values[-1] = xc, fc
                continue
        else:  # inside contraction
            xc = centroid + 0.5 * (worst - centroid)
            fc = f(xc)
            if fc < values[-1]:
                simplex[-1], values[-1] = xc, fc
                continue
        # shrink towards the best vertex
        for i in range(1, dim + 1):
            simplex[i] = simplex[0] + 0.5 * (simplex[i] - simplex[0])
            values[i] = f(simplex[i])
    best = int(np.argmin(values))
    return NMResult(x=simplex[best], f=values[best], evals=evals, iterations=it, converged=converged,
                    history=history)


@dataclass
class FitResult:
    theta: tuple
    loglik: float
    evals: int
    converged: bool
    f_identifiable: float  # sigma2 * beta^(-2 nu)


def fit(plan, ws, locs, z, tol, start=(0.5, 0.05, 1.0), nu=None, ftol=1e-9, max_evals=1000, step=0.1,
        progress=None):
    """MLE of theta = (sigma2, beta, nu) by l(theta) evaluations on the GPU.

    plan/ws: a binding.Plan and its workspace; locs/z: ordered device tensors.
    With `nu` given the smoothness is held fixed and only (sigma2, beta) are
    fitted.  `progress(evals, best_l)` is called every 25 evaluations."""
    import torch

    out = torch.empty(3, dtype=torch.float64, device=z.device)

    def theta_of(x):
        if nu is None:
            return (math.exp(x[0]), math.exp(x[1]), math.exp(x[2]))
        return (math.exp(x[0]), math.exp(x[1]), float(nu))

    count = [0]
    best = [-math.inf]

    def objective(x):
        th = theta_of(x)
        plan.loglik(ws, locs, z, th, tol, out=out)
        val = float(out[2].item())
        count[0] += 1
        best[0] = max(best[0], val)
        if progress is not None and count[0] % 25 == 0:
            progress(count[0], best[0])
        return -val

    x0 = np.log(np.asarray(start if nu is None else start[:2], dtype=np.float64))
    res = nelder_mead(objective, x0, step=step, ftol=ftol, max_evals=max_evals)
    th = theta_of(res.x)
    return FitResult(theta=th, loglik=-res.f, evals=res.evals, converged=res.converged,
                     f_identifiable=th[0] * th[1] ** (-2.0 * th[2]))
