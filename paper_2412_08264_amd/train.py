"""End-to-end bilevel training on the GPU: gradient descent on theta (Algorithm 2) with the
backtracking line search of Algorithm 1, every hypergradient from a recycled Hessian solve.

Per outer iteration i, all on the library's kernels:
  * refresh of the recycle space from the previous system's space and Krylov basis at the new
    (x_hat_i, theta_i) (bl_recycle_update, RGen-L(R) unless another rule is chosen);
  * the Hessian solve H w = x_hat_i - x*, warm started from the previous solution, by recycled CG
    or RMINRES with the hypergradient-error stop (threshold hg_rel times the previous
    hypergradient norm) or the residual stop;
  * the hypergradient J w, the descent direction d = -grad L, and the Armijo backtracking
    tau = beta rho^(j-1), accept when L(theta + tau d) <= L(theta) + eta tau grad L . d, each trial
    point needing a lower-level L-BFGS solve warm started from the previous trial's minimiser;
    next beta = 2 tau.
The host holds theta (p values) and the scalar decisions; the upper loss 1/2 ||x - x*||^2 is a
device reduction.
"""
from __future__ import annotations

import time

import numpy as np

from . import bilevel as B


def upper_loss(x, xstar) -> float:
    d = x - xstar
    return 0.5 * float((d * d).sum())


def train(S: B.Session, y, xstar, theta0, outer: int, s: int = 0, solver: str = "cg", stop: str = "resid",
          tol: float = 1e-10, hg_rel: float = 1e-8, check_every: int = 1, gtol: float = 1e-8, eta: float = 1e-4,
          rho: float = 0.5, beta0: float = 1.0, max_backtrack: int = 30, lbfgs_iters: int = 20000,
          max_iter: int = 20000, select: str = "rgen-l-r") -> dict:
    """Run ``outer`` descent steps from theta0.  ``S`` is a Session of the problem (its recycle
    capacity bounds s); y, xstar are device vectors.  solver: "cg" | "rminres".  Returns per-step
    records: theta (outer + 1 values), loss (outer + 1), accepted tau, Hessian-solve iterations,
    lower-level L-BFGS iterations, and wall-clock seconds of the lower solves, refreshes,
    Hessian solves and hypergradients."""
    import torch

    if solver not in ("cg", "rminres"):
        raise ValueError(f"unknown solver {solver!r}")
    theta = np.array(theta0, dtype=np.float64)
    x = y.clone()
    clock = {"lower": 0.0, "refresh": 0.0, "solve": 0.0, "hypergradient": 0.0}

    def timed(key, fn, *a, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn(*a, **kw)
        torch.cuda.synchronize()
        clock[key] += time.perf_counter() - t0
        return out

    lb = [timed("lower", S.lower_solve, theta, y, x, gtol=gtol, max_iter=lbfgs_iters).iters]
    c1 = upper_loss(x, xstar)
    beta = beta0
    S.reset()
    w = torch.zeros_like(x)
    prev_hg = None
    hist = {"theta": [], "loss": [], "tau": [], "iters": [], "lbfgs_iters": lb, "seconds": clock}
    for i in range(outer):
        g = x - xstar
        if s and i > 0:
            timed("refresh", S.refresh, theta, x, s=s, select=select)
        use_hg = stop == "hgerr" and S.rs.s_cur > 0 and prev_hg is not None and select.startswith("rgen")
        st = timed("solve", S.solve, theta, x, g, w, tol=tol, stop="hgerr" if use_hg else "resid",
                   hg_tol=hg_rel * prev_hg if use_hg else 0.0, check_every=check_every if use_hg else 1,
                   store_basis=s > 0, recycle=s > 0, max_iter=max_iter, rr_every=0, method=solver)
        grad = timed("hypergradient", S.hypergradient, theta, x, w)
        prev_hg = float(np.linalg.norm(grad))
        hist["theta"].append(theta.copy())
        hist["loss"].append(c1)
        hist["iters"].append(st.iters)
        d = -grad
        c2 = float(grad @ d)
        xprev = x
        tau_acc = 0.0
        for j in range(1, max_backtrack + 1):
            tau = beta * rho ** (j - 1)
            th_j = theta + tau * d
            x_j = xprev.clone()
            lb.append(timed("lower", S.lower_solve, th_j, y, x_j, gtol=gtol, max_iter=lbfgs_iters).iters)
            c0 = upper_loss(x_j, xstar)
            if c0 <= c1 + eta * tau * c2:
                theta, x, c1, beta, tau_acc = th_j, x_j, c0, 2.0 * tau, tau
                break
            xprev = x_j
        else:
            beta = beta * rho ** max_backtrack
        hist["tau"].append(tau_acc)
    hist["theta"].append(theta.copy())
    hist["loss"].append(c1)
    return hist
