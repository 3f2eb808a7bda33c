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

Batch training with Adam (train_adam): the summed upper loss over images sharing theta, every
step's Hessian solves advanced together by one batch engine (continuous admission), Adam on the
summed hypergradient.
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


def adam_update(theta, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
                zero_mean_blocks=None):
    """Adam (Kingma and Ba, 2015) on the host's p parameters; zero_mean_blocks = (n_filters, fsize)
    keeps each filter's taps zero-mean by projecting their step.  Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    step = lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    if zero_mean_blocks is not None:
        nf, fs = zero_mean_blocks
        step = step.reshape(nf, 1 + fs * fs).copy()
        step[:, 1:] -= step[:, 1:].mean(axis=1, keepdims=True)
        step = step.ravel()
    return theta - step, m, v


def train_adam(ctx: B.Context, problems, ys, xstars, theta0, steps: int, lr: float = 1e-2, s: int = 0,
               stop: str = "resid", tol: float = 1e-10, hg_rel: float = 1e-8, check_every: int = 1,
               v_cap: int = 64, gtol: float = 1e-8, lbfgs_iters: int = 20000, max_iter: int = 20000,
               zero_mean_blocks=None, rr_every: int = 50) -> dict:
    """Adam on the summed upper loss of a batch of images sharing theta (Section 5.2 trains on a
    batch with Adam).  ``ctx`` is a Context whose workspace covers every problem with recycle
    capacity (s, v_cap); ys, xstars are device vectors per image.

    Per step: every image's Hessian solve H_k w_k = x_hat_k - x*_k is admitted to one batch engine
    (its own recycle space refreshed from its previous space and Krylov basis, its own warm start
    and error-estimate threshold hg_rel times its previous hypergradient norm) and the engine
    advances them together; the hypergradient is the sum of the J_k w_k; Adam updates theta on the
    host; every image's lower-level problem is re-solved at the new theta, warm started from its
    previous reconstruction.  Returns per-step records: theta and summed loss (steps + 1 each),
    gradient norms, Hessian-solve iterations per image, and wall-clock seconds of the lower
    solves, refreshes, batched solves and hypergradients."""
    import torch

    K = len(problems)
    theta = np.array(theta0, dtype=np.float64)
    clock = {"lower": 0.0, "refresh": 0.0, "solve": 0.0, "hypergradient": 0.0}

    def timed(key, fn, *a, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn(*a, **kw)
        torch.cuda.synchronize()
        clock[key] += time.perf_counter() - t0
        return out

    xh = [y.clone() for y in ys]
    for k in range(K):
        timed("lower", ctx.lower_solve_p, problems[k], theta, ys[k], xh[k], gtol=gtol, max_iter=lbfgs_iters)
    recs = [B.Recycle(P.h * P.w, s, v_cap if s else 0, ctx.device, P) if s else None for P in problems]
    ws = [torch.zeros_like(x) for x in xh]
    prev_hg = [None] * K
    arena = sum(B.Engine.slot_bytes(P, s) for P in problems)
    eng = B.Engine(cap=min(K, 64), arena_bytes=arena, device=ctx.device, ctx=ctx.ctx)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    loss = lambda: sum(upper_loss(xh[k], xstars[k]) for k in range(K))
    hist = {"theta": [theta.copy()], "loss": [loss()], "grad_norm": [], "iters": [], "seconds": clock}
    try:
        for t in range(1, steps + 1):
            gs = [xh[k] - xstars[k] for k in range(K)]
            if s:
                for k in range(K):
                    if recs[k].rs.s_cur or recs[k].rs.v_cur:
                        timed("refresh", ctx.refresh_p, problems[k], recs[k], theta, xh[k], s=s)
            # the batched solve: admit as slots free up, advance all running solves together
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pending, slot_of, its = list(range(K)), {}, [0] * K
            while pending or slot_of:
                while pending:
                    k = pending[0]
                    use_hg = stop == "hgerr" and s and recs[k].rs.s_cur > 0 and prev_hg[k] is not None
                    opts = B.solve_opts(tol=tol, stop="hgerr" if use_hg else "resid",
                                        hg_tol=hg_rel * prev_hg[k] if use_hg else 0.0, max_iter=max_iter,
                                        check_every=check_every if use_hg else 1, rr_every=rr_every,
                                        store_basis=bool(s))
                    slot = eng.admit(problems[k], theta, xh[k], gs[k], ws[k], recs[k], opts)
                    if slot is None:
                        break
                    slot_of[slot] = k
                    pending.pop(0)
                for slot in eng.step():
                    k = slot_of.pop(slot)
                    st = eng.retire(slot)
                    if st.status != B.BL_OK:
                        raise B.BLError(st.status, f"batched Hessian solve of image {k}")
                    its[k] = st.iters
            torch.cuda.synchronize()
            clock["solve"] += time.perf_counter() - t0
            grad = np.zeros_like(theta)
            for k in range(K):
                hg = timed("hypergradient", ctx.hypergradient_p, problems[k], theta, xh[k], ws[k])
                prev_hg[k] = float(np.linalg.norm(hg))
                grad += hg
            theta, m, v = adam_update(theta, grad, m, v, t, lr, zero_mean_blocks=zero_mean_blocks)
            for k in range(K):
                timed("lower", ctx.lower_solve_p, problems[k], theta, ys[k], xh[k], gtol=gtol, max_iter=lbfgs_iters)
            hist["theta"].append(theta.copy())
            hist["loss"].append(loss())
            hist["grad_norm"].append(float(np.linalg.norm(grad)))
            hist["iters"].append(its)
    finally:
        eng.close()
    return hist
