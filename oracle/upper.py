"""Upper level: frozen trajectories and recycled solve sequences (Sections 2.1 and 5).

Trajectory (Algorithms 1 and 2).  The printed sign conventions disagree (the
Armijo rule steps along -d while the algorithms step along +d with
d = D^2_{theta x} Phi^T w = -grad L); reading used: d = -grad L, accept
theta + tau d when L(theta + tau d) <= L(theta) + eta tau grad L^T d, tau = beta rho^{j-1},
eta = 1e-4, rho = 0.5, beta_0 = 1, next beta = 2 tau.  Lower-level solves are
warm started from the previous reconstruction.

Training (Algorithm 2 with Algorithm 1, end to end): the same descent, with every Hessian
system solved by recycled CG or RMINRES (refresh of U, C, Z, mu from the previous system's
space and Krylov basis, warm start from the previous solution) instead of the reference solve;
the hypergradient-error stop uses ``hg_rel`` times the previous hypergradient norm.

Solve sequence (Section 5's fixed-sequence protocol).  Given the frozen
{theta_i, x_hat_i}, solve every H^{(i)} w = g^{(i)} with recycled CG, warm started
from w^{(i-1)}, refreshing U, C, Z, mu between systems (outer RGen-L(R)).
The first system has no recycle space and uses the residual test.  With the
hypergradient-error test the threshold is ``hg_rel`` times the norm of the
previous system's hypergradient.
"""
from __future__ import annotations

import numpy as np

from . import krylov, lbfgs, recycle, rminres
from .problem import upper_loss


def hypergradient(prob, xhat, theta, xstar, w0=None, tol: float = 1e-13):
    """Reference hypergradient J H^{-1} g (Section 5: no recycling, tolerance 1e-13)."""
    g = np.asarray(xhat).ravel() - np.asarray(xstar).ravel()
    w, _ = krylov.reference_solve(lambda v: prob.hvp(xhat, theta, v), g, tol=tol)
    return prob.jac_apply(xhat, theta, w), w


def trajectory(prob, xstar, theta0, outer: int, gtol: float = 1e-8, x0=None, eta: float = 1e-4,
               rho: float = 0.5, beta0: float = 1.0, max_backtrack: int = 30, lbfgs_iters: int = 20000):
    """Gradient descent with backtracking; returns lists of theta_i and x_hat_i (i < outer)."""
    theta = np.array(theta0, dtype=np.float64)
    xs = np.asarray(xstar).ravel()
    x0 = prob.y.ravel() if x0 is None else np.asarray(x0).ravel()

    def solve_lower(th, xinit):
        x, info = lbfgs.lbfgs(lambda v: prob.phi(v, th), lambda v: prob.grad(v, th), xinit, gtol=gtol,
                              max_iter=lbfgs_iters)
        return x

    xhat = solve_lower(theta, x0)
    c1 = upper_loss(xhat, xs)
    beta = beta0
    thetas, xhats = [], []
    for _ in range(outer):
        thetas.append(theta.copy())
        xhats.append(xhat.copy())
        grad_L, _ = hypergradient(prob, xhat, theta, xs)
        d = -grad_L
        c2 = float(grad_L @ d)
        xprev = xhat
        accepted = False
        for j in range(1, max_backtrack + 1):
            tau = beta * rho ** (j - 1)
            th_j = theta + tau * d
            x_j = solve_lower(th_j, xprev)
            c0 = upper_loss(x_j, xs)
            if c0 <= c1 + eta * tau * c2:
                theta, xhat, c1, beta = th_j, x_j, c0, 2.0 * tau
                accepted = True
                break
            xprev = x_j
        if not accepted:
            # no decrease found: keep theta (the sequence then repeats the last system)
            beta = beta * rho ** max_backtrack
    return thetas, xhats


def solve_sequence(prob, thetas, xhats, xstar, s: int, tol: float = 1e-10, stop: str = "resid",
                   hg_rel: float = 1e-7, v_cap: int = 64, max_iter: int = 10000, recycle_on: bool = True,
                   warm: bool = True):
    """Solve the frozen sequence with recycled CG; returns per-system records."""
    xs = np.asarray(xstar).ravel()
    U = V = None
    w_prev = None
    prev_hg = None
    out = []
    for th, xh in zip(thetas, xhats):
        hvp = lambda v, xh=xh, th=th: prob.hvp(xh, th, v)
        jac = lambda v, xh=xh, th=th: prob.jac_apply(xh, th, v)
        g = xh - xs
        rs = {"U": None, "C": None, "Z": None, "mu": None, "t": 0}
        if recycle_on and (U is not None or V is not None):
            rs = recycle.refresh(hvp, jac, U, V, s)
        use_hg = stop == "hgerr" and rs["U"] is not None and prev_hg is not None
        res = krylov.recycled_cg(hvp, g, w_prev if warm else None, rs["U"], rs["C"], rs["Z"], rs["mu"], tol=tol,
                                 stop="hgerr" if use_hg else "resid",
                                 hg_tol=hg_rel * prev_hg if use_hg else 0.0, max_iter=max_iter, v_cap=v_cap)
        hg = jac(res["w"])
        out.append({"w": res["w"], "iters": res["iters"], "status": res["status"], "hg": hg, "t": rs["t"],
                    "w0": w_prev, "rs": rs})
        U, V = rs["U"], res["V"]
        w_prev = res["w"]
        prev_hg = float(np.linalg.norm(hg))
    return out


def train(prob, xstar, theta0, outer: int, s: int = 0, solver: str = "cg", stop: str = "resid",
          tol: float = 1e-10, hg_rel: float = 1e-8, v_cap: int = 64, gtol: float = 1e-8, eta: float = 1e-4,
          rho: float = 0.5, beta0: float = 1.0, max_backtrack: int = 30, lbfgs_iters: int = 20000,
          max_iter: int = 20000):
    """Gradient descent with backtracking where each hypergradient comes from a recycled solve.

    solver "cg": recycled CG (its normalised residuals form the next basis); "rminres": RMINRES
    (its Lanczos vectors form the next basis).  Returns a dict of per-step records: theta, loss,
    accepted step tau, Hessian-solve iterations."""
    theta = np.array(theta0, dtype=np.float64)
    xs = np.asarray(xstar).ravel()
    x0 = prob.y.ravel()

    def solve_lower(th, xinit):
        x, _ = lbfgs.lbfgs(lambda v: prob.phi(v, th), lambda v: prob.grad(v, th), xinit, gtol=gtol,
                           max_iter=lbfgs_iters)
        return x

    xhat = solve_lower(theta, x0)
    c1 = upper_loss(xhat, xs)
    beta = beta0
    U = V = None
    w = np.zeros_like(xs)
    prev_hg = None
    hist = {"theta": [], "loss": [], "tau": [], "iters": []}
    for _ in range(outer):
        hvp = lambda v, xh=xhat, th=theta: prob.hvp(xh, th, v)
        jac = lambda v, xh=xhat, th=theta: prob.jac_apply(xh, th, v)
        g = xhat - xs
        rs = {"U": None, "C": None, "Z": None, "mu": None}
        if s and (U is not None or V is not None):
            rs = recycle.refresh(hvp, jac, U, V, s)
        use_hg = stop == "hgerr" and rs["U"] is not None and prev_hg is not None
        kw = dict(tol=tol, stop="hgerr" if use_hg else "resid", hg_tol=hg_rel * prev_hg if use_hg else 0.0,
                  max_iter=max_iter)
        if solver == "cg":
            res = krylov.recycled_cg(hvp, g, w, rs["U"], rs["C"], rs["Z"], rs["mu"], v_cap=v_cap, **kw)
            V = res["V"]
        else:
            res = rminres.rminres(hvp, g, w, rs["U"], rs["C"], rs["Z"], rs["mu"], v_cap=v_cap, **kw)
            V = res["V"]
        U = rs["U"]
        w = res["w"]
        grad_L = jac(w)
        prev_hg = float(np.linalg.norm(grad_L))
        hist["theta"].append(theta.copy())
        hist["loss"].append(c1)
        hist["iters"].append(res["iters"])
        d = -grad_L
        c2 = float(grad_L @ d)
        xprev = xhat
        tau_acc = 0.0
        for j in range(1, max_backtrack + 1):
            tau = beta * rho ** (j - 1)
            th_j = theta + tau * d
            x_j = solve_lower(th_j, xprev)
            c0 = upper_loss(x_j, xs)
            if c0 <= c1 + eta * tau * c2:
                theta, xhat, c1, beta, tau_acc = th_j, x_j, c0, 2.0 * tau, tau
                break
            xprev = x_j
        else:
            beta = beta * rho ** max_backtrack
        hist["tau"].append(tau_acc)
    hist["theta"].append(theta.copy())
    hist["loss"].append(c1)
    return hist
