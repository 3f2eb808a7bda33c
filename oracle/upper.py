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

Batch training with Adam (Section 5.2 trains on a batch of images with Adam): the upper loss
is the sum over the images of 1/2 ||x_hat_k - x*_k||^2 (the config's batch loss is a sum), so
its hypergradient is the sum of the images' J_k w_k, each from its own recycled solve (own
recycle space, own warm start).  Adam (Kingma and Ba, 2015): m = b1 m + (1 - b1) g,
v = b2 v + (1 - b2) g^2, step = lr m_hat / (sqrt(v_hat) + eps) with the bias corrections
m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t); theta -= step.  Filter regularisers: each
filter's tap block of the step is projected onto zero mean, so the filters stay zero-mean.

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
                   warm: bool = True, recurrence: str = "textbook"):
    """Solve the frozen sequence with recycled CG; returns per-system records.  recurrence:
    the CG form (recycled_cg's option)."""
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
                                 hg_tol=hg_rel * prev_hg if use_hg else 0.0, max_iter=max_iter, v_cap=v_cap,
                                 recurrence=recurrence)
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


def adam_step(theta, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
              zero_mean_blocks=None):
    """One Adam update (t >= 1); zero_mean_blocks = (n_filters, fsize) projects each filter's tap
    block of the step onto zero mean.  Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    step = lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    if zero_mean_blocks is not None:
        nf, fs = zero_mean_blocks
        f2 = fs * fs
        step = step.reshape(nf, 1 + f2).copy()
        step[:, 1:] -= step[:, 1:].mean(axis=1, keepdims=True)
        step = step.ravel()
    return theta - step, m, v


def train_adam(probs, xstars, theta0, steps: int, lr: float = 1e-2, s: int = 0, stop: str = "resid",
               tol: float = 1e-10, hg_rel: float = 1e-8, v_cap: int = 64, gtol: float = 1e-8,
               lbfgs_iters: int = 20000, max_iter: int = 20000, zero_mean_blocks=None, recurrence: str = "textbook"):
    """Adam on the summed upper loss of a batch of images (problems ``probs`` with ground truths
    ``xstars``), ``steps`` updates from theta0.  Per step and image: lower-level L-BFGS solve at
    the current theta warm started from that image's previous reconstruction; refresh of the
    image's recycle space (s > 0; from the previous step's); recycled CG on H_k w_k = x_hat_k - x*_k
    warm started from the image's previous w_k (the error-estimate stop at hg_rel times the image's
    previous hypergradient norm, when it has a recycle space); J_k w_k summed into the gradient.
    Returns per-step records: theta (steps + 1), loss (steps + 1: the summed upper loss at each
    theta), gradient norms, Hessian-solve iterations per image.  recurrence: the CG form
    (recycled_cg's option)."""
    theta = np.array(theta0, dtype=np.float64)
    xs = [np.asarray(x).ravel() for x in xstars]
    K = len(probs)

    def lower(k, th, xinit):
        x, _ = lbfgs.lbfgs(lambda v: probs[k].phi(v, th), lambda v: probs[k].grad(v, th), xinit, gtol=gtol,
                           max_iter=lbfgs_iters)
        return x

    xh = [lower(k, theta, probs[k].y.ravel()) for k in range(K)]
    U = [None] * K
    V = [None] * K
    w = [np.zeros_like(x) for x in xs]
    prev_hg = [None] * K
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = {"theta": [theta.copy()], "loss": [sum(upper_loss(xh[k], xs[k]) for k in range(K))], "grad_norm": [],
            "iters": []}
    for t in range(1, steps + 1):
        grad = np.zeros_like(theta)
        its = []
        for k in range(K):
            hvp = lambda q, k=k: probs[k].hvp(xh[k], theta, q)
            jac = lambda q, k=k: probs[k].jac_apply(xh[k], theta, q)
            rs = {"U": None, "C": None, "Z": None, "mu": None}
            if s and (U[k] is not None or V[k] is not None):
                rs = recycle.refresh(hvp, jac, U[k], V[k], s)
            use_hg = stop == "hgerr" and rs["U"] is not None and prev_hg[k] is not None
            res = krylov.recycled_cg(hvp, xh[k] - xs[k], w[k], rs["U"], rs["C"], rs["Z"], rs["mu"], tol=tol,
                                     stop="hgerr" if use_hg else "resid",
                                     hg_tol=hg_rel * prev_hg[k] if use_hg else 0.0, max_iter=max_iter,
                                     v_cap=v_cap if s else 0, recurrence=recurrence)
            U[k], V[k], w[k] = rs["U"], res["V"], res["w"]
            hg = jac(w[k])
            prev_hg[k] = float(np.linalg.norm(hg))
            grad += hg
            its.append(res["iters"])
        theta, m, v = adam_step(theta, grad, m, v, t, lr, zero_mean_blocks=zero_mean_blocks)
        xh = [lower(k, theta, xh[k]) for k in range(K)]
        hist["theta"].append(theta.copy())
        hist["loss"].append(sum(upper_loss(xh[k], xs[k]) for k in range(K)))
        hist["grad_norm"].append(float(np.linalg.norm(grad)))
        hist["iters"].append(its)
    return hist
