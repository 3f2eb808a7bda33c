"""L-BFGS for the lower-level problem (Section 5: history 10, backtracking, gradient-norm stop).

The paper fixes the history size and the gradient-norm stop but not the line
search details; reading used here (and by the HIP library):
  * two-loop recursion with initial scaling gamma = s^T y / y^T y of the newest pair;
  * backtracking Armijo line search, c1 = 1e-4, halving, first trial step 1
    (the very first iteration, with no pair yet, tries 1 / ||grad||);
  * a pair is kept only if s^T y > 1e-12 ||s|| ||y||;
  * a direction that is not a descent direction is replaced by -grad;
  * stop when ||grad||_2 <= gtol or after max_iter iterations.
Warm starts simply pass the previous solution as ``x0``.
"""
from __future__ import annotations

import numpy as np


def lbfgs(fun, grad, x0, gtol: float = 1e-8, max_iter: int = 20000, m: int = 10,
          c1: float = 1e-4, max_backtrack: int = 60):
    """Minimise ``fun``; returns (x, info) with info = {iters, grad_norm, nfev, converged}."""
    x = np.array(x0, dtype=np.float64).ravel().copy()
    f = fun(x)
    g = grad(x)
    S, Y = [], []
    nfev = 1
    it = 0
    gnorm = float(np.linalg.norm(g))
    while gnorm > gtol and it < max_iter:
        # two-loop recursion: d = -H_k g
        q = g.copy()
        alphas = []
        for s_j, y_j in reversed(list(zip(S, Y))):
            rho = 1.0 / float(y_j @ s_j)
            a = rho * float(s_j @ q)
            alphas.append((a, rho))
            q -= a * y_j
        if S:
            gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
        else:
            gamma = 1.0 / gnorm
        r = gamma * q
        for (s_j, y_j), (a, rho) in zip(zip(S, Y), reversed(alphas)):
            b = rho * float(y_j @ r)
            r += (a - b) * s_j
        d = -r
        slope = float(g @ d)
        if slope >= 0.0:
            d = -g
            slope = -gnorm * gnorm
        # backtracking Armijo
        t = 1.0
        for _ in range(max_backtrack):
            x_new = x + t * d
            f_new = fun(x_new)
            nfev += 1
            if f_new <= f + c1 * t * slope:
                break
            t *= 0.5
        else:
            break
        g_new = grad(x_new)
        s_vec, y_vec = x_new - x, g_new - g
        sy = float(s_vec @ y_vec)
        if sy > 1e-12 * np.linalg.norm(s_vec) * np.linalg.norm(y_vec):
            S.append(s_vec)
            Y.append(y_vec)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        x, f, g = x_new, f_new, g_new
        gnorm = float(np.linalg.norm(g))
        it += 1
    return x, {"iters": it, "grad_norm": gnorm, "nfev": nfev, "converged": gnorm <= gtol, "f": f}


def newton_polish(grad, dense_hessian, x, steps: int = 5):
    """A few dense Newton steps x -= H^{-1} grad (tiny images; for finite-difference pins)."""
    x = np.array(x, dtype=np.float64).copy()
    for _ in range(steps):
        x = x - np.linalg.solve(dense_hessian(x), grad(x))
    return x
