"""Plain and recycled conjugate gradients for H w = g, with the two stop tests.

Recycled CG.  The paper's solver is RMINRES (Section 2.2.2, Algorithm 3): the
correction is V_k y + U z with the Lanczos vectors kept orthogonal to C = HU,
C^T C = I, and the coupled least-squares problem (eq. coupled) splitting into
eq. y_solve and eq. zk_answer.  The paper defines no recycled CG; the reading
used here is the Galerkin counterpart on the same augmented space: with
P = I - C C^T,
  1. r0 = g - H w0;  w0 += U C^T r0;  r0 -= C C^T r0     (as in Algorithm 3's set-up)
  2. CG on P H restricted to range(P): every H p is projected, q - C (C^T q),
     which is the augmented Lanczos relation (eq. arnoldi_aug_matrix) in CG form;
  3. the recycle-space coefficient accumulates z -= alpha C^T q and the solution is
     finished with w += U z, the CG analogue of eq. zk_answer.
With U empty it is textbook CG (Hestenes-Stiefel), by the same code path.

Stop tests (Section 4):
  * residual: ||r_j|| <= tol ||g|| (the paper's test is absolute; here relative);
  * hypergradient-error estimate (eq. hg-err-stop-lowrank): with Z = W V_H and mu the
    selected Ritz generalized singular values, ||mu . (Z^T r_j)|| <= hg_tol.
The first test at j = 0 allows zero iterations.

The solver also returns the CG coefficients alpha_j and rho_j = r_j . r_j of the iterations whose
normalised residual went into V (what the inner refresh of recycle.py reads through the
CG form of the Lanczos relation).
"""
from __future__ import annotations

import numpy as np

OK, NOT_CONVERGED, INDEFINITE = 0, 4, 5


def recycled_cg(hvp, g, w0=None, U=None, C=None, Z=None, mu=None, tol: float = 1e-10,
                stop: str = "resid", hg_tol: float = 0.0, max_iter: int = 10000, v_cap: int = 64,
                check_every: int = 1, recurrence: str = "textbook", record: bool = False):
    """Solve H w = g.  ``hvp(v)`` applies H.  Returns a dict (see keys at the end)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    n = g.size
    w = np.zeros(n) if w0 is None else np.array(w0, dtype=np.float64).ravel().copy()
    s = 0 if U is None else U.shape[1]
    r = g - hvp(w)
    if s:
        c0 = C.T @ r
        w = w + U @ c0
        r = r - C @ c0
    gnorm = float(np.linalg.norm(g))
    p = r.copy()
    rho = float(r @ r)
    zacc = np.zeros(s)
    V = []
    alphas, rhos = [], []       # CG coefficients of the iterations whose residual went into V
    hist_res, hist_nsc = [], []

    def nsc(rv):
        return float(np.linalg.norm(mu * (Z.T @ rv)))

    def met(rv, rho_v, j):
        res = np.sqrt(max(rho_v, 0.0))
        est = nsc(rv) if (Z is not None and mu is not None and len(mu)) else np.nan
        if record:
            hist_res.append(res)
            hist_nsc.append(est)
        if rho_v == 0.0:
            return True
        if j % check_every:
            return False
        if stop == "hgerr":
            return est <= hg_tol
        return res <= tol * gnorm

    status = OK
    iters = 0
    done = met(r, rho, 0)
    while not done and iters < max_iter:
        # V: basis of the generated Krylov space, one normalised residual per iteration run
        stored = len(V) < v_cap
        if stored:
            V.append(r / np.sqrt(rho))
            rhos.append(rho)
        q = hvp(p)
        e = C.T @ q if s else np.zeros(0)
        sigma = float(p @ q)
        if sigma <= 0.0:
            status = INDEFINITE
            break
        alpha = rho / sigma
        if stored:
            alphas.append(alpha)
        if recurrence == "single":
            rq, qq, ee = float(r @ q), float(q @ q), float(e @ e)
        w += alpha * p
        zacc -= alpha * e
        r -= alpha * (q - C @ e) if s else alpha * q
        rho_new = float(r @ r)
        iters += 1
        done = met(r, rho_new, iters)
        if done:
            rho = rho_new
            break
        if recurrence == "single":
            # Chronopoulos-Gear: beta from the recurrence of the projected residual's norm
            # (C^T r = 0, C^T C = I), anchored on the explicit r.r of the previous iterate
            beta = (rho - 2.0 * alpha * rq + alpha * alpha * (qq - ee)) / rho
        else:
            beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
    if not done and status == OK:
        status = NOT_CONVERGED
    if s:
        w = w + U @ zacc
    return {"w": w, "iters": iters, "status": status, "res_norm": float(np.sqrt(max(rho, 0.0))),
            "g_norm": gnorm, "V": np.stack(V, axis=1) if V else np.zeros((n, 0)),
            "hist_res": hist_res, "hist_nsc": hist_nsc, "r": r, "zacc": zacc,
            "alpha": np.array(alphas), "rho": np.array(rhos)}


def deflated_cg(hvp, g, w0=None, U=None, C=None, Z=None, mu=None, tol: float = 1e-10, stop: str = "resid",
                hg_tol: float = 0.0, max_iter: int = 10000, v_cap: int = 64, check_every: int = 1,
                record: bool = False):
    """Deflated CG of Saad, Yeung, Erhel and Guyomarc'h (2000): the reading of the recycled
    solver that the paper leaves open beside the Galerkin form above (Section 2.2.2 defines only
    RMINRES), with the recycle space U and C = H U of the refresh as the deflation space.  With
    E = U^T C (= U^T H U, symmetric positive definite):
      1. r = g - H w0;  w = w0 + U E^{-1} U^T r;  r -= C E^{-1} U^T r      (so U^T r = 0)
      2. mu = E^{-1} C^T r;  p = r - U mu
      3. per iteration: q = H p;  alpha = rho / (p . q);  w += alpha p;  r -= alpha q;
         rho' = r . r;  stop test;  beta = rho' / rho;  mu = E^{-1} C^T r;  p = r + beta p - U mu.
    The residuals stay orthogonal to U and the directions H-conjugate to it (C^T p = 0); the
    iterate minimises the energy-norm error over w0 + range(U) + the directions.  Same stop tests
    and returned keys as recycled_cg; V holds the normalised residuals."""
    g = np.asarray(g, dtype=np.float64).ravel()
    n = g.size
    w = np.zeros(n) if w0 is None else np.array(w0, dtype=np.float64).ravel().copy()
    s = 0 if U is None else U.shape[1]
    r = g - hvp(w)
    if s:
        E = 0.5 * (U.T @ C + C.T @ U)
        c = np.linalg.solve(E, U.T @ r)
        w = w + U @ c
        r = r - C @ c
    gnorm = float(np.linalg.norm(g))
    rho = float(r @ r)
    p = r - U @ np.linalg.solve(E, C.T @ r) if s else r.copy()
    V, hist_res, hist_nsc, P = [], [], [], []

    def met(rv, rho_v, j):
        res = np.sqrt(max(rho_v, 0.0))
        est = float(np.linalg.norm(mu * (Z.T @ rv))) if (Z is not None and mu is not None and len(mu)) else np.nan
        if record:
            hist_res.append(res)
            hist_nsc.append(est)
        if rho_v == 0.0:
            return True
        if j % check_every:
            return False
        if stop == "hgerr":
            return est <= hg_tol
        return res <= tol * gnorm

    status, iters = OK, 0
    done = met(r, rho, 0)
    while not done and iters < max_iter:
        if len(V) < v_cap:
            V.append(r / np.sqrt(rho))
        if record:
            P.append(p.copy())
        q = hvp(p)
        sigma = float(p @ q)
        if sigma <= 0.0:
            status = INDEFINITE
            break
        alpha = rho / sigma
        w += alpha * p
        r -= alpha * q
        rho_new = float(r @ r)
        iters += 1
        done = met(r, rho_new, iters)
        if done:
            rho = rho_new
            break
        beta = rho_new / rho
        p = r + beta * p - (U @ np.linalg.solve(E, C.T @ r) if s else 0.0)
        rho = rho_new
    if not done and status == OK:
        status = NOT_CONVERGED
    return {"w": w, "iters": iters, "status": status, "res_norm": float(np.sqrt(max(rho, 0.0))),
            "g_norm": gnorm, "V": np.stack(V, axis=1) if V else np.zeros((n, 0)),
            "hist_res": hist_res, "hist_nsc": hist_nsc, "r": r, "P": P}


def cg(hvp, g, w0=None, tol: float = 1e-10, max_iter: int = 10000, v_cap: int = 64, record: bool = False,
       recurrence: str = "textbook"):
    """Plain CG: the recycled solver with an empty recycle space."""
    return recycled_cg(hvp, g, w0, tol=tol, max_iter=max_iter, v_cap=v_cap, record=record, recurrence=recurrence)


def reference_solve(hvp, g, tol: float = 1e-13, max_iter: int = 100000, replace_every: int = 50):
    """High-accuracy reference (Section 5: no recycling, tolerance 1e-13).

    Cold-start CG; every ``replace_every`` iterations the recursive residual is
    replaced by the true residual g - H w, and the run stops at the tolerance or
    when the true residual stops decreasing over a window.
    """
    g = np.asarray(g, dtype=np.float64).ravel()
    w = np.zeros_like(g)
    r = g.copy()
    p = r.copy()
    rho = float(r @ r)
    gnorm = float(np.linalg.norm(g))
    best = np.inf
    stall = 0
    it = 0
    while it < max_iter:
        if np.sqrt(rho) <= tol * gnorm:
            break
        q = hvp(p)
        alpha = rho / float(p @ q)
        w += alpha * p
        r -= alpha * q
        it += 1
        if it % replace_every == 0:
            r = g - hvp(w)
            tr = float(np.linalg.norm(r))
            if tr <= tol * gnorm:
                break
            if tr < 0.5 * best:
                best, stall = tr, 0
            else:
                stall += 1
                if stall >= 4:
                    break
        rho_new = float(r @ r)
        p = r + (rho_new / rho) * p
        rho = rho_new
    return w, it


def true_hg_error(J, Hinv_r):
    """||J H^{-1} r|| (eq. hg-error-stop), for diagnostics with dense J and H^{-1} r."""
    return float(np.linalg.norm(J @ Hinv_r))
