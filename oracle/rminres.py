"""RMINRES for H w = g (Section 2.2.2, Algorithm 3) with the explicit residual of Appendix A.

Test infrastructure: a plain FP64 CPU implementation that the GPU path is checked against.

The correction is V_k y + U z (eq. correction_term) minimising the residual over the
augmented space (eq. coupled), with U, C = H U, C^T C = I, and the Lanczos vectors kept
orthogonal to C (eq. arnoldi_aug_matrix).  The steps follow Algorithm 3:
  set-up   r0 = g - H w0;  w0 += U C^T r0;  r0 -= C C^T r0;  beta_1 = ||r0||, v_1 = r0 / beta_1
  Lanczos  H v_k; b_k = U C^T H v_k; project against C; alpha_k; three-term recurrence;
           beta_{k+1} = ||v_{k+1}||
  QR       the two previous Givens rotations on the new column of T_k, then a new rotation
           annihilating beta_{k+1}; zeta_k = -s_k zeta_{k-1} (so |zeta_k| = ||r_k||)
  update   three-term recurrences of v~ and b~, and w_k = w_{k-1} + c_k zeta_{k-1} (v~_k - b~_k).

Two readings where the printed text conflicts with itself:
  * sign of b~ in the update: eq. zk_answer puts the recycle part of the correction at
    C^T r0 - C^T H V y, so b~ (the image of U C^T H V under the same recurrence as v~) enters
    with a minus sign, as in Appendix A's residual update; the algorithm's plus is a typo.
  * Appendix A's recurrences for H v~_k and H b~_k need H v~_{k-2} and H b~_{k-2} (the
    k - 2 terms of the v~ and b~ recurrences carry H like the k - 1 terms), so seven
    n-vectors are kept: r, H v_k, C C^T H v_k, and H v~, H b~ at k - 1 and k - 2.

Stop tests, taken on iterates j with j % check_every == 0 (and on any exact zero residual):
  * residual: |zeta_j| <= tol ||g|| (the paper's test is absolute; here relative, like CG);
  * hypergradient-error estimate (Section 4, eq. hg-err-stop-lowrank): ||mu . (Z^T r_j)|| <= hg_tol
    with r_j the explicit residual of Appendix A.
MINRES needs no definiteness: an indefinite H is solved, not reported.
"""
from __future__ import annotations

import numpy as np

OK, NOT_CONVERGED, BREAKDOWN = 0, 4, 6


def rminres(hvp, g, w0=None, U=None, C=None, Z=None, mu=None, tol: float = 1e-10, stop: str = "resid",
            hg_tol: float = 0.0, max_iter: int = 10000, check_every: int = 1, record: bool = False,
            v_cap: int = 64):
    """Solve H w = g by RMINRES.  ``hvp(v)`` applies H.  Returns a dict (keys at the end); "V"
    holds the Lanczos vectors v_1 .. v_m of the steps taken (m <= v_cap), a basis of the Krylov
    space K_m((I - C C^T) H, r0) for the next refresh."""
    g = np.asarray(g, dtype=np.float64).ravel()
    n = g.size
    w = np.zeros(n) if w0 is None else np.array(w0, dtype=np.float64).ravel().copy()
    s = 0 if U is None else U.shape[1]
    zero = np.zeros(n)

    # set-up: residual of the warm start, its recycle-space part moved into w
    r = g - hvp(w)
    if s:
        c0 = C.T @ r
        w = w + U @ c0
        r = r - C @ c0
    gnorm = float(np.linalg.norm(g))
    beta = float(np.linalg.norm(r))          # beta_1
    v_prev = zero
    v = r / beta if beta > 0.0 else zero     # v_1
    zeta = beta                              # zeta_0

    # rotations (c_{k-1}, s_{k-1}) and (c_{k-2}, s_{k-2}) seen by step k = 1
    c1, s1, c2, s2 = 1.0, 0.0, 0.0, 0.0
    vt1 = vt2 = bt1 = bt2 = zero             # v~_{k-1}, v~_{k-2}, b~_{k-1}, b~_{k-2}
    Hvt1 = Hvt2 = Hbt1 = Hbt2 = zero         # their images under H (Appendix A)
    hist_res, hist_nsc = [], []

    def met(rv, res, j):
        est = float(np.linalg.norm(mu * (Z.T @ rv))) if (Z is not None and mu is not None and len(mu)) else np.nan
        if record:
            hist_res.append(res)
            hist_nsc.append(est)
        if res == 0.0:
            return True
        if j % check_every:
            return False
        if stop == "hgerr":
            return est <= hg_tol
        return res <= tol * gnorm

    status = OK
    iters = 0
    Vs = []
    done = met(r, abs(zeta), 0)
    while not done and iters < max_iter:
        k = iters + 1
        if len(Vs) < v_cap:
            Vs.append(v)
        # new Lanczos vector, orthogonal to C
        Hv = hvp(v)
        e = C.T @ Hv if s else np.zeros(0)
        b = U @ e if s else zero             # b_k = U C^T H v_k
        CCHv = C @ e if s else zero
        u = Hv - CCHv
        alpha = float(v @ u)
        u = u - alpha * v - beta * v_prev
        beta_next = float(np.linalg.norm(u))
        # previous two rotations applied to the new column (beta_k, alpha_k, beta_{k+1})
        gamma = s2 * beta
        delta = c1 * c2 * beta + s1 * alpha
        eps = -s1 * c2 * beta + c1 * alpha
        # new rotation annihilating beta_{k+1}
        eps_t = float(np.hypot(eps, beta_next))
        if eps_t == 0.0:
            status = BREAKDOWN
            break
        ck, sk = eps / eps_t, beta_next / eps_t
        tau = ck * zeta                      # c_k zeta_{k-1}
        zeta = -sk * zeta                    # zeta_k
        # solution update
        vt = (v - gamma * vt2 - delta * vt1) / eps_t
        bt = (b - gamma * bt2 - delta * bt1) / eps_t
        w = w + tau * (vt - bt)
        # explicit residual (Appendix A): r_k = r_{k-1} - tau H (v~_k - b~_k)
        Hvt = (Hv - delta * Hvt1 - gamma * Hvt2) / eps_t
        Hbt = (CCHv - delta * Hbt1 - gamma * Hbt2) / eps_t
        r = r - tau * (Hvt - Hbt)
        # shift the recurrences
        vt2, vt1, bt2, bt1 = vt1, vt, bt1, bt
        Hvt2, Hvt1, Hbt2, Hbt1 = Hvt1, Hvt, Hbt1, Hbt
        c2, s2, c1, s1 = c1, s1, ck, sk
        v_prev, v = v, (u / beta_next if beta_next > 0.0 else zero)
        beta = beta_next
        iters = k
        done = met(r, abs(zeta), k)
    if not done and status == OK:
        status = NOT_CONVERGED
    return {"w": w, "iters": iters, "status": status, "res_norm": abs(zeta), "g_norm": gnorm, "r": r,
            "hist_res": hist_res, "hist_nsc": hist_nsc,
            "V": np.stack(Vs, axis=1) if Vs else np.zeros((n, 0))}
