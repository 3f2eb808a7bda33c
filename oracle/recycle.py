"""Recycle-space refresh from Ritz generalized singular vectors (Section 3.2), FP64.

Outer variant (eq. subtle-new): the space for system i is extracted from
W = [U^{(i-1)}, V^{(i-1)}] using the *new* Hessian H^{(i)} and adjoint Jacobian J^{(i)}.
Inner variant (eq. subtle-old): the projected matrix uses the previous Hessian H^{(i-1)}
(what the previous solve's Lanczos relation already holds); only the s chosen vectors are
multiplied by H^{(i)}.  It takes the semi-orthogonal leading part of the stored basis
(:func:`semiorthogonal_prefix`).

Readings taken where the paper is silent:
  * W is orthonormalised before projecting (the paper's W is only "full rank";
    with orthonormal W the Ritz-GSV triplets depend on range(W) alone).
    Columns are processed in the order [U, V] by Gram-Schmidt with a second
    pass; a column whose norm after projection is below ``rank_tol`` times its
    original norm is dropped.
  * GSVD of the pair (G, M) = (J W, W^T H W) by the Paige-Saunders construction
    the paper follows (QR of the stacked pair, then SVDs) in :func:`gsvd_ps`;
    an independent textbook route (SVD of G M^{-1}, eq. gritz-decomp) in
    :func:`gsvd_via_quotient` serves as a check.
  * RGen-L(R): right vectors W X of the s largest mu (Table 1).  If G has rank
    r_G < s (the TV problems have p = 2 < t) only r_G values are non-zero; the
    remaining s - r_G slots take Ritz vectors of H on range(W N), N an orthonormal
    basis of null(G), for the smallest Ritz values (Ritz-S), with mu = 0.
  * ``C~ = H U~`` is formed as Y X~ from the already computed Y = H W; thin QR
    C~ = C R (diag R > 0), U = U~ R^{-1} (Section 2.2.2).
  * Z = W V_H (selected columns; zero for filled slots) and mu feed the
    hypergradient-error estimate ||mu . (Z^T r)|| of eq. hg-err-stop-lowrank.
  * Other selections of Table 2 on the same projected matrices (:func:`select`): Ritz and
    harmonic Ritz vectors of sizes S, L, M, and the L, R, M sides of RGen-L.  Readings: size M
    keeps ceil(s/2) smallest and floor(s/2) largest values; the left vector of each right vector
    x is v = M x / ||M x|| (the GSVD's M x = beta v fixes its sign), and side M is x/||x|| + v.
"""
from __future__ import annotations

import numpy as np

RANK_TOL = 1e-8       # relative column-norm drop threshold of the orthonormalisation
G_RANK_TOL = 1e-6     # singular values of G below this times the largest count as zero


def orthonormalize(W: np.ndarray, rank_tol: float = RANK_TOL):
    """Gram-Schmidt with re-orthogonalisation, in column order; returns (Q, kept column indices)."""
    n, t = W.shape
    Q = np.zeros((n, 0))
    kept = []
    for c in range(t):
        v = W[:, c].astype(np.float64).copy()
        nrm0 = float(np.linalg.norm(v))
        if nrm0 == 0.0:
            continue
        for _ in range(2):
            v -= Q @ (Q.T @ v)
        nrm = float(np.linalg.norm(v))
        if nrm <= rank_tol * nrm0:
            continue
        Q = np.concatenate([Q, (v / nrm)[:, None]], axis=1)
        kept.append(c)
    return Q, kept


def gsvd_ps(G: np.ndarray, M: np.ndarray) -> dict:
    """GSVD of (G, M), M invertible, via QR of [G; M] and an SVD of the lower block.

    [G; M] = [Q1; Q2] R;  Q2 = V_H diag(beta) Y^T;  X = R^{-1} Y;
    then M X = V_H diag(beta) and G X = Q1 Y has orthogonal columns of norms
    alpha (= sqrt(1 - beta^2)), so mu = alpha / beta.  Returned in ascending mu
    (the ordering of the GSVD theorem).
    """
    p, t = G.shape
    Q, R = np.linalg.qr(np.vstack([G, M]))
    Q1, Q2 = Q[:p], Q[p:]
    VH, beta, Yt = np.linalg.svd(Q2)
    Y = Yt.T
    GX = Q1 @ Y
    # alpha from the column norms of Q1 Y: accurate also where beta is close to 1
    alpha = np.linalg.norm(GX, axis=0)
    mu = alpha / beta
    X = np.linalg.solve(R, Y)
    VJ = np.where(alpha > 1e-14, GX / np.where(alpha > 1e-14, alpha, 1.0), 0.0)
    return {"alpha": alpha, "beta": beta, "mu": mu, "X": X, "V_H": VH, "V_J": VJ}


def gsvd_via_quotient(G: np.ndarray, M: np.ndarray) -> dict:
    """Check route: G M^{-1} = V_J diag(mu) V_H^T (eq. gritz-decomp); X is proportional to M^{-1} V_H."""
    S = np.linalg.solve(M.T, G.T).T
    _, sig, Vt = np.linalg.svd(S, full_matrices=True)
    t = M.shape[0]
    mu = np.zeros(t)
    mu[:sig.size] = sig
    VH = Vt.T
    X = np.linalg.solve(M, VH)
    order = np.argsort(mu, kind="stable")
    return {"mu": mu[order], "V_H": VH[:, order], "X": X[:, order]}


def g_rank(G: np.ndarray, tol: float = G_RANK_TOL) -> int:
    sig = np.linalg.svd(G, compute_uv=False)
    if sig.size == 0 or sig[0] == 0.0:
        return 0
    return int(np.sum(sig > tol * sig[0]))


def select_rgen_large(G: np.ndarray, M: np.ndarray, s: int) -> dict:
    """RGen-L(R) selection with the null-space fill rule; returns X~ (t x s'), V_H~, mu~."""
    t = M.shape[0]
    s_eff = min(s, t)
    gs = gsvd_ps(G, M)
    rG = g_rank(G)
    k = min(s_eff, rG)
    idx = np.argsort(-gs["mu"], kind="stable")[:k]
    X = gs["X"][:, idx]
    VH = gs["V_H"][:, idx]
    mu = gs["mu"][idx]
    nfill = s_eff - k
    if nfill > 0:
        _, _, Vt = np.linalg.svd(G, full_matrices=True)
        N = Vt[rG:].T                           # orthonormal basis of null(G)
        lam, Qn = np.linalg.eigh(N.T @ M @ N)   # Ritz values ascending
        Xf = N @ Qn[:, :nfill]
        X = np.concatenate([X, Xf], axis=1)
        VH = np.concatenate([VH, np.zeros((t, nfill))], axis=1)
        mu = np.concatenate([mu, np.zeros(nfill)])
    return {"X": X, "V_H": VH, "mu": mu, "rank_G": rG}


# Selections of Table 2 built here: vector type and size (S: the s smallest values, L: the s
# largest, M: ceil(s/2) smallest and floor(s/2) largest), and for RGen-L the side (R: right
# vectors W X, L: left vectors W V_H, M: their normalised sum).
SELECTIONS = ("rgen-l-r", "rgen-l-l", "rgen-l-m", "ritz-s", "ritz-l", "ritz-m", "hritz-s", "hritz-l", "hritz-m")
# RGen of sizes S and M: only where J W has full column rank (p >= t), so that every generalized
# singular value is positive and "the smallest" is defined without ties among zeros.
SELECTIONS_FULL_RANK = ("rgen-s-r", "rgen-s-l", "rgen-s-m", "rgen-m-r", "rgen-m-l", "rgen-m-m")


def size_pick(t: int, s: int, size: str) -> list:
    """Positions, in a list of t values sorted ascending, of the s values a size rule keeps:
    smallest first for S, largest first for L, and for M the smallest ceil(s/2) (ascending)
    followed by the largest floor(s/2) (descending)."""
    s = min(s, t)
    if size == "s":
        return list(range(s))
    if size == "l":
        return list(range(t - 1, t - 1 - s, -1))
    lo = (s + 1) // 2
    return list(range(lo)) + list(range(t - 1, t - 1 - (s - lo), -1))


def select_ritz(M: np.ndarray, s: int, size: str) -> dict:
    """Ritz vectors (eq. ritz-matrix-decomp): eigenvectors of W^T H W (W orthonormal), chosen by
    their Ritz values."""
    lam, Q = np.linalg.eigh(M)
    idx = size_pick(M.shape[0], s, size)
    k = len(idx)
    return {"X": Q[:, idx], "V_H": np.zeros((M.shape[0], k)), "mu": np.zeros(k), "rank_G": 0,
            "values": lam[idx]}


def select_hritz(M: np.ndarray, YtY: np.ndarray, s: int, size: str) -> dict:
    """Harmonic Ritz vectors (eq. harmonic-ritz): (HW)^T HW rho = theta (HW)^T W rho, with
    (HW)^T W = W^T H W = M.  Solved as the symmetric-definite problem M rho = nu (Y^T Y) rho
    (Y = H W of full column rank), theta = 1 / nu, and chosen by theta."""
    import scipy.linalg
    nu, R = scipy.linalg.eigh(M, YtY)
    theta = 1.0 / nu
    order = np.argsort(theta, kind="stable")
    idx = [order[j] for j in size_pick(M.shape[0], s, size)]
    k = len(idx)
    return {"X": R[:, idx], "V_H": np.zeros((M.shape[0], k)), "mu": np.zeros(k), "rank_G": 0,
            "values": theta[idx]}


def rgen_side(M: np.ndarray, sel: dict, side: str) -> dict:
    """Side of the RGen-L vectors.  The GSVD ties each left vector to its right one,
    M x_i = beta_i v_i with beta_i > 0, so v = M x / ||M x|| fixes its sign; this holds for the
    filled slots (mu = 0, beta = 1) too.  Side L takes v, side M the normalised x + v; Z and mu
    stay those of the GSVD."""
    if side == "r":
        return sel
    X = sel["X"] / np.linalg.norm(sel["X"], axis=0, keepdims=True)
    Vl = M @ X
    Vl = Vl / np.linalg.norm(Vl, axis=0, keepdims=True)
    out = dict(sel)
    out["X"] = Vl if side == "l" else X + Vl
    return out


def select_rgen_size(G: np.ndarray, M: np.ndarray, s: int, size: str) -> dict:
    """RGen of size S or M (Table 2): the smallest, or ceil(s/2) smallest and floor(s/2) largest,
    generalized singular values of (G, M); needs rank G = t."""
    t = M.shape[0]
    rG = g_rank(G)
    if rG < t:
        raise ValueError("RGen sizes S and M need J W of full column rank")
    gs = gsvd_ps(G, M)   # ascending mu
    idx = size_pick(t, s, size)
    return {"X": gs["X"][:, idx], "V_H": gs["V_H"][:, idx], "mu": gs["mu"][idx], "rank_G": rG}


def select(G, M, YtY, s: int, rule: str) -> dict:
    """Dispatch a selection rule of SELECTIONS or SELECTIONS_FULL_RANK."""
    kind, size, *rest = rule.split("-")
    if kind == "rgen":
        sel = select_rgen_large(G, M, s) if size == "l" else select_rgen_size(G, M, s, size)
        return rgen_side(M, sel, rest[0])
    if kind == "ritz":
        return select_ritz(M, s, size)
    if kind == "hritz":
        return select_hritz(M, YtY, s, size)
    raise ValueError(f"unknown selection {rule}")


def build_from_selection(W: np.ndarray, Y: np.ndarray, sel: dict, Ut=None) -> dict:
    """U~ = W X~, C~ = Y X~ (= H U~), thin QR C~ = C R, U = U~ R^{-1}, Z = W V_H~.  With Ut
    given, U~ = Ut and Y already holds H U~ (X~ = I)."""
    X = sel["X"] / np.linalg.norm(sel["X"], axis=0, keepdims=True)
    Ut = W @ X if Ut is None else Ut
    Ct = Y @ X
    Qc, Rc = np.linalg.qr(Ct)
    sgn = np.sign(np.diag(Rc))
    sgn[sgn == 0] = 1.0
    Qc = Qc * sgn
    Rc = Rc * sgn[:, None]
    U = np.linalg.solve(Rc.T, Ut.T).T          # U~ R^{-1}
    return {"U": U, "C": Qc, "Z": W @ sel["V_H"], "mu": sel["mu"].copy()}


def refresh(hvp, jac_apply, U_prev, V_prev, s: int, rank_tol: float = RANK_TOL, select_rule: str = "rgen-l-r",
            hvp_old=None) -> dict:
    """Recycle-space refresh (RGen-L(R) by default; any rule of SELECTIONS).  ``hvp(v)`` and
    ``jac_apply(v)`` use the new (x_hat, theta).

    Outer variant (``hvp_old`` None, eq. subtle-new): the projected matrix is W^T H^{(i)} W.
    Inner variant (``hvp_old`` the previous system's product, eq. subtle-old): it is
    W^T H^{(i-1)} W, and only the s selected vectors meet the new Hessian (C~ = H^{(i)} U~).
    The paper changes only the Hessian between the two (Section 3.1; Section 5.1, "Inner versus
    outer recycling strategies"); reading: J stays the new J^{(i)} in both.

    Selections other than RGen leave mu = 0 and Z = 0: the error-estimate test is then undefined
    and solves use the residual test."""
    v_used = 0 if V_prev is None else V_prev.shape[1]
    if hvp_old is not None and V_prev is not None:
        v_used = semiorthogonal_prefix(V_prev)
        V_prev = V_prev[:, :v_used]
    blocks = [B for B in (U_prev, V_prev) if B is not None and B.shape[1] > 0]
    if not blocks or s <= 0:
        return {"U": None, "C": None, "Z": None, "mu": None, "t": 0, "rank_G": 0, "v_used": v_used}
    W, kept = orthonormalize(np.concatenate(blocks, axis=1), rank_tol)
    t = W.shape[1]
    proj = hvp if hvp_old is None else hvp_old
    Y = np.stack([proj(W[:, c]) for c in range(t)], axis=1)
    M = 0.5 * (W.T @ Y + Y.T @ W)
    rgen = select_rule.startswith("rgen")
    G = np.stack([jac_apply(W[:, c]) for c in range(t)], axis=1) if rgen else None
    YtY = Y.T @ Y if select_rule.startswith("hritz") else None
    sel = select(G, M, YtY, s, select_rule)
    if hvp_old is None:
        out = build_from_selection(W, Y, sel)
    else:
        # C~ = H^{(i)} U~ by s products with the new Hessian
        X = sel["X"] / np.linalg.norm(sel["X"], axis=0, keepdims=True)
        Ynew = np.stack([hvp(W @ X[:, c]) for c in range(X.shape[1])], axis=1)
        out = build_from_selection(W, Ynew, dict(sel, X=np.eye(X.shape[1])), Ut=W @ X)
    out.update({"t": t, "rank_G": sel["rank_G"], "W": W, "M": M, "G": G, "Y": Y, "sel": sel,
                "dropped": len(np.concatenate(blocks, axis=1).T) - len(kept), "v_used": v_used})
    return out


SEMIORTH_TOL = 2.0 ** -26    # sqrt of the FP64 unit roundoff


def semiorthogonal_prefix(V: np.ndarray, tol: float = SEMIORTH_TOL) -> int:
    """Number of leading columns of a stored Krylov basis that are semi-orthogonal: every pair
    |v_i . v_j| and every |v_j . v_j - 1| within sqrt(eps).  Reading for the inner refresh: the
    previous solve's relation V^T H V = T (eq. arnoldi_aug_matrix in CG form) holds to working
    precision only while the computed basis keeps this property (Simon's semi-orthogonality
    condition for the Lanczos process); the residuals after the first column that breaks it are
    not used.  Applied by the oracle's inner refresh so that both sides project the same basis."""
    Gm = V.T @ V
    k = V.shape[1]
    for j in range(k):
        if abs(Gm[j, j] - 1.0) > tol or (j > 0 and np.abs(Gm[:j, j]).max() > tol):
            return j
    return k


def cg_lanczos_matrix(alpha: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """V^T A V for the normalised CG residuals v_j = r_j / sqrt(rho_j), j < k, from the CG
    coefficients alone (the Lanczos relation eq. arnoldi-matrix-id written for CG; with the
    recycle space it is eq. arnoldi_aug_matrix, A = (I - C C^T) H on range(C)^perp, and
    V^T H V = V^T A V there since V is orthogonal to C).

    From A p_j = (r_j - r_{j+1}) / alpha_j and p_j = r_j + beta_{j-1} p_{j-1}
    (beta_{j-1} = rho_j / rho_{j-1}):
        A r_j = (1/alpha_j + beta_{j-1}/alpha_{j-1}) r_j - r_{j+1}/alpha_j - (beta_{j-1}/alpha_{j-1}) r_{j-1},
    and the residuals are orthogonal, so T is tridiagonal with
        T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}   (no second term for j = 0),
        T_{j,j+1} = T_{j+1,j} = -sqrt(rho_{j+1}/rho_j) / alpha_j.
    In floating point it equals V^T H V while the stored residuals stay orthogonal."""
    k = len(rho)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alpha[j] + ((rho[j] / rho[j - 1]) / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = -np.sqrt(rho[j + 1] / rho[j]) / alpha[j]
    return T


def principal_angles(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Principal angles (radians) between range(A) and range(B)."""
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    # sines from the component of range(B) outside range(A): accurate for small angles
    sines = np.linalg.svd(Qb - Qa @ (Qa.T @ Qb), compute_uv=False)
    return np.sort(np.arcsin(np.clip(sines, 0.0, 1.0)))
