"""Recycle-space refresh from Ritz generalized singular vectors (Section 3.2), FP64.

Outer variant (eq. subtle-new): the space for system i is extracted from
W = [U^{(i-1)}, V^{(i-1)}] using the *new* Hessian H^{(i)} and adjoint Jacobian J^{(i)}.

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
G_RANK_TOL = 1e-8     # singular values of G below this times the largest count as zero


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


def build_from_selection(W: np.ndarray, Y: np.ndarray, sel: dict) -> dict:
    """U~ = W X~, C~ = Y X~ (= H U~), thin QR C~ = C R, U = U~ R^{-1}, Z = W V_H~."""
    X = sel["X"] / np.linalg.norm(sel["X"], axis=0, keepdims=True)
    Ut = W @ X
    Ct = Y @ X
    Qc, Rc = np.linalg.qr(Ct)
    sgn = np.sign(np.diag(Rc))
    sgn[sgn == 0] = 1.0
    Qc = Qc * sgn
    Rc = Rc * sgn[:, None]
    U = np.linalg.solve(Rc.T, Ut.T).T          # U~ R^{-1}
    return {"U": U, "C": Qc, "Z": W @ sel["V_H"], "mu": sel["mu"].copy()}


def refresh(hvp, jac_apply, U_prev, V_prev, s: int, rank_tol: float = RANK_TOL, select_rule: str = "rgen-l-r") -> dict:
    """Outer refresh (RGen-L(R) by default; any rule of SELECTIONS).  ``hvp(v)``/``jac_apply(v)``
    use the new (x_hat, theta).  Selections other than RGen leave mu = 0 and Z = 0: the
    error-estimate test is then undefined and solves use the residual test."""
    blocks = [B for B in (U_prev, V_prev) if B is not None and B.shape[1] > 0]
    if not blocks or s <= 0:
        return {"U": None, "C": None, "Z": None, "mu": None, "t": 0, "rank_G": 0}
    W, kept = orthonormalize(np.concatenate(blocks, axis=1), rank_tol)
    t = W.shape[1]
    Y = np.stack([hvp(W[:, c]) for c in range(t)], axis=1)
    M = 0.5 * (W.T @ Y + Y.T @ W)
    rgen = select_rule.startswith("rgen")
    G = np.stack([jac_apply(W[:, c]) for c in range(t)], axis=1) if rgen else None
    YtY = Y.T @ Y if select_rule.startswith("hritz") else None
    sel = select(G, M, YtY, s, select_rule)
    out = build_from_selection(W, Y, sel)
    out.update({"t": t, "rank_G": sel["rank_G"], "W": W, "M": M, "G": G, "Y": Y, "sel": sel,
                "dropped": len(np.concatenate(blocks, axis=1).T) - len(kept)})
    return out


def principal_angles(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Principal angles (radians) between range(A) and range(B)."""
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    # sines from the component of range(B) outside range(A): accurate for small angles
    sines = np.linalg.svd(Qb - Qa @ (Qa.T @ Qb), compute_uv=False)
    return np.sort(np.arcsin(np.clip(sines, 0.0, 1.0)))
