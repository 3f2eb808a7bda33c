"""Pins of the oracle's projected GSVD, Ritz-GSV selection, refresh and error estimate."""
import numpy as np
import pytest

import synth
from oracle import krylov, problem, recycle


def spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


@pytest.mark.parametrize("p,t", [(30, 12), (12, 12), (3, 10)])
def test_gsvd_identities(p, t):
    """GSVD theorem: alpha^2 + beta^2 = 1, G X = V_J diag(alpha), M X = V_H diag(beta), mu ascending."""
    rng = np.random.default_rng(p * 100 + t)
    G = rng.standard_normal((p, t))
    M = spd(t, 50.0, t)
    gs = recycle.gsvd_ps(G, M)
    a, b, X = gs["alpha"], gs["beta"], gs["X"]
    assert np.abs(a * a + b * b - 1.0).max() < 1e-14 * 10
    assert np.all(np.diff(gs["mu"]) >= -1e-14)
    assert np.abs(M @ X - gs["V_H"] * b).max() < 1e-12 * np.abs(M).max() * np.abs(X).max()
    nz = a > 1e-14
    assert np.abs(G @ X[:, nz] - gs["V_J"][:, nz] * a[nz]).max() < 1e-12 * np.abs(G).max() * np.abs(X).max()
    assert np.abs(gs["V_H"].T @ gs["V_H"] - np.eye(t)).max() < 1e-13
    VJ = gs["V_J"][:, nz]
    assert np.abs(VJ.T @ VJ - np.eye(VJ.shape[1])).max() < 1e-10   # columns divided by small alpha
    if p < t:
        assert int(np.sum(gs["mu"] > 1e-10)) == p


@pytest.mark.parametrize("p,t", [(40, 15), (15, 15), (2, 12)])
def test_gsvd_two_routes_agree(p, t):
    rng = np.random.default_rng(7 + p + t)
    G = rng.standard_normal((p, t))
    M = spd(t, 30.0, p + t)
    a = recycle.gsvd_ps(G, M)
    b = recycle.gsvd_via_quotient(G, M)
    k = min(p, t)
    ma, mb = a["mu"][-k:], b["mu"][-k:]
    assert np.abs(ma - mb).max() <= 1e-10 * ma.max()
    for j in range(1, k + 1):   # right vectors agree up to scale/sign
        xa, xb = a["X"][:, -j], b["X"][:, -j]
        ang = recycle.principal_angles(xa[:, None], xb[:, None]).max()
        assert ang < 1e-8


def test_gsvd_special_case_identity_J():
    """G = I: generalized singular values are the reciprocals of the eigenvalues of M."""
    t = 9
    M = spd(t, 20.0, 3)
    gs = recycle.gsvd_ps(np.eye(t), M)
    lam = np.linalg.eigvalsh(M)
    assert np.abs(np.sort(gs["mu"]) - np.sort(1.0 / lam)).max() < 1e-12


def test_gsvd_special_case_full_space_is_svd_of_J_Hinv():
    """W = I (full space): mu are the singular values of J H^{-1}."""
    n, p = 14, 20
    H = spd(n, 40.0, 4)
    J = np.random.default_rng(5).standard_normal((p, n))
    gs = recycle.gsvd_ps(J, H)
    sv = np.linalg.svd(J @ np.linalg.inv(H), compute_uv=False)
    assert np.abs(np.sort(gs["mu"])[::-1] - sv).max() < 1e-11 * sv.max()


@pytest.mark.parametrize("p", [20, 3])
def test_error_estimate_exact_on_full_space(p):
    """Full GSVD with square W: ||mu . (V_H^T r)|| equals ||J H^{-1} r|| for any r (Section 4)."""
    n = 16
    H = spd(n, 25.0, 6)
    J = np.random.default_rng(7).standard_normal((p, n))
    gs = recycle.gsvd_ps(J, H)
    rng = np.random.default_rng(8)
    for _ in range(3):
        r = rng.standard_normal(n)
        est = np.linalg.norm(gs["mu"] * (gs["V_H"].T @ r))
        true = np.linalg.norm(J @ np.linalg.solve(H, r))
        assert abs(est - true) <= 1e-12 * true


def test_orthonormalize_drops_dependent_columns():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((50, 6))
    W = np.concatenate([A, A[:, :2] @ np.array([[1.0], [2.0]]), rng.standard_normal((50, 2))], axis=1)
    Q, kept = recycle.orthonormalize(W)
    assert kept == [0, 1, 2, 3, 4, 5, 7, 8]
    assert np.abs(Q.T @ Q - np.eye(8)).max() < 1e-14
    assert recycle.principal_angles(Q, W[:, kept]).max() < 1e-12


def test_selection_fill_rule_for_low_rank_G():
    t, s = 12, 5
    M = spd(t, 40.0, 10)
    G = np.random.default_rng(11).standard_normal((2, t))
    sel = recycle.select_rgen_large(G, M, s)
    assert sel["rank_G"] == 2
    assert np.all(sel["mu"][:2] > 0) and np.all(sel["mu"][2:] == 0)
    # filled right vectors lie in null(G) and are the Ritz-S vectors of M restricted to null(G)
    Xf = sel["X"][:, 2:]
    assert np.abs(G @ Xf).max() < 1e-12
    _, _, Vt = np.linalg.svd(G)
    N = Vt[2:].T
    lam, Q = np.linalg.eigh(N.T @ M @ N)
    assert recycle.principal_angles(Xf, N @ Q[:, :3]).max() < 1e-10


def tv_setup(side=12, seed=21):
    wl = synth.custom("t", side, "tv", 6, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=4, seed=seed)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xh = inst["xstar"].ravel() + 0.05 * synth.unit_noise(prob.n, seed + 1)
    return wl, inst, prob, xh


def test_refresh_invariants_and_basis_independence():
    wl, inst, prob, xh = tv_setup()
    th = inst["theta0"]
    hvp = lambda v: prob.hvp(xh, th, v)
    jac = lambda v: prob.jac_apply(xh, th, v)
    g = xh - inst["xstar"].ravel()
    res = krylov.cg(hvp, g, tol=1e-10, v_cap=20)
    rs = recycle.refresh(hvp, jac, None, res["V"], s=6)
    U, C = rs["U"], rs["C"]
    HU = np.stack([hvp(U[:, j]) for j in range(U.shape[1])], axis=1)
    assert np.linalg.norm(HU - C) <= 1e-12 * np.linalg.norm(C)
    assert np.abs(C.T @ C - np.eye(C.shape[1])).max() <= 1e-14
    # re-basing W (a rotation of the stored vectors) leaves range(U) unchanged
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((res["V"].shape[1],) * 2))
    rs2 = recycle.refresh(hvp, jac, None, res["V"] @ Q, s=6)
    assert recycle.principal_angles(rs["U"], rs2["U"]).max() < 1e-8
    assert np.abs(rs["mu"] - rs2["mu"]).max() <= 1e-10 * rs["mu"].max()


def test_recycled_sequence_reaches_same_solution_as_plain():
    wl, inst, prob, xh = tv_setup(10, 31)
    xs = inst["xstar"].ravel()
    thetas = [inst["theta0"] + 0.01 * k for k in range(4)]
    xhats = [xh + 0.001 * k * synth.unit_noise(prob.n, 40 + k) for k in range(4)]
    plain = __import__("oracle.upper", fromlist=["x"]).solve_sequence(prob, thetas, xhats, xs, s=5,
                                                                       recycle_on=False, tol=1e-12)
    rec = __import__("oracle.upper", fromlist=["x"]).solve_sequence(prob, thetas, xhats, xs, s=5, tol=1e-12)
    for a, b, th, x in zip(plain, rec, thetas, xhats):
        Hd = prob.dense_hessian(x, th)
        w = np.linalg.solve(Hd, x - xs)
        kappa = np.linalg.cond(Hd)
        for r in (a, b):
            assert np.linalg.norm(r["w"] - w) <= kappa * 1e-12 * 10 * np.linalg.norm(w)


@pytest.mark.parametrize("p,t,s", [(30, 12, 5), (12, 12, 12), (400, 20, 7)])
def test_rgen_large_picks_largest_quotient_singular_values(p, t, s):
    """p >= t (filter regulariser): RGen-L keeps the s largest generalized singular values of (G, M),
    i.e. the s largest singular values of G M^{-1} (eq. gritz-decomp); its right vectors X span
    M^{-1} V_top and its left vectors V_H span V_top, V_top the matching right singular vectors."""
    rng = np.random.default_rng(p + 3 * t + s)
    G = rng.standard_normal((p, t))
    M = spd(t, 60.0, p + t)
    sel = recycle.select_rgen_large(G, M, s)
    S = G @ np.linalg.inv(M)
    _, sig, Vt = np.linalg.svd(S)
    assert sel["rank_G"] == t
    assert np.all(np.diff(sel["mu"]) <= 0.0)
    assert np.abs(sel["mu"] - sig[:s]).max() <= 1e-10 * sig[0]
    Vtop = Vt[:s].T
    assert recycle.principal_angles(sel["V_H"], Vtop).max() < 1e-8
    assert recycle.principal_angles(sel["X"], np.linalg.solve(M, Vtop)).max() < 1e-8


# ------------------------------------------------------------------ inner refresh (eq. subtle-old)
def _tv_pair(seed=131):
    """A 20 x 18 TV problem at two nearby (x_hat, theta): the systems i-1 and i of a sequence."""
    wl = synth.custom("t", 20, "tv", 4, width=18, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=5, seed=seed)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xs = inst["xstar"].ravel()
    x0 = xs + 0.05 * synth.unit_noise(prob.n, seed + 1)
    x1 = x0 + 0.01 * synth.unit_noise(prob.n, seed + 2)
    t0 = np.array(inst["theta0"])
    t1 = t0 + np.array([0.05, -0.03])
    return prob, xs, (x0, t0), (x1, t1)


def test_cg_lanczos_matrix_is_projected_hessian():
    """The CG form of the Lanczos relation: V^T H V of the stored normalised residuals equals
    the tridiagonal matrix built from the CG coefficients alone, with and without a recycle
    space (then V is also orthogonal to C, so U^T H V = C^T V = 0)."""
    prob, xs, (x0, t0), _ = _tv_pair()
    hvp = lambda v: prob.hvp(x0, t0, v)
    g = x0 - xs
    first = krylov.cg(hvp, g, tol=1e-12, v_cap=14)
    V = first["V"]
    assert V.shape[1] == 14 and len(first["alpha"]) == 14 and len(first["rho"]) == 14
    HV = np.stack([hvp(V[:, j]) for j in range(14)], axis=1)
    T = recycle.cg_lanczos_matrix(first["alpha"], first["rho"])
    assert np.abs(T - V.T @ HV).max() <= 1e-9 * np.abs(T).max()    # rounding: the residuals lose orthogonality
    assert np.count_nonzero(np.triu(T, 2)) == 0
    # recycled: CG on (I - C C^T) H with C = H U from an outer refresh of the first basis
    rs = recycle.refresh(hvp, lambda v: prob.jac_apply(x0, t0, v), None, V, s=4)
    second = krylov.recycled_cg(hvp, g + 0.1 * synth.unit_noise(prob.n, 7), None, rs["U"], rs["C"], tol=1e-12,
                                v_cap=10)
    V2 = second["V"]
    HV2 = np.stack([hvp(V2[:, j]) for j in range(V2.shape[1])], axis=1)
    T2 = recycle.cg_lanczos_matrix(second["alpha"], second["rho"])
    assert np.abs(T2 - V2.T @ HV2).max() <= 1e-9 * np.abs(T2).max()
    UtHV = rs["U"].T @ HV2
    assert np.abs(UtHV).max() <= 1e-10 * np.abs(T2).max()
    assert np.abs(rs["C"].T @ V2).max() <= 1e-12


def test_inner_refresh_from_lanczos_relation():
    """Inner refresh (eq. subtle-old): its projected matrix W^T H^{(i-1)} W, formed by the
    oracle from products with the previous Hessian, equals X^T blockdiag(U^T C, T) X assembled
    from the previous solve's relation (U^T H^{(i-1)} U = U^T C, U^T H^{(i-1)} V = 0, V^T H^{(i-1)} V
    = T from the CG coefficients), W = [U, V] X; only the s selected vectors meet H^{(i)}."""
    prob, xs, (x0, t0), (x1, t1) = _tv_pair(141)
    h0 = lambda v: prob.hvp(x0, t0, v)
    h1 = lambda v: prob.hvp(x1, t1, v)
    jac1 = lambda v: prob.jac_apply(x1, t1, v)
    first = krylov.cg(h0, x0 - xs, tol=1e-12, v_cap=12)
    rs0 = recycle.refresh(h0, lambda v: prob.jac_apply(x0, t0, v), None, first["V"], s=4)
    prev = krylov.recycled_cg(h0, x0 - xs, first["w"], rs0["U"], rs0["C"], tol=1e-13, v_cap=10)
    U, C, V = rs0["U"], rs0["C"], prev["V"]
    assert V.shape[1] == 10
    calls = {"old": 0, "new": 0}

    def count(h, key):
        def f(v):
            calls[key] += 1
            return h(v)
        return f

    ref = recycle.refresh(count(h1, "new"), jac1, U, V, s=4, hvp_old=count(h0, "old"))
    assert calls == {"old": ref["t"], "new": 4}
    W = ref["W"]
    X = np.linalg.lstsq(np.concatenate([U, V], axis=1), W, rcond=None)[0]
    M0 = np.zeros((14, 14))
    M0[:4, :4] = 0.5 * (U.T @ C + C.T @ U)
    M0[4:, 4:] = recycle.cg_lanczos_matrix(prev["alpha"], prev["rho"])
    M_rel = X.T @ M0 @ X
    assert np.abs(M_rel - ref["M"]).max() <= 1e-9 * np.abs(ref["M"]).max()
    # the recycle space it returns satisfies the invariants of the new system
    HU = np.stack([h1(ref["U"][:, j]) for j in range(ref["U"].shape[1])], axis=1)
    assert np.linalg.norm(HU - ref["C"]) <= 1e-12 * np.linalg.norm(ref["C"])
    assert np.abs(ref["C"].T @ ref["C"] - np.eye(ref["C"].shape[1])).max() <= 1e-13
    # and differs from the outer variant's, which projects with the new Hessian
    out = recycle.refresh(h1, jac1, U, V, s=4)
    assert np.abs(out["M"] - ref["M"]).max() > 1e-6 * np.abs(ref["M"]).max()


def test_inner_equals_outer_for_an_unchanged_hessian():
    """With H^{(i)} = H^{(i-1)} the two variants are one definition: same mu, same spaces."""
    prob, xs, (x0, t0), _ = _tv_pair(151)
    h0 = lambda v: prob.hvp(x0, t0, v)
    jac = lambda v: prob.jac_apply(x0, t0, v)
    first = krylov.cg(h0, x0 - xs, tol=1e-10, v_cap=16)
    a = recycle.refresh(h0, jac, None, first["V"], s=5)
    b = recycle.refresh(h0, jac, None, first["V"], s=5, hvp_old=h0)
    assert np.abs(a["M"] - b["M"]).max() == 0.0
    assert np.abs(a["mu"] - b["mu"]).max() <= 1e-12 * a["mu"].max()
    assert recycle.principal_angles(a["U"], b["U"]).max() <= 1e-9
    assert recycle.principal_angles(a["C"], b["C"]).max() <= 1e-9
    assert recycle.principal_angles(a["Z"][:, :2], b["Z"][:, :2]).max() <= 1e-9


def test_semiorthogonal_prefix():
    """Leading columns with pairwise products and norms within sqrt(eps) of orthonormal; a
    column breaking it ends the prefix, whatever follows."""
    rng = np.random.default_rng(5)
    Q = np.linalg.qr(rng.standard_normal((60, 12)))[0]
    assert recycle.semiorthogonal_prefix(Q) == 12
    Qb = Q.copy()
    Qb[:, 7] += 1e-6 * Qb[:, 2]
    Qb[:, 7] /= np.linalg.norm(Qb[:, 7])
    assert recycle.semiorthogonal_prefix(Qb) == 7
    Qn = Q.copy()
    Qn[:, 4] *= 1.0 + 1e-7
    assert recycle.semiorthogonal_prefix(Qn) == 4
    # CG residuals of a long solve lose orthogonality: the prefix stops before the end
    prob, xs, (x0, t0), _ = _tv_pair(161)
    res = krylov.cg(lambda v: prob.hvp(x0, t0, v), x0 - xs, tol=1e-14, v_cap=200)
    k = recycle.semiorthogonal_prefix(res["V"])
    assert 10 < k < res["V"].shape[1]
    Vk = res["V"][:, :k]
    assert np.abs(Vk.T @ Vk - np.eye(k)).max() <= recycle.SEMIORTH_TOL
