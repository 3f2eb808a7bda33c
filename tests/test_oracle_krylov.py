"""Pins of the oracle's plain and recycled CG.

* dense direct solve; finite termination on small SPD systems;
* recycled CG equals, iterate by iterate, the Galerkin solution over the augmented
  space w0 + span(U) + K_k(P H P, P r0) computed by brute force with dense algebra;
* invariants: C^T r = 0, recursive residual = true residual;
* one-step exactness when range(U) contains w* - w0;
* the single-reduction recurrence option gives the same solve.
"""
import numpy as np
import pytest

from oracle import krylov


def spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T


def recycle_pair(H, s, seed):
    rng = np.random.default_rng(seed)
    Ut = rng.standard_normal((H.shape[0], s))
    Qc, Rc = np.linalg.qr(H @ Ut)
    return Ut @ np.linalg.inv(Rc), Qc


def test_cg_matches_direct_solve():
    H = spd(60, 1e3, 0)
    g = np.random.default_rng(1).standard_normal(60)
    res = krylov.cg(lambda v: H @ v, g, tol=1e-13)
    w = np.linalg.solve(H, g)
    assert res["status"] == krylov.OK
    assert np.linalg.norm(res["w"] - w) / np.linalg.norm(w) < 1e3 * 1e-13 * 10


def test_cg_finite_termination():
    H = spd(12, 10.0, 2)
    g = np.random.default_rng(3).standard_normal(12)
    res = krylov.cg(lambda v: H @ v, g, tol=1e-14, max_iter=12)
    assert res["iters"] <= 12
    assert np.linalg.norm(H @ res["w"] - g) <= 1e-12 * np.linalg.norm(g)


def galerkin_iterate(H, g, w0, U, C, k):
    """Brute force: w = w0 + U c0 + xi - U C^T H xi, xi = K_k-Galerkin solution of P H P xi = P r0."""
    n = H.shape[0]
    P = np.eye(n) - C @ C.T
    r0 = g - H @ w0
    c0 = C.T @ r0
    b = P @ r0
    Op = P @ H @ P
    cols = [b]
    for _ in range(k - 1):
        cols.append(Op @ cols[-1])
    Kb, _ = np.linalg.qr(np.stack(cols, axis=1))
    y = np.linalg.solve(Kb.T @ Op @ Kb, Kb.T @ b)
    xi = Kb @ y
    return w0 + U @ c0 + xi - U @ (C.T @ (H @ xi))


@pytest.mark.parametrize("s", [0, 3, 6])
def test_recycled_cg_is_augmented_galerkin(s):
    n = 40
    H = spd(n, 50.0, 4)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(n)
    w0 = rng.standard_normal(n) * 0.1
    U, C = recycle_pair(H, s, 6) if s else (np.zeros((n, 0)), np.zeros((n, 0)))
    for k in (1, 3, 7):
        res = krylov.recycled_cg(lambda v: H @ v, g, w0, U if s else None, C if s else None, tol=0.0, max_iter=k)
        ref = galerkin_iterate(H, g, w0, U, C, k)
        assert res["iters"] == k
        assert np.linalg.norm(res["w"] - ref) <= 1e-10 * np.linalg.norm(ref)


def test_recycled_cg_invariants_and_solution():
    n, s = 80, 5
    H = spd(n, 200.0, 7)
    g = np.random.default_rng(8).standard_normal(n)
    U, C = recycle_pair(H, s, 9)
    res = krylov.recycled_cg(lambda v: H @ v, g, None, U, C, tol=1e-12)
    assert res["status"] == krylov.OK
    w = np.linalg.solve(H, g)
    assert np.linalg.norm(res["w"] - w) <= 200 * 1e-12 * 10 * np.linalg.norm(w)
    # recursive residual (of the finished iterate) against the true one; orthogonality to C
    true_r = g - H @ res["w"]
    assert np.linalg.norm(true_r - res["r"]) <= 1e-12 * np.linalg.norm(g)
    assert np.linalg.norm(C.T @ res["r"]) <= 1e-13 * np.linalg.norm(g)
    # stored basis: orthonormal and orthogonal to C in exact arithmetic; in floating point
    # the leading vectors keep that to rounding (orthogonality decays as Ritz values converge)
    V = res["V"][:, :8]
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-8
    assert np.abs(C.T @ res["V"]).max() < 1e-10


def test_one_step_exactness():
    n = 50
    H = spd(n, 100.0, 10)
    g = np.random.default_rng(11).standard_normal(n)
    w0 = np.random.default_rng(12).standard_normal(n)
    wstar = np.linalg.solve(H, g)
    Ut = (wstar - w0)[:, None]
    c = H @ Ut
    nrm = np.linalg.norm(c)
    U, C = Ut / nrm, c / nrm
    res = krylov.recycled_cg(lambda v: H @ v, g, w0, U, C, tol=1e-10)
    assert res["iters"] == 0
    assert np.linalg.norm(res["w"] - wstar) <= 1e-12 * np.linalg.norm(wstar)


def test_single_reduction_recurrence():
    """Single-reduction form (the GPU's fused FP64 step): beta from the recurrence
    rho - 2 alpha r.q + alpha^2 (q.q - e.e) anchored on the explicit r.r of the previous iterate,
    alpha and every stop test from the explicit r.r.  It reaches the same true residual as the
    textbook form within a few iterations (rounding changes CG's path over ~180 iterations),
    and agrees with it to rounding at small counts; the recurrence really enters (the iterates
    differ in the last bits)."""
    n, s = 70, 4
    H = spd(n, 300.0, 13)
    g = np.random.default_rng(14).standard_normal(n)
    U, C = recycle_pair(H, s, 15)
    a = krylov.recycled_cg(lambda v: H @ v, g, None, U, C, tol=1e-11)
    b = krylov.recycled_cg(lambda v: H @ v, g, None, U, C, tol=1e-11, recurrence="single")
    assert np.linalg.norm(g - H @ a["w"]) / np.linalg.norm(g) <= 1e-10
    assert np.linalg.norm(g - H @ b["w"]) / np.linalg.norm(g) <= 1e-10
    assert abs(a["iters"] - b["iters"]) <= 3
    assert not np.array_equal(a["w"], b["w"])
    # at a fixed small iteration count the two recurrences agree to rounding
    a5 = krylov.recycled_cg(lambda v: H @ v, g, None, U, C, tol=0.0, max_iter=5)
    b5 = krylov.recycled_cg(lambda v: H @ v, g, None, U, C, tol=0.0, max_iter=5, recurrence="single")
    assert np.linalg.norm(a5["w"] - b5["w"]) <= 1e-12 * np.linalg.norm(a5["w"])


def test_indefinite_detected():
    n = 20
    H = spd(n, 10.0, 16)
    H[0, 0] = -50.0
    g = np.zeros(n)
    g[0] = 1.0
    res = krylov.recycled_cg(lambda v: H @ v, g, tol=1e-12)
    assert res["status"] == krylov.INDEFINITE


def test_hg_stop_uses_estimate():
    n, s = 60, 4
    H = spd(n, 100.0, 17)
    g = np.random.default_rng(18).standard_normal(n)
    U, C = recycle_pair(H, s, 19)
    Z = np.linalg.qr(np.random.default_rng(20).standard_normal((n, s)))[0]
    mu = np.array([3.0, 2.0, 1.0, 0.0])
    res = krylov.recycled_cg(lambda v: H @ v, g, None, U, C, Z, mu, stop="hgerr", hg_tol=1e-3, record=True)
    est = np.linalg.norm(mu * (Z.T @ res["r"]))
    assert est <= 1e-3
    assert res["hist_nsc"][-1] == pytest.approx(est, rel=1e-10)
    assert all(e > 1e-3 for e in res["hist_nsc"][:-1])


def test_reference_solve_tight():
    H = spd(40, 1e4, 21)
    g = np.random.default_rng(22).standard_normal(40)
    w, _ = krylov.reference_solve(lambda v: H @ v, g)
    assert np.linalg.norm(H @ w - g) <= 1e-12 * np.linalg.norm(g)


# ------------------------------------------------------------------ deflated CG (the O5 alternative)
@pytest.mark.parametrize("s", [3, 8])
def test_deflated_cg_minimises_energy_error_over_augmented_space(s):
    """Deflated CG (Saad et al. 2000): after j iterations the iterate is the energy-norm best
    approximation of w* over w0 + span(U, p_0, ..., p_{j-1}) (brute force: the Galerkin system
    of that basis); its residuals stay orthogonal to U and its directions H-conjugate to U."""
    H = spd(50, 3e3, 11 + s)
    rng = np.random.default_rng(12)
    g = rng.standard_normal(50)
    w0 = rng.standard_normal(50)
    U, C = recycle_pair(H, s, 13)
    wstar = np.linalg.solve(H, g)
    for j in (1, 4, 9):
        res = krylov.deflated_cg(lambda v: H @ v, g, w0, U, C, tol=0.0, max_iter=j, record=True)
        Bm = np.concatenate([U, np.stack(res["P"], axis=1)], axis=1)
        c = np.linalg.solve(Bm.T @ H @ Bm, Bm.T @ (g - H @ w0))
        best = w0 + Bm @ c
        assert np.linalg.norm(res["w"] - best) <= 1e-9 * np.linalg.norm(wstar)
        assert np.abs(U.T @ res["r"]).max() <= 1e-10 * np.linalg.norm(g)
        for p in res["P"]:
            assert np.abs(C.T @ p).max() <= 1e-10 * np.linalg.norm(p)
        # the recursive residual is the true residual
        assert np.linalg.norm(res["r"] - (g - H @ res["w"])) <= 1e-10 * np.linalg.norm(g)


def test_deflated_cg_special_cases():
    """No deflation space: textbook CG, bit for bit the same arithmetic as plain CG; w* - w0 in
    range(U): the set-up alone gives w* (zero iterations); converges to the dense solution."""
    H = spd(40, 1e3, 21)
    rng = np.random.default_rng(22)
    g = rng.standard_normal(40)
    a = krylov.deflated_cg(lambda v: H @ v, g, tol=1e-10)
    b = krylov.cg(lambda v: H @ v, g, tol=1e-10)
    assert a["iters"] == b["iters"] and np.array_equal(a["w"], b["w"])
    wstar = np.linalg.solve(H, g)
    w0 = rng.standard_normal(40)
    Ut = np.concatenate([(wstar - w0)[:, None], rng.standard_normal((40, 2))], axis=1)
    Qc, Rc = np.linalg.qr(H @ Ut)
    U = Ut @ np.linalg.inv(Rc)
    one = krylov.deflated_cg(lambda v: H @ v, g, w0, U, Qc, tol=1e-9)
    assert one["iters"] == 0 and np.linalg.norm(one["w"] - wstar) <= 1e-10 * np.linalg.norm(wstar)
    U, C = recycle_pair(H, 5, 23)
    full = krylov.deflated_cg(lambda v: H @ v, g, w0, U, C, tol=1e-12)
    assert full["status"] == krylov.OK
    assert np.linalg.norm(full["w"] - wstar) <= 1e-8 * np.linalg.norm(wstar)
