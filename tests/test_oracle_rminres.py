"""Pins of the oracle's RMINRES (Section 2.2.2, Algorithm 3; residual of Appendix A).

* every iterate equals the minimiser of ||g - H x|| over w0 + range(U) + K_k((I - CC^T) H, r0')
  (eq. coupled), found by brute force with a dense least-squares solve; on indefinite H too;
  a plus sign on b~ in the update (as printed in Algorithm 3) fails this;
* |zeta_k| equals the true residual norm ||g - H w_k|| at every step (MINRES's QR relation);
* the explicit residual of Appendix A equals g - H w_k; without H on its k - 2 terms it fails;
* the residual norm never increases; finite termination in n steps; a direct solve;
* stop tests: zero iterations when the start already passes; check_every; the estimate
  test stops at the first tested iterate whose estimate passes; the iteration limit.
"""
import numpy as np
import pytest

from oracle import rminres


def sym(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.asarray(eigs)) @ Q.T


def recycle_pair(H, s, seed):
    """U, C with C = H U and C^T C = I (thin QR of H U~, U = U~ R^{-1})."""
    rng = np.random.default_rng(seed)
    Ut = rng.standard_normal((H.shape[0], s))
    Qc, Rc = np.linalg.qr(H @ Ut)
    return Ut @ np.linalg.inv(Rc), Qc


def minres_iterate(H, g, w0, U, C, k):
    """Brute force of eq. coupled: min over x in w0 + range(U) + K_k(P H, P r0) of ||g - H x||."""
    n = H.shape[0]
    r0 = g - H @ w0
    cols = []
    if U is not None:
        P = np.eye(n) - C @ C.T
        b = P @ r0
        Op = P @ H
    else:
        b, Op = r0, H
    kc = [b]
    for _ in range(k - 1):
        kc.append(Op @ kc[-1])
    Kb, _ = np.linalg.qr(np.stack(kc, axis=1))
    basis = Kb if U is None else np.concatenate([Kb, U], axis=1)
    coef, *_ = np.linalg.lstsq(H @ basis, r0, rcond=None)
    return w0 + basis @ coef


def run_steps(H, g, w0, U, C, k):
    return rminres.rminres(lambda v: H @ v, g, w0, U, C, tol=0.0, max_iter=k)


@pytest.mark.parametrize("indef", [False, True])
@pytest.mark.parametrize("s", [0, 3])
def test_iterates_minimise_residual_over_augmented_space(indef, s):
    n = 40
    eigs = np.geomspace(1.0, 50.0, n)
    if indef:
        eigs[::3] *= -1.0
    H = sym(n, eigs, 10 + s)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(n)
    w0 = 0.1 * rng.standard_normal(n)
    U, C = recycle_pair(H, s, 12) if s else (None, None)
    for k in (1, 2, 3, 5, 8):
        res = run_steps(H, g, w0, U, C, k)
        assert res["iters"] == k
        ref = minres_iterate(H, g, w0, U, C, k)
        assert np.linalg.norm(res["w"] - ref) <= 1e-9 * np.linalg.norm(ref), k


def test_plus_sign_on_b_fails_the_pin():
    """The recycle part enters with a minus sign: the printed plus sign is not minimal."""
    n, s, k = 30, 3, 4
    H = sym(n, np.geomspace(1.0, 20.0, n), 21)
    g = np.random.default_rng(22).standard_normal(n)
    U, C = recycle_pair(H, s, 23)
    ref = minres_iterate(H, g, np.zeros(n), U, C, k)
    assert np.linalg.norm(run_steps(H, g, None, U, C, k)["w"] - ref) <= 1e-9 * np.linalg.norm(ref)
    w_plus = plus_sign_iterate(H, g, U, C, k)
    assert np.linalg.norm(g - H @ w_plus) > 1.01 * np.linalg.norm(g - H @ ref)


def plus_sign_iterate(H, g, U, C, k):
    """Algorithm 3 with the update as printed, w += c_k zeta_{k-1} (v~_k + b~_k)."""
    n = g.size
    r = g.copy()
    c0 = C.T @ r
    w = U @ c0
    r = r - C @ c0
    beta = np.linalg.norm(r)
    v_prev, v = np.zeros(n), r / beta
    zeta = beta
    c1, s1, c2, s2 = 1.0, 0.0, 0.0, 0.0
    vt1 = vt2 = bt1 = bt2 = np.zeros(n)
    for _ in range(k):
        Hv = H @ v
        b = U @ (C.T @ Hv)
        u = Hv - C @ (C.T @ Hv)
        alpha = v @ u
        u = u - alpha * v - beta * v_prev
        bn = np.linalg.norm(u)
        gamma = s2 * beta
        delta = c1 * c2 * beta + s1 * alpha
        eps = -s1 * c2 * beta + c1 * alpha
        et = np.hypot(eps, bn)
        ck, sk = eps / et, bn / et
        tau = ck * zeta
        zeta = -sk * zeta
        vt = (v - gamma * vt2 - delta * vt1) / et
        bt = (b - gamma * bt2 - delta * bt1) / et
        w = w + tau * (vt + bt)
        vt2, vt1, bt2, bt1 = vt1, vt, bt1, bt
        c2, s2, c1, s1 = c1, s1, ck, sk
        v_prev, v = v, u / bn
        beta = bn
    return w


@pytest.mark.parametrize("s", [0, 4])
def test_zeta_is_true_residual_norm_and_appendix_residual(s):
    n = 50
    eigs = np.linspace(-3.0, 10.0, n)
    eigs[np.abs(eigs) < 0.2] = 0.5
    H = sym(n, eigs, 30 + s)
    g = np.random.default_rng(31).standard_normal(n)
    U, C = recycle_pair(H, s, 32) if s else (None, None)
    res = rminres.rminres(lambda v: H @ v, g, None, U, C, tol=0.0, max_iter=25, record=True)
    hist = res["hist_res"]
    assert len(hist) == 26
    for k in (1, 5, 12, 25):
        w = run_steps(H, g, None, U, C, k)["w"]
        true = np.linalg.norm(g - H @ w)
        assert abs(hist[k] - true) <= 1e-10 * np.linalg.norm(g), k
    # explicit residual of Appendix A against g - H w
    r_true = g - H @ res["w"]
    assert np.linalg.norm(res["r"] - r_true) <= 1e-10 * np.linalg.norm(g)
    if s:
        assert np.linalg.norm(C.T @ res["r"]) <= 1e-10 * np.linalg.norm(g)
    # non-increasing residual norms (minimal residual over nested spaces)
    assert all(b <= a * (1 + 1e-12) + 1e-14 for a, b in zip(hist, hist[1:]))


def test_appendix_recurrence_needs_h_on_older_terms():
    """Dropping H from the k - 2 terms (as printed) makes the explicit residual drift."""
    n = 40
    H = sym(n, np.geomspace(1.0, 30.0, n), 41)
    g = np.random.default_rng(42).standard_normal(n)
    # replay the oracle's scalars with the printed (H-less) k - 2 terms
    res = rminres.rminres(lambda v: H @ v, g, tol=0.0, max_iter=12)
    wrong = printed_recurrence_residual(H, g, 12)
    assert np.linalg.norm(res["r"] - (g - H @ res["w"])) <= 1e-10 * np.linalg.norm(g)
    assert np.linalg.norm(wrong - (g - H @ res["w"])) > 1e-3 * np.linalg.norm(g)


def printed_recurrence_residual(H, g, k):
    """Plain MINRES (U empty) whose residual drops H from the gamma terms."""
    n = g.size
    r = g.copy()
    beta = np.linalg.norm(r)
    v_prev, v = np.zeros(n), r / beta
    zeta = beta
    c1, s1, c2, s2 = 1.0, 0.0, 0.0, 0.0
    vt1 = vt2 = Hvt1 = Hvt2 = np.zeros(n)
    for _ in range(k):
        Hv = H @ v
        alpha = v @ Hv
        u = Hv - alpha * v - beta * v_prev
        bn = np.linalg.norm(u)
        gamma = s2 * beta
        delta = c1 * c2 * beta + s1 * alpha
        eps = -s1 * c2 * beta + c1 * alpha
        et = np.hypot(eps, bn)
        ck, sk = eps / et, bn / et
        tau = ck * zeta
        zeta = -sk * zeta
        vt = (v - gamma * vt2 - delta * vt1) / et
        Hvt = (Hv - delta * Hvt1 - gamma * vt2) / et       # printed form
        r = r - tau * Hvt
        vt2, vt1, Hvt2, Hvt1 = vt1, vt, Hvt1, Hvt
        c2, s2, c1, s1 = c1, s1, ck, sk
        v_prev, v = v, u / bn
        beta = bn
    return r


def test_finite_termination_and_direct_solve():
    n = 16
    eigs = np.concatenate([-np.geomspace(1.0, 4.0, 6), np.geomspace(1.0, 8.0, 10)])
    H = sym(n, eigs, 51)
    g = np.random.default_rng(52).standard_normal(n)
    # n steps in exact arithmetic; rounding leaves the n-th residual near 1e-11 here
    res = rminres.rminres(lambda v: H @ v, g, tol=1e-9, max_iter=n)
    assert res["status"] == rminres.OK and res["iters"] == n
    w = np.linalg.solve(H, g)
    assert np.linalg.norm(res["w"] - w) <= 1e-9 * np.linalg.norm(w)


def test_zero_iterations_when_start_passes():
    H = sym(10, np.linspace(1.0, 5.0, 10), 61)
    w = np.random.default_rng(62).standard_normal(10)
    g = H @ w
    res = rminres.rminres(lambda v: H @ v, g, w, tol=1e-8)
    assert res["iters"] == 0 and res["status"] == rminres.OK
    assert np.array_equal(res["w"], w)
    res = rminres.rminres(lambda v: H @ v, np.zeros(10))
    assert res["iters"] == 0 and res["res_norm"] == 0.0


def test_check_every_and_limit():
    n = 60
    H = sym(n, np.geomspace(1.0, 1e3, n), 71)
    g = np.random.default_rng(72).standard_normal(n)
    every = rminres.rminres(lambda v: H @ v, g, tol=1e-6, record=True)
    k1 = every["iters"]
    res4 = rminres.rminres(lambda v: H @ v, g, tol=1e-6, check_every=4)
    assert res4["iters"] == -(-k1 // 4) * 4
    lim = rminres.rminres(lambda v: H @ v, g, tol=1e-12, max_iter=7)
    assert lim["status"] == rminres.NOT_CONVERGED and lim["iters"] == 7
    assert np.array_equal(lim["w"], run_steps(H, g, None, None, None, 7)["w"])


def test_estimate_stop_first_passing_tested_iterate():
    n, s = 50, 5
    H = sym(n, np.geomspace(1.0, 100.0, n), 81)
    g = np.random.default_rng(82).standard_normal(n)
    U, C = recycle_pair(H, s, 83)
    Z = np.linalg.qr(np.random.default_rng(84).standard_normal((n, s)))[0]
    mu = np.array([3.0, 2.0, 1.0, 0.5, 0.0])
    full = rminres.rminres(lambda v: H @ v, g, None, U, C, Z, mu, tol=0.0, max_iter=40, record=True)
    est = np.array(full["hist_nsc"])
    # the estimate is ||mu . Z^T r_j|| of the true residual at every step
    for j in (0, 3, 9):
        wj = run_steps(H, g, None, U, C, j)["w"] if j else None
        rj = g - H @ (wj if j else (U @ (C.T @ g)))
        assert abs(est[j] - np.linalg.norm(mu * (Z.T @ rj))) <= 1e-10 * np.linalg.norm(g)
    thr = float(np.sort(est[1:30])[len(est[1:30]) // 2])
    for every in (1, 3):
        res = rminres.rminres(lambda v: H @ v, g, None, U, C, Z, mu, stop="hgerr", hg_tol=thr, check_every=every)
        first = next(j for j in range(0, 41, every) if est[j] <= thr)
        assert res["iters"] == first and res["status"] == rminres.OK


def test_indefinite_filter_hessian_solved_where_cg_stops():
    """Filters at a point with large responses: phi'' < 0 makes H indefinite.  CG reports it;
    RMINRES reaches the tolerance, and its solution satisfies H w = g."""
    import synth
    from oracle import krylov, problem

    wl = synth.custom("indef", 12, "filters", 2, rect_min=2, rect_max=4, seed=111)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"].copy()
    f2 = wl.filter_size ** 2
    for j in range(wl.n_filters):
        th[j * (1 + f2)] = np.log(50.0)
    x = 8.0 * synth.unit_noise(prob.n, 112)
    g = synth.unit_noise(prob.n, 113)
    hvp = lambda v: prob.hvp(x, th, v)
    Hd = np.stack([hvp(col) for col in np.eye(prob.n)], axis=1)
    ev = np.linalg.eigvalsh(0.5 * (Hd + Hd.T))
    assert ev[0] < 0.0 < ev[-1]
    assert krylov.cg(hvp, g, tol=1e-10, max_iter=2000)["status"] == krylov.INDEFINITE
    res = rminres.rminres(hvp, g, tol=1e-10, max_iter=2000)
    assert res["status"] == rminres.OK
    assert np.linalg.norm(g - hvp(res["w"])) <= 2e-10 * np.linalg.norm(g)
    assert np.linalg.norm(res["w"] - np.linalg.solve(Hd, g)) <= 1e-6 * np.linalg.norm(res["w"])


def test_tv_solve_matches_reference_and_cg():
    """SPD TV Hessian: RMINRES and CG reach the same solution, with and without recycling."""
    import synth
    from oracle import krylov, problem, recycle

    wl = synth.custom("tvm", 16, "tv", 4, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=4, seed=7)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"]
    xh = inst["xstar"].ravel() + 0.05 * synth.unit_noise(prob.n, 8)
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    wref, _ = krylov.reference_solve(hvp, g)
    plain = rminres.rminres(hvp, g, tol=1e-11)
    assert plain["status"] == rminres.OK
    assert np.linalg.norm(plain["w"] - wref) <= 1e-8 * np.linalg.norm(wref)
    cg0 = krylov.cg(hvp, g, tol=1e-10, v_cap=16)
    rs = recycle.refresh(hvp, lambda v: prob.jac_apply(xh, th, v), None, cg0["V"], s=4)
    rec = rminres.rminres(hvp, g, None, rs["U"], rs["C"], tol=1e-11)
    assert rec["status"] == rminres.OK and rec["iters"] <= plain["iters"]
    assert np.linalg.norm(rec["w"] - wref) <= 1e-8 * np.linalg.norm(wref)
