"""Pins of the oracle's objectives, Hessian-vector products and hypergradients.

Dense Hessians assembled from the formulas, central finite differences,
forward-mode identities and the quadratic special case (phi = s^2, where the
lower-level solution is one linear solve).
"""
import numpy as np
import pytest

import synth
from oracle import lbfgs, ops, problem


def tv_case(h=8, w=8, seed=5):
    wl = synth.custom("t", h, "tv", 4, width=w, blur_radius=2, blur_sigma=1.5, rect_min=1, rect_max=3, seed=seed)
    inst = synth.instance(wl)
    return wl, inst, problem.make_problem(wl, inst["xstar"], inst["e"])


def foe_case(h=8, w=8, seed=6, penalty="log", n_filters=2, fsize=3):
    wl = synth.custom("f", h, "filters", 4, width=w, blur_radius=1, blur_sigma=1.0, rect_min=1, rect_max=3, seed=seed,
                      n_filters=n_filters, filter_size=fsize)
    inst = synth.instance(wl)
    filt = synth.zero_mean_filters(n_filters, fsize, np.random.default_rng(seed + 1), std=0.3)
    theta = synth.initial_theta(wl, filt)
    return wl, inst, problem.make_problem(wl, inst["xstar"], inst["e"], penalty), theta


def fd_grad(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def test_tv_gradient_and_hvp_fd():
    wl, inst, prob = tv_case()
    th = inst["theta0"] + np.array([1.0, 2.0])   # larger smoothing keeps FD well conditioned
    rng = np.random.default_rng(0)
    x = rng.standard_normal(prob.n) * 0.3
    g = prob.grad(x, th)
    gfd = fd_grad(lambda v: prob.phi(v, th), x)
    assert np.linalg.norm(g - gfd) / np.linalg.norm(g) < 1e-8
    v = rng.standard_normal(prob.n)
    hv = prob.hvp(x, th, v)
    hfd = (prob.grad(x + 1e-6 * v, th) - prob.grad(x - 1e-6 * v, th)) / 2e-6
    assert np.linalg.norm(hv - hfd) / np.linalg.norm(hv) < 1e-7


def test_tv_dense_hessian_spd_and_matches_hvp():
    wl, inst, prob = tv_case(6, 7)
    th = inst["theta0"]
    x = np.random.default_rng(1).standard_normal(prob.n) * 0.2
    Hd = prob.dense_hessian(x, th)
    Hh = np.stack([prob.hvp(x, th, col) for col in np.eye(prob.n)], axis=1)
    assert np.abs(Hd - Hh).max() <= 1e-13 * np.abs(Hd).max()
    assert np.abs(Hh - Hh.T).max() <= 1e-14 * np.abs(Hh).max()
    assert np.linalg.eigvalsh(Hd).min() > 0.0
    np.linalg.cholesky(Hd)


def test_tv_reduces_to_least_squares():
    wl, inst, prob = tv_case()
    x = np.random.default_rng(2).standard_normal(prob.n)
    th = np.array([-60.0, np.log(0.01)])
    ls = 2.0 * ops.correlate_adjoint(prob.A(x) - prob.y, prob.kernel).ravel()
    assert np.abs(prob.grad(x, th) - ls).max() < 1e-20 + 1e-12 * np.abs(ls).max()


@pytest.mark.parametrize("penalty", ["log", "quad"])
def test_filters_gradient_hvp_dense(penalty):
    wl, inst, prob, th = foe_case(penalty=penalty)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(prob.n) * 0.5
    g = prob.grad(x, th)
    gfd = fd_grad(lambda v: prob.phi(v, th), x)
    assert np.linalg.norm(g - gfd) / np.linalg.norm(g) < 1e-8
    Hd = prob.dense_hessian(x, th)
    Hh = np.stack([prob.hvp(x, th, col) for col in np.eye(prob.n)], axis=1)
    assert np.abs(Hd - Hh).max() <= 1e-13 * np.abs(Hd).max()
    assert np.abs(Hh - Hh.T).max() <= 1e-14 * np.abs(Hh).max()


@pytest.mark.parametrize("penalty", ["log", "quad"])
def test_filters_dtheta_grad_fd(penalty):
    """Columns of D_theta grad_x Phi against central differences of grad_x Phi in theta."""
    wl, inst, prob, th = foe_case(penalty=penalty)
    x = np.random.default_rng(4).standard_normal(prob.n) * 0.5
    Dt = prob.dtheta_grad(x, th)
    for j in range(prob.p):
        e = np.zeros(prob.p)
        e[j] = 1e-6
        col = (prob.grad(x, th + e) - prob.grad(x, th - e)) / 2e-6
        assert np.linalg.norm(Dt[:, j] - col) <= 1e-7 * max(1.0, np.linalg.norm(col))


def test_tv_dtheta_grad_fd():
    wl, inst, prob = tv_case()
    th = inst["theta0"]
    x = np.random.default_rng(5).standard_normal(prob.n) * 0.3
    Dt = prob.dtheta_grad(x, th)
    for j in range(2):
        e = np.zeros(2)
        e[j] = 1e-6
        col = (prob.grad(x, th + e) - prob.grad(x, th - e)) / 2e-6
        assert np.linalg.norm(Dt[:, j] - col) <= 1e-6 * np.linalg.norm(col)


@pytest.mark.parametrize("kind", ["tv", "log"])
def test_jac_apply_is_adjoint_of_mixed_derivative(kind):
    if kind == "tv":
        wl, inst, prob = tv_case()
        th = inst["theta0"]
        kw = {}
    else:
        wl, inst, prob, th = foe_case()
        kw = {"project": False}
    rng = np.random.default_rng(6)
    x = rng.standard_normal(prob.n) * 0.4
    w = rng.standard_normal(prob.n)
    assert np.allclose(prob.jac_apply(x, th, w, **kw), -prob.dtheta_grad(x, th).T @ w, rtol=1e-12, atol=1e-13)


def solve_lower_exact(prob, th, x0):
    x, _ = lbfgs.lbfgs(lambda v: prob.phi(v, th), lambda v: prob.grad(v, th), x0, gtol=1e-6)
    return lbfgs.newton_polish(lambda v: prob.grad(v, th), lambda v: prob.dense_hessian(v, th), x, steps=6)


def upper_of(prob, th, xstar, x0):
    """Upper loss at theta; the lower solve is Newton from a nearby minimiser (quadratic convergence)."""
    x = lbfgs.newton_polish(lambda v: prob.grad(v, th), lambda v: prob.dense_hessian(v, th), x0, steps=6)
    assert np.linalg.norm(prob.grad(x, th)) < 1e-11
    return problem.upper_loss(x, xstar), x


@pytest.mark.parametrize("kind", ["tv", "log"])
def test_hypergradient_central_fd(kind):
    """Hypergradient J H^{-1} g against central FD of the upper loss (Newton-polished lower solves)."""
    if kind == "tv":
        wl, inst, prob = tv_case()
        th = inst["theta0"]
        project = {}
    else:
        wl, inst, prob, th = foe_case()
        project = {"project": False}
    xs = inst["xstar"].ravel()
    xh = solve_lower_exact(prob, th, prob.y.ravel())
    Hd = prob.dense_hessian(xh, th)
    w = np.linalg.solve(Hd, xh - xs)
    hg = prob.jac_apply(xh, th, w, **project)
    fd = np.zeros(prob.p)
    for j in range(prob.p):
        hstep = 1e-5 * max(1.0, abs(th[j]))
        e = np.zeros(prob.p)
        e[j] = hstep
        fp, _ = upper_of(prob, th + e, xs, xh)
        fm, _ = upper_of(prob, th - e, xs, xh)
        fd[j] = (fp - fm) / (2 * hstep)
    assert np.linalg.norm(hg - fd) / np.linalg.norm(hg) < 1e-5


def test_quadratic_special_case_closed_form_hypergradient():
    """phi = s^2: x_hat = (2A^TA + eps I + sum 2 lam_j K_j^T K_j)^{-1} 2 A^T y exactly; FD of the closed form."""
    wl, inst, prob, th = foe_case(penalty="quad", seed=9)
    xs = inst["xstar"].ravel()
    Am = ops.dense_correlation(prob.h, prob.w, prob.kernel)

    def xhat(t):
        lam, ks = prob.unpack(t)
        Hm = 2 * Am.T @ Am + prob.eps * np.eye(prob.n)
        for j in range(prob.N):
            Km = ops.dense_correlation(prob.h, prob.w, ks[j])
            Hm = Hm + 2 * lam[j] * Km.T @ Km
        return np.linalg.solve(Hm, 2 * Am.T @ prob.y.ravel())

    xh = xhat(th)
    assert np.linalg.norm(prob.grad(xh, th)) < 1e-10
    w = np.linalg.solve(prob.dense_hessian(xh, th), xh - xs)
    hg = prob.jac_apply(xh, th, w, project=False)
    fd = np.zeros(prob.p)
    for j in range(prob.p):
        e = np.zeros(prob.p)
        e[j] = 1e-6
        fd[j] = (problem.upper_loss(xhat(th + e), xs) - problem.upper_loss(xhat(th - e), xs)) / 2e-6
    assert np.linalg.norm(hg - fd) / np.linalg.norm(hg) < 1e-7


def test_forward_mode_identity():
    """[grad L]_j = g^T dx_hat/dtheta_j with dx_hat/dtheta_j = -H^{-1} d_theta_j grad_x Phi (p solves)."""
    wl, inst, prob, th = foe_case(seed=11)
    x = np.random.default_rng(7).standard_normal(prob.n) * 0.3
    g = np.random.default_rng(8).standard_normal(prob.n)
    Hd = prob.dense_hessian(x, th)
    Hd = Hd + (abs(min(0.0, np.linalg.eigvalsh(Hd).min())) + 1.0) * np.eye(prob.n)
    hvp_solve = np.linalg.solve(Hd, g)
    Dt = prob.dtheta_grad(x, th)
    fwd = np.array([g @ (-np.linalg.solve(Hd, Dt[:, j])) for j in range(prob.p)])
    # adjoint route uses the same (shifted) H through w = H^{-1} g
    adj = prob.jac_apply(x, th, hvp_solve, project=False)
    assert np.linalg.norm(adj - fwd) <= 1e-10 * np.linalg.norm(fwd)


def test_zero_mean_projection():
    wl, inst, prob, th = foe_case()
    x = np.random.default_rng(9).standard_normal(prob.n)
    w = np.random.default_rng(10).standard_normal(prob.n)
    a = prob.jac_apply(x, th, w, project=True)
    b = problem.project_zero_mean(prob.jac_apply(x, th, w, project=False), prob.N, prob.f)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
    taps = a.reshape(prob.N, -1)[:, 1:]
    assert np.abs(taps.sum(axis=1)).max() < 1e-13


def _lbfgs_min(prob, th, x0, gtol):
    return lbfgs.lbfgs(lambda v: prob.phi(v, th), lambda v: prob.grad(v, th), x0, gtol=gtol)


@pytest.mark.parametrize("kind,side", [("tv", 8), ("tv", 16), ("log", 8), ("log", 16)])
def test_lbfgs_reaches_the_minimiser(kind, side):
    """L-BFGS (Section 5: history 10, gradient-norm stop) returns a point within ||grad|| / lambda_min(H)
    of the minimiser, the minimiser being found independently by Newton's method to ||grad|| < 1e-12."""
    if kind == "tv":
        wl, inst, prob = tv_case(side, side, seed=30 + side)
        th = inst["theta0"]
    else:
        wl, inst, prob, th = foe_case(side, side, seed=40 + side)
    gtol = 1e-8
    x, info = _lbfgs_min(prob, th, prob.y.ravel(), gtol)
    assert info["converged"] and info["iters"] > 0
    gn = float(np.linalg.norm(prob.grad(x, th)))
    assert gn <= gtol
    xn = lbfgs.newton_polish(lambda v: prob.grad(v, th), lambda v: prob.dense_hessian(v, th), x, steps=6)
    assert np.linalg.norm(prob.grad(xn, th)) < 1e-12
    lam_min = float(np.linalg.eigvalsh(prob.dense_hessian(xn, th)).min())
    assert lam_min > 0.0
    assert np.linalg.norm(x - xn) <= 1.5 * gn / lam_min + 1e-14


def test_lbfgs_quadratic_penalty_closed_form():
    """phi = s^2: the lower-level minimiser is one linear solve; L-BFGS must land on it."""
    wl, inst, prob, th = foe_case(penalty="quad", seed=12)
    Am = ops.dense_correlation(prob.h, prob.w, prob.kernel)
    lam, ks = prob.unpack(th)
    Hm = 2 * Am.T @ Am + prob.eps * np.eye(prob.n)
    for j in range(prob.N):
        Km = ops.dense_correlation(prob.h, prob.w, ks[j])
        Hm = Hm + 2 * lam[j] * Km.T @ Km
    x_cf = np.linalg.solve(Hm, 2 * Am.T @ prob.y.ravel())
    gtol = 1e-9
    x, info = _lbfgs_min(prob, th, prob.y.ravel(), gtol)
    assert info["converged"]
    lam_min = float(np.linalg.eigvalsh(Hm).min())
    assert np.linalg.norm(x - x_cf) <= 1.5 * gtol / lam_min
