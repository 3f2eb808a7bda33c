"""Lower-level objectives, their derivatives and the hypergradient map, FP64.

Setting (Section 2.1, eqs. bl2, implicit-update-context, hg-full, hess_sys, hypgrad):
  x_hat(theta) = argmin_x Phi(x, theta),  upper loss l(x) = 1/2 ||x - x*||^2,
  H = D^2_xx Phi(x_hat, theta),  g = grad l(x_hat) = x_hat - x*,
  hypergradient = J H^{-1} g  with  J = -(D_theta grad_x Phi)^T  (p x n).

Two regularisers:

* Smoothed TV (the deblurring workloads), p = 2, theta = (log weight, log smoothing):
    Phi = ||A x - y||^2 + e^{theta0} sum_i sqrt(|(D x)_i|^2 + e^{2 theta1}).
* Fields of experts (eq. ll2ex): N learned f x f filters k_j with weights e^{w_j},
    Phi = ||A x - y||^2 + eps/2 ||x||^2 + sum_j e^{w_j} sum_i phi((K_j x)_i),
  phi(s) = log(1 + s^2) (the paper's deconvolution choice) or s^2 (its inpainting choice),
  theta = [w_1, k_1 (row-major), ..., w_N, k_N] (interleaved layout of Section 5).
  The data term carries no 1/2 here because the workload recipes state ||Ax - y||^2.
  Filters are zero-mean; ``J`` optionally projects each filter's coefficient block
  onto zero mean (the constraint's tangent space).

All derivative formulas are derived by hand from these objectives; the pins in the
tests check them against dense matrices, finite differences and forward mode.
"""
from __future__ import annotations

import numpy as np

from . import ops


class TVProblem:
    p = 2

    def __init__(self, h: int, w: int, radius: int, sigma: float, y: np.ndarray):
        self.h, self.w, self.n = h, w, h * w
        self.radius, self.sigma = radius, sigma
        self.kernel = ops.gaussian_kernel(radius, sigma)
        self.y = np.asarray(y, dtype=np.float64).reshape(h, w)

    # -- helpers
    def _img(self, v):
        return np.asarray(v, dtype=np.float64).reshape(self.h, self.w)

    def A(self, v):
        return ops.correlate(self._img(v), self.kernel)

    @staticmethod
    def _lam_gam2(theta):
        return float(np.exp(theta[0])), float(np.exp(2.0 * theta[1]))

    def _state(self, x, theta):
        lam, gam2 = self._lam_gam2(theta)
        a, b = ops.grad_fwd(self._img(x))
        psi = np.sqrt(a * a + b * b + gam2)
        return lam, gam2, a, b, psi

    # -- objective and derivatives in x
    def phi(self, x, theta) -> float:
        lam, gam2, a, b, psi = self._state(x, theta)
        res = self.A(x) - self.y
        return float(np.sum(res * res) + lam * np.sum(psi))

    def grad(self, x, theta) -> np.ndarray:
        lam, gam2, a, b, psi = self._state(x, theta)
        data = 2.0 * ops.correlate_adjoint(self.A(x) - self.y, self.kernel)
        reg = lam * ops.grad_fwd_adjoint(a / psi, b / psi)
        return (data + reg).ravel()

    def hessian_blocks(self, x, theta):
        """Per-pixel 2x2 blocks B_i = d(u/psi(u))/du at u = (Dx)_i = (psi^2 I - u u^T) / psi^3."""
        lam, gam2, a, b, psi = self._state(x, theta)
        p3 = psi ** 3
        return lam, (b * b + gam2) / p3, (-a * b) / p3, (a * a + gam2) / p3

    def hvp(self, x, theta, v) -> np.ndarray:
        """H v = 2 A^T A v + lambda D^T (B D v)."""
        lam, b11, b12, b22 = self.hessian_blocks(x, theta)
        V = self._img(v)
        data = 2.0 * ops.correlate_adjoint(ops.correlate(V, self.kernel), self.kernel)
        da, db = ops.grad_fwd(V)
        reg = lam * ops.grad_fwd_adjoint(b11 * da + b12 * db, b12 * da + b22 * db)
        return (data + reg).ravel()

    # -- mixed derivative and hypergradient
    def dtheta_grad(self, x, theta) -> np.ndarray:
        """n x p matrix D_theta grad_x Phi (columns: d/dtheta0, d/dtheta1)."""
        lam, gam2, a, b, psi = self._state(x, theta)
        c0 = lam * ops.grad_fwd_adjoint(a / psi, b / psi)
        # d/dtheta1 of lam D^T (Dx / psi): d psi/d theta1 = gam2 / psi
        c1 = -lam * gam2 * ops.grad_fwd_adjoint(a / psi ** 3, b / psi ** 3)
        return np.stack([c0.ravel(), c1.ravel()], axis=1)

    def jac_apply(self, x, theta, w) -> np.ndarray:
        """J w = -(D_theta grad_x Phi)^T w, via <D x/psi, D w> forms (eq. hypgrad)."""
        lam, gam2, a, b, psi = self._state(x, theta)
        da, db = ops.grad_fwd(self._img(w))
        g0 = -lam * np.sum((a * da + b * db) / psi)
        g1 = lam * gam2 * np.sum((a * da + b * db) / psi ** 3)
        return np.array([g0, g1])

    def dense_hessian(self, x, theta) -> np.ndarray:
        """H from its formula with dense A (Toeplitz) and dense D (tiny images only)."""
        lam, b11, b12, b22 = self.hessian_blocks(x, theta)
        Am = ops.dense_correlation(self.h, self.w, self.kernel)
        Dm = ops.dense_grad_fwd(self.h, self.w)
        n = self.n
        Bm = np.zeros((2 * n, 2 * n))
        idx = np.arange(n)
        Bm[idx, idx] = b11.ravel()
        Bm[idx, n + idx] = b12.ravel()
        Bm[n + idx, idx] = b12.ravel()
        Bm[n + idx, n + idx] = b22.ravel()
        return 2.0 * Am.T @ Am + lam * Dm.T @ Bm @ Dm


def _penalty(kind: str):
    if kind == "log":
        return (lambda s: np.log1p(s * s),
                lambda s: 2.0 * s / (1.0 + s * s),
                lambda s: 2.0 * (1.0 - s * s) / (1.0 + s * s) ** 2)
    if kind == "quad":
        return (lambda s: s * s, lambda s: 2.0 * s, lambda s: 2.0 * np.ones_like(s))
    raise ValueError(kind)


class FilterProblem:
    def __init__(self, h: int, w: int, radius: int, sigma: float, y: np.ndarray,
                 n_filters: int, fsize: int, eps: float, penalty: str = "log"):
        self.h, self.w, self.n = h, w, h * w
        self.radius, self.sigma = radius, sigma
        self.kernel = ops.gaussian_kernel(radius, sigma)
        self.y = np.asarray(y, dtype=np.float64).reshape(h, w)
        self.N, self.f, self.eps = n_filters, fsize, eps
        self.p = n_filters * (1 + fsize * fsize)
        self.pen, self.dpen, self.ddpen = _penalty(penalty)

    def _img(self, v):
        return np.asarray(v, dtype=np.float64).reshape(self.h, self.w)

    def A(self, v):
        return ops.correlate(self._img(v), self.kernel)

    def unpack(self, theta):
        """theta -> (lambda_j = e^{w_j}, k_j as f x f arrays)."""
        f2 = self.f * self.f
        th = np.asarray(theta, dtype=np.float64).reshape(self.N, 1 + f2)
        return np.exp(th[:, 0]), th[:, 1:].reshape(self.N, self.f, self.f)

    def offsets(self):
        """Tap offsets (da, db) of a filter, row-major over the f x f taps."""
        c = self.f // 2
        return [(a - c, b - c) for a in range(self.f) for b in range(self.f)]

    def responses(self, x, theta):
        lam, ks = self.unpack(theta)
        X = self._img(x)
        return lam, ks, [ops.correlate(X, ks[j]) for j in range(self.N)]

    def phi(self, x, theta) -> float:
        lam, ks, Kx = self.responses(x, theta)
        X = self._img(x)
        res = self.A(X) - self.y
        val = np.sum(res * res) + 0.5 * self.eps * np.sum(X * X)
        for j in range(self.N):
            val += lam[j] * np.sum(self.pen(Kx[j]))
        return float(val)

    def grad(self, x, theta) -> np.ndarray:
        lam, ks, Kx = self.responses(x, theta)
        X = self._img(x)
        g = 2.0 * ops.correlate_adjoint(self.A(X) - self.y, self.kernel) + self.eps * X
        for j in range(self.N):
            g += lam[j] * ops.correlate_adjoint(self.dpen(Kx[j]), ks[j])
        return g.ravel()

    def hvp(self, x, theta, v) -> np.ndarray:
        """H v = 2 A^T A v + eps v + sum_j lambda_j K_j^T (phi''(K_j x) . K_j v)."""
        lam, ks, Kx = self.responses(x, theta)
        V = self._img(v)
        out = 2.0 * ops.correlate_adjoint(ops.correlate(V, self.kernel), self.kernel) + self.eps * V
        for j in range(self.N):
            out += lam[j] * ops.correlate_adjoint(self.ddpen(Kx[j]) * ops.correlate(V, ks[j]), ks[j])
        return out.ravel()

    def dtheta_grad(self, x, theta) -> np.ndarray:
        """n x p matrix D_theta grad_x Phi, column by column.

        d/dw_j:    lambda_j K_j^T phi'(K_j x)
        d/dk_j[a]: lambda_j (S_a^T phi'(K_j x) + K_j^T (phi''(K_j x) . S_a x)),  (S_a x)_i = x_{i+a}.
        """
        lam, ks, Kx = self.responses(x, theta)
        X = self._img(x)
        cols = []
        for j in range(self.N):
            d1, d2 = self.dpen(Kx[j]), self.ddpen(Kx[j])
            cols.append(lam[j] * ops.correlate_adjoint(d1, ks[j]).ravel())
            for (da, db) in self.offsets():
                col = ops.shift(d1, -da, -db) + ops.correlate_adjoint(d2 * ops.shift(X, da, db), ks[j])
                cols.append(lam[j] * col.ravel())
        return np.stack(cols, axis=1)

    def jac_apply(self, x, theta, w, project: bool = True) -> np.ndarray:
        """J w = -(D_theta grad_x Phi)^T w as inner products:

        [J w]_{w_j}    = -lambda_j <phi'(K_j x), K_j w>
        [J w]_{k_j[a]} = -lambda_j (<phi'(K_j x), S_a w> + <phi''(K_j x) . K_j w, S_a x>)
        then (``project``) each filter's tap block minus its mean.
        """
        lam, ks, Kx = self.responses(x, theta)
        X, Wm = self._img(x), self._img(w)
        out = []
        for j in range(self.N):
            d1, d2 = self.dpen(Kx[j]), self.ddpen(Kx[j])
            Kw = ops.correlate(Wm, ks[j])
            out.append(-lam[j] * np.sum(d1 * Kw))
            taps = np.array([-lam[j] * (np.sum(d1 * ops.shift(Wm, da, db)) + np.sum(d2 * Kw * ops.shift(X, da, db)))
                             for (da, db) in self.offsets()])
            if project:
                taps = taps - taps.mean()
            out.extend(taps.tolist())
        return np.array(out)

    def dense_hessian(self, x, theta) -> np.ndarray:
        lam, ks, Kx = self.responses(x, theta)
        Am = ops.dense_correlation(self.h, self.w, self.kernel)
        Hm = 2.0 * Am.T @ Am + self.eps * np.eye(self.n)
        for j in range(self.N):
            Km = ops.dense_correlation(self.h, self.w, ks[j])
            Hm += lam[j] * Km.T @ np.diag(self.ddpen(Kx[j]).ravel()) @ Km
        return Hm


def project_zero_mean(theta_grad: np.ndarray, n_filters: int, fsize: int) -> np.ndarray:
    """Subtract from each filter's tap block of a p-vector its mean (weights untouched)."""
    f2 = fsize * fsize
    g = np.array(theta_grad, dtype=np.float64).reshape(n_filters, 1 + f2)
    g[:, 1:] -= g[:, 1:].mean(axis=1, keepdims=True)
    return g.ravel()


def make_problem(wl, xstar, e, penalty: str = "log"):
    """Problem of a synthetic workload: y = A x* + noise * e formed with the oracle's own blur."""
    y = ops.blur(np.asarray(xstar, dtype=np.float64), wl.blur_radius, wl.blur_sigma) + wl.noise * np.asarray(e)
    if wl.reg == "tv":
        return TVProblem(wl.h, wl.w, wl.blur_radius, wl.blur_sigma, y)
    return FilterProblem(wl.h, wl.w, wl.blur_radius, wl.blur_sigma, y, wl.n_filters, wl.filter_size, wl.eps,
                         penalty)


def upper_loss(x, xstar) -> float:
    """l(x) = 1/2 ||x - x*||^2 (Section 2.1)."""
    d = np.asarray(x).ravel() - np.asarray(xstar).ravel()
    return 0.5 * float(d @ d)
