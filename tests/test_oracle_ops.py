"""Pins of the oracle's forward operators against closed forms and SciPy's correlation."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ops


@pytest.mark.parametrize("r,sigma", [(2, 1.5), (4, 2.5), (5, 3.0)])
def test_gaussian_kernel_closed_form(r, sigma):
    k = ops.gaussian_kernel(r, sigma)
    assert k.shape == (2 * r + 1, 2 * r + 1)
    assert abs(k.sum() - 1.0) < 1e-15
    # entry ratio fixed by exp(-(a^2+b^2)/(2 sigma^2))
    for a, b in [(1, 0), (2, 1), (r, r)]:
        ratio = k[r + a, r + b] / k[r, r]
        assert abs(ratio - np.exp(-(a * a + b * b) / (2 * sigma * sigma))) < 1e-14
    # separable: rank one
    assert np.linalg.matrix_rank(k, tol=1e-14) == 1


@pytest.mark.parametrize("shape", [(7, 9), (16, 16), (5, 13)])
def test_correlate_matches_scipy(shape):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(shape)
    k = rng.standard_normal((7, 7))
    ref = ndimage.correlate(x, k, mode="constant", cval=0.0)
    assert np.abs(ops.correlate(x, k) - ref).max() < 1e-13
    ref_blur = ndimage.correlate(x, ops.gaussian_kernel(2, 1.5), mode="constant", cval=0.0)
    assert np.abs(ops.blur(x, 2, 1.5) - ref_blur).max() < 1e-14


def test_blur_matrix_symmetric_and_adjoints():
    h, w = 6, 7
    A = ops.dense_correlation(h, w, ops.gaussian_kernel(2, 1.5))
    assert np.abs(A - A.T).max() == 0.0
    rng = np.random.default_rng(1)
    k = rng.standard_normal((5, 5))
    K = ops.dense_correlation(h, w, k)
    for _ in range(3):
        x = rng.standard_normal((h, w))
        y = rng.standard_normal((h, w))
        assert np.abs(ops.correlate(x, k).ravel() - K @ x.ravel()).max() < 1e-13
        assert np.abs(ops.correlate_adjoint(y, k).ravel() - K.T @ y.ravel()).max() < 1e-13


def test_forward_differences():
    h, w = 5, 6
    rng = np.random.default_rng(2)
    x = rng.standard_normal((h, w))
    a, b = ops.grad_fwd(x)
    # explicit definition
    for i in range(h):
        for j in range(w):
            ea = x[i, j + 1] - x[i, j] if j < w - 1 else 0.0
            eb = x[i + 1, j] - x[i, j] if i < h - 1 else 0.0
            assert a[i, j] == ea and b[i, j] == eb
    Dm = ops.dense_grad_fwd(h, w)
    assert np.abs(Dm @ x.ravel() - np.concatenate([a.ravel(), b.ravel()])).max() < 1e-14
    p, q = rng.standard_normal((h, w)), rng.standard_normal((h, w))
    p[:, -1] = 0.0
    q[-1, :] = 0.0
    assert np.abs(ops.grad_fwd_adjoint(p, q).ravel() - Dm.T @ np.concatenate([p.ravel(), q.ravel()])).max() < 1e-14
    # constants are in the kernel of D
    a0, b0 = ops.grad_fwd(np.full((h, w), 3.0))
    assert not a0.any() and not b0.any()
