"""Forward operators of the deblurring problems (eq. var-reg and eq. ll2ex), FP64.

Images are h x w arrays, row-major; vectors of length n = h*w are their ravel().

* ``A``: same-size correlation with the normalised Gaussian kernel
  ``k[a,b] = g[a] g[b] / (sum g)^2``, ``g[a] = exp(-a^2 / (2 sigma^2))``, |a|,|b| <= r,
  zero outside the image.  The kernel is symmetric, so ``A`` is a symmetric matrix.
* ``D``: forward differences (horizontal, vertical); the difference that would
  leave the image (last column / last row) is zero.
* ``K``: same-size correlation with a small filter, zero outside the image
  (the paper's "convolution" in eq. ll2ex, read as a correlation).

All operators are written as sums of shifted copies so that each can be checked
by eye against its definition; dense matrices built element by element from the
same definitions serve the pins.
"""
from __future__ import annotations

import numpy as np


def shift(x: np.ndarray, dr: int, dc: int) -> np.ndarray:
    """``z[i, j] = x[i + dr, j + dc]`` where that index is inside the image, else 0."""
    h, w = x.shape
    z = np.zeros_like(x)
    r0, r1 = max(0, -dr), min(h, h - dr)
    c0, c1 = max(0, -dc), min(w, w - dc)
    if r0 < r1 and c0 < c1:
        z[r0:r1, c0:c1] = x[r0 + dr:r1 + dr, c0 + dc:c1 + dc]
    return z


def gaussian_kernel(radius: int, sigma: float) -> np.ndarray:
    """(2r+1) x (2r+1) normalised Gaussian kernel (sums to one)."""
    a = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-a * a / (2.0 * sigma * sigma))
    return np.outer(g, g) / (g.sum() ** 2)


def correlate(x: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Same-size zero-padded correlation ``sum_{a,b} k[a,b] x[i+a-c, j+b-c]`` (k odd-sized, centre c)."""
    c = k.shape[0] // 2
    out = np.zeros_like(x)
    for a in range(k.shape[0]):
        for b in range(k.shape[1]):
            if k[a, b] != 0.0:
                out += k[a, b] * shift(x, a - c, b - c)
    return out


def correlate_adjoint(y: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Adjoint of :func:`correlate`: ``sum_{a,b} k[a,b] y[i-(a-c), j-(b-c)]`` (zero outside)."""
    c = k.shape[0] // 2
    out = np.zeros_like(y)
    for a in range(k.shape[0]):
        for b in range(k.shape[1]):
            if k[a, b] != 0.0:
                out += k[a, b] * shift(y, c - a, c - b)
    return out


def blur(x: np.ndarray, radius: int, sigma: float) -> np.ndarray:
    """``A x``."""
    return correlate(x, gaussian_kernel(radius, sigma))


def grad_fwd(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """``D x = (a, b)``: a = x[i, j+1] - x[i, j] (0 on the last column), b = x[i+1, j] - x[i, j] (0 on the last row)."""
    a = shift(x, 0, 1) - x
    a[:, -1] = 0.0
    b = shift(x, 1, 0) - x
    b[-1, :] = 0.0
    return a, b


def grad_fwd_adjoint(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """``D^T (a, b)``; entries of a on the last column and of b on the last row are ignored."""
    am = a.copy()
    am[:, -1] = 0.0
    bm = b.copy()
    bm[-1, :] = 0.0
    return (shift(am, 0, -1) - am) + (shift(bm, -1, 0) - bm)


# ---------------------------------------------------------------- dense forms (pins, tiny images only)

def dense_correlation(h: int, w: int, k: np.ndarray) -> np.ndarray:
    """n x n matrix of :func:`correlate`, written entry by entry from its definition."""
    n = h * w
    c = k.shape[0] // 2
    M = np.zeros((n, n))
    for i in range(h):
        for j in range(w):
            for a in range(k.shape[0]):
                for b in range(k.shape[1]):
                    ii, jj = i + a - c, j + b - c
                    if 0 <= ii < h and 0 <= jj < w:
                        M[i * w + j, ii * w + jj] += k[a, b]
    return M


def dense_grad_fwd(h: int, w: int) -> np.ndarray:
    """2n x n matrix of :func:`grad_fwd` (rows 0..n-1: horizontal, n..2n-1: vertical)."""
    n = h * w
    Dm = np.zeros((2 * n, n))
    for i in range(h):
        for j in range(w):
            p = i * w + j
            if j < w - 1:
                Dm[p, p] = -1.0
                Dm[p, p + 1] = 1.0
            if i < h - 1:
                Dm[n + p, p] = -1.0
                Dm[n + p, p + w] = 1.0
    return Dm
