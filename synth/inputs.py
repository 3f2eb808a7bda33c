"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method: it draws ground-truth images
(random axis-aligned rectangles on a zero background), standard-normal noise
fields, zero-mean random filters and initial hyperparameters, and it records the
workload recipes.  Applying the blur, forming measurements and everything after
that is done separately by the oracle and by the HIP library.

Rectangle recipe (the paper only says "random rectangles"): for each rectangle
draw two distinct integers in [0, side] for the rows and two for the columns,
sort each pair, and paint the half-open box with a value drawn from U[0, 1];
later rectangles overwrite earlier ones.  Generator: numpy PCG64
(``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    """Recipe of one synthetic deblurring workload."""

    name: str
    h: int
    w: int
    rect_min: int
    rect_max: int
    blur_radius: int
    blur_sigma: float
    noise: float
    seed: int
    reg: str                      # "tv" or "filters"
    s: int                        # recycle dimension
    tol: float                    # relative residual tolerance of the Hessian solve
    outer: int                    # outer (upper-level) iterations of the frozen sequence
    n_filters: int = 0
    filter_size: int = 0
    filter_seed: int = 0
    eps: float = 0.0
    prec: str = "fp64"            # "fp64" or "mixed"
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.h * self.w

    @property
    def p(self) -> int:
        return 2 if self.reg == "tv" else self.n_filters * (1 + self.filter_size ** 2)


TV_THETA0 = (math.log(0.05), math.log(0.01))
FILTER_WEIGHT0 = math.log(0.05)

WORKLOADS = {
    # 32x32 smoothed-TV deblurring, FP64, s=10, tol 1e-10, 20 outer steps.
    "tv32": Workload("tv32", 32, 32, 1, 5, 2, 1.5, 0.01, 1001, "tv", 10, 1e-10, 20),
    # 256x256 smoothed-TV deblurring, FP64, s=20, 30 outer steps.
    "tv256": Workload("tv256", 256, 256, 8, 20, 4, 2.5, 0.01, 2001, "tv", 20, 1e-10, 30),
    # 512x512 eight 7x7 zero-mean filters, log(1+s^2) penalty, mixed precision, s=30, 40 steps.
    "foe512": Workload("foe512", 512, 512, 8, 20, 5, 3.0, 0.02, 3001, "filters", 30, 1e-10, 40,
                       n_filters=8, filter_size=7, filter_seed=3002, eps=1e-6, prec="mixed"),
}


def rectangles(h: int, w: int, n_min: int, n_max: int, rng: np.random.Generator) -> np.ndarray:
    """Ground truth: ``n_min..n_max`` rectangles with U[0,1] values on zeros (h x w, float64)."""
    x = np.zeros((h, w), dtype=np.float64)
    count = int(rng.integers(n_min, n_max + 1))
    for _ in range(count):
        r0, r1 = np.sort(rng.choice(h + 1, size=2, replace=False))
        c0, c1 = np.sort(rng.choice(w + 1, size=2, replace=False))
        x[r0:r1, c0:c1] = rng.uniform(0.0, 1.0)
    return x


def zero_mean_filters(n_filters: int, size: int, rng: np.random.Generator, std: float = 0.1) -> np.ndarray:
    """``n_filters`` filters of ``size x size`` taps drawn N(0, std^2), then made zero-mean."""
    k = rng.normal(0.0, std, size=(n_filters, size, size))
    return k - k.mean(axis=(1, 2), keepdims=True)


def initial_theta(wl: Workload, filters: np.ndarray | None = None) -> np.ndarray:
    """Initial hyperparameters.

    TV: ``(log 0.05, log 0.01)`` = (log weight, log smoothing).
    Filters: interleaved per filter ``[w_1, k_1 (f*f taps, row-major), w_2, k_2, ...]``
    with ``w_j = log 0.05``.
    """
    if wl.reg == "tv":
        return np.array(TV_THETA0, dtype=np.float64)
    f2 = wl.filter_size ** 2
    th = np.empty(wl.n_filters * (1 + f2), dtype=np.float64)
    for j in range(wl.n_filters):
        th[j * (1 + f2)] = FILTER_WEIGHT0
        th[j * (1 + f2) + 1:(j + 1) * (1 + f2)] = filters[j].ravel()
    return th


def instance(wl: Workload, seed: int | None = None) -> dict:
    """Draw one instance: ground truth, unit noise field, filters, initial theta.

    The measurement is ``y = A x* + noise * e``; forming it needs the blur and is
    left to the consumer.
    """
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    xstar = rectangles(wl.h, wl.w, wl.rect_min, wl.rect_max, rng)
    e = rng.standard_normal((wl.h, wl.w))
    filters = None
    if wl.reg == "filters":
        filters = zero_mean_filters(wl.n_filters, wl.filter_size, np.random.default_rng(wl.filter_seed))
    return {"xstar": xstar, "e": e, "filters": filters, "theta0": initial_theta(wl, filters)}


def unit_noise(shape, seed: int) -> np.ndarray:
    """Standard-normal field with its own seed (stand-in perturbations, random right-hand sides)."""
    return np.random.default_rng(seed).standard_normal(shape)


def batch_sides(count: int, seed: int, sides=(128, 192, 256, 384, 512)) -> list[int]:
    """Image sides of a batched training set, uniform over ``sides``."""
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.choice(np.array(sides), size=count)]


def custom(name: str, side: int, reg: str, s: int, width: int | None = None, **kw) -> Workload:
    """A ``side x width`` workload with the blur/noise recipe of the TV or filter family."""
    if reg == "tv":
        base = dict(rect_min=8, rect_max=20, blur_radius=4, blur_sigma=2.5, noise=0.01, tol=1e-10)
    else:
        base = dict(rect_min=8, rect_max=20, blur_radius=5, blur_sigma=3.0, noise=0.02, tol=1e-10,
                    n_filters=8, filter_size=7, filter_seed=3002, eps=1e-6)
    base.update(kw)
    seed = base.pop("seed", 7000 + side)
    outer = base.pop("outer", 8)
    return Workload(name, side, side if width is None else width, base.pop("rect_min"), base.pop("rect_max"), base.pop("blur_radius"),
                    base.pop("blur_sigma"), base.pop("noise"), seed, reg, s, base.pop("tol"), outer, **base)


def batch_set(count: int = 64, seed: int = 4000, s: int = 20) -> list[Workload]:
    """Batched training set: ``count`` images whose sides are uniform over {128, ..., 512}
    (drawn with ``seed``), rectangles 8-20, the filter family's blur (11x11, sigma 3), noise 0.02
    and its eight 7x7 filters (shared theta: one filter seed for all), recycle dimension s.
    Image k draws its rectangles and noise with seed ``seed + 1 + k``."""
    sides = batch_sides(count, seed)
    return [custom(f"batch{k}", side, "filters", s, seed=seed + 1 + k, prec="mixed")
            for k, side in enumerate(sides)]


SERVE_SIDES = (64, 128, 256, 512, 1024)
SERVE_S = (10, 30, 50)


def serve_samples(count: int = 256, seed: int = 5000) -> list[Workload]:
    """Resident training samples of the served stream: side uniform over SERVE_SIDES, TV (the
    256x256 family's blur and noise) or eight 7x7 filters (the 512x512 family's) with equal
    probability, recycle dimension uniform over SERVE_S.  Sample k draws its image with seed
    ``seed + 1 + k``."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        side = int(rng.choice(np.array(SERVE_SIDES)))
        reg = "tv" if rng.random() < 0.5 else "filters"
        s = int(rng.choice(np.array(SERVE_S)))
        out.append(custom(f"serve{k}", side, reg, s, seed=seed + 1 + k))
    return out


def poisson_arrivals(rate: float, duration: float, count: int, seed: int = 5001) -> list[tuple[float, int]]:
    """Arrival times (seconds) of a Poisson stream of the given rate over ``duration`` seconds,
    each naming a sample drawn uniformly from ``count``."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            return out
        out.append((t, int(rng.integers(count))))


def theta_drift(wl: Workload, steps: int, seed: int, scale: float = 0.02) -> list[np.ndarray]:
    """A frozen outer-step path of hyperparameters for a served sample: theta_0 (the recipe's
    initial value) followed by steps - 1 increments of a seeded normal direction scaled to
    ``scale`` times the norm of theta_0 (filters: the tap increments are made zero-mean per
    filter, as the filter parameterisation requires)."""
    filters = None
    if wl.reg == "filters":
        filters = zero_mean_filters(wl.n_filters, wl.filter_size, np.random.default_rng(wl.filter_seed))
    th = initial_theta(wl, filters)
    rng = np.random.default_rng(seed)
    path = [th.copy()]
    for _ in range(steps - 1):
        d = rng.standard_normal(th.shape)
        if wl.reg == "filters":
            f2 = wl.filter_size ** 2
            for j in range(wl.n_filters):
                blk = d[j * (1 + f2) + 1:(j + 1) * (1 + f2)]
                blk -= blk.mean()
        th = th + scale * np.linalg.norm(path[0]) / np.linalg.norm(d) * d
        path.append(th.copy())
    return path
