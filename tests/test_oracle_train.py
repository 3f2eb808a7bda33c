"""Pins of the oracle's end-to-end training loop (Algorithm 2 with Algorithm 1's backtracking;
hypergradients from recycled solves).

* with no recycling and tight solves it follows the reference trajectory (hypergradients from
  the 1e-13 reference solve): the same accepted steps and parameters to 1e-7;
* every accepted step meets the Armijo decrease, so the upper loss decreases;
* recycled CG with the error-estimate stop and RMINRES follow the same path to the accuracy of
  their hypergradients.
"""
import numpy as np
import pytest

import synth
from oracle import lbfgs, problem, upper


@pytest.fixture(scope="module")
def case():
    wl = synth.custom("tr", 16, "tv", 4, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=5, seed=31)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    return wl, inst, prob


def test_plain_training_follows_reference_trajectory(case):
    wl, inst, prob = case
    thetas, _ = upper.trajectory(prob, inst["xstar"], inst["theta0"], 4)
    hist = upper.train(prob, inst["xstar"], inst["theta0"], 4, s=0, tol=1e-12)
    for a, b in zip(hist["theta"][:4], thetas):
        assert np.linalg.norm(a - b) <= 1e-7 * np.linalg.norm(b)


@pytest.mark.parametrize("solver,stop", [("cg", "hgerr"), ("rminres", "hgerr"), ("rminres", "resid")])
def test_recycled_training(case, solver, stop):
    wl, inst, prob = case
    plain = upper.train(prob, inst["xstar"], inst["theta0"], 4, s=0, tol=1e-12)
    hist = upper.train(prob, inst["xstar"], inst["theta0"], 4, s=4, solver=solver, stop=stop, tol=1e-10,
                       hg_rel=1e-9)
    # Armijo decrease at every accepted step
    loss = hist["loss"]
    assert all(b < a for a, b in zip(loss, loss[1:]))
    assert all(t > 0 for t in hist["tau"])
    for a, b in zip(hist["theta"], plain["theta"]):
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
    # recycling does not cost iterations over the sequence on this problem
    assert sum(hist["iters"][1:]) <= sum(plain["iters"][1:]) + 4


# ------------------------------------------------------------------ batch training with Adam
@pytest.fixture(scope="module")
def batch_case():
    """Two TV images of different sizes sharing theta (the batched-training setting)."""
    out = []
    for k, (h, w) in enumerate([(16, 14), (12, 18)]):
        wl = synth.custom(f"b{k}", h, "tv", 4, width=w, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=5,
                          seed=41 + k)
        inst = synth.instance(wl)
        out.append((wl, inst, problem.make_problem(wl, inst["xstar"], inst["e"])))
    return out


def test_adam_first_step_is_lr_times_sign_of_summed_hypergradient(batch_case):
    """From m = v = 0, Adam's first step is lr g / (|g| + eps) per component; g is the sum over
    the batch of the images' hypergradients (each from the reference solve)."""
    probs = [c[2] for c in batch_case]
    xstars = [c[1]["xstar"] for c in batch_case]
    th0 = batch_case[0][1]["theta0"]
    hist = upper.train_adam(probs, xstars, th0, 1, lr=1e-2, tol=1e-13)
    g = np.zeros(2)
    for prob, xs in zip(probs, xstars):
        xh, _ = lbfgs.lbfgs(lambda v, p=prob: p.phi(v, th0), lambda v, p=prob: p.grad(v, th0), prob.y.ravel(),
                            gtol=1e-8, max_iter=20000)
        g += upper.hypergradient(prob, xh, th0, xs)[0]
    assert abs(hist["grad_norm"][0] - np.linalg.norm(g)) <= 1e-6 * np.linalg.norm(g)
    step = hist["theta"][0] - hist["theta"][1]
    assert np.allclose(step, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-6, atol=0)


def test_adam_constant_gradient_and_zero_mean_projection():
    """For a constant gradient the bias-corrected moments are g and g^2 at every step, so every
    step is lr g / (|g| + eps); with filter blocks the step keeps each block's taps zero-mean and
    leaves the weights' steps alone."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(2 * 10)
    th = np.zeros_like(g)
    m = v = np.zeros_like(g)
    for t in range(1, 6):
        th_new, m, v = upper.adam_step(th, g, m, v, t, 0.05)
        assert np.allclose(th - th_new, 0.05 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        th = th_new
    th0 = np.zeros_like(g)
    th1, _, _ = upper.adam_step(th0, g, np.zeros_like(g), np.zeros_like(g), 1, 0.05, zero_mean_blocks=(2, 3))
    st = (th0 - th1).reshape(2, 10)
    assert np.abs(st[:, 1:].sum(axis=1)).max() <= 1e-15
    plain = 0.05 * g / (np.abs(g) + 1e-8)
    assert np.allclose(st[:, 0], plain.reshape(2, 10)[:, 0], rtol=1e-15)


def test_recycled_adam_follows_plain(batch_case):
    """Recycled CG (s = 4, error-estimate stop) in Adam training follows the path of tight plain
    solves to the accuracy of the hypergradients."""
    probs = [c[2] for c in batch_case]
    xstars = [c[1]["xstar"] for c in batch_case]
    th0 = batch_case[0][1]["theta0"]
    plain = upper.train_adam(probs, xstars, th0, 3, lr=2e-2, tol=1e-12)
    rec = upper.train_adam(probs, xstars, th0, 3, lr=2e-2, s=4, stop="hgerr", tol=1e-10, hg_rel=1e-9)
    for a, b in zip(rec["theta"], plain["theta"]):
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
    assert rec["loss"][-1] < rec["loss"][0]
