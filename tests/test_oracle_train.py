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
from oracle import problem, upper


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
