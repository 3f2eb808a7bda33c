"""Pins of the oracle's recycle-space selections other than RGen-L(R) (Section 3.1, eqs.
ritz-matrix-decomp and harmonic-ritz; Section 3.2, the sides of the Ritz generalized singular
vectors; Table 2: sizes S, L, M).

* size rule: positions of the kept values;
* Ritz vectors: with W spanning all of R^n they are eigenvectors of H (Eig-S / Eig-L), checked
  against the eigenvectors H was built from; a Galerkin residual orthogonal to range(W);
* harmonic Ritz vectors: the Petrov-Galerkin condition (HW)^T (H x - theta x) = 0; their values
  are the reciprocals of the Ritz values of H^{-1} on range(HW) (formed with an explicit inverse);
  on an invariant subspace they are exact eigenvalues;
* RGen sides: (W V_H)^T H (W X) is diagonal with a positive diagonal (the GSVD diagonalisation);
  the M side bisects the angle between each right vector and its left vector;
* the refresh with every rule keeps C = H U and C^T C = I; non-RGen rules leave mu = 0, Z = 0.
"""
import numpy as np
import pytest

from oracle import recycle


def sym_known(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.asarray(eigs)) @ Q.T, Q


def test_size_rule():
    assert recycle.size_pick(10, 4, "s") == [0, 1, 2, 3]
    assert recycle.size_pick(10, 4, "l") == [9, 8, 7, 6]
    assert recycle.size_pick(10, 4, "m") == [0, 1, 9, 8]
    assert recycle.size_pick(10, 5, "m") == [0, 1, 2, 9, 8]
    assert recycle.size_pick(3, 5, "s") == [0, 1, 2]
    assert recycle.size_pick(3, 5, "m") == [0, 1, 2]


@pytest.mark.parametrize("size", ["s", "l", "m"])
def test_ritz_on_whole_space_are_eigenvectors(size):
    n, s = 14, 4
    eigs = np.geomspace(1.0, 100.0, n)
    H, Q = sym_known(n, eigs, 1)
    sel = recycle.select_ritz(H, s, size)          # W = I: M = H
    want = Q[:, recycle.size_pick(n, s, size)]
    assert recycle.principal_angles(sel["X"], want).max() <= 1e-10
    assert np.allclose(np.sort(sel["values"]), np.sort(eigs[recycle.size_pick(n, s, size)]), rtol=1e-12)


def test_ritz_galerkin_condition():
    n, t = 40, 9
    H, _ = sym_known(n, np.linspace(-2.0, 30.0, n), 2)
    W, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n, t)))
    sel = recycle.select_ritz(W.T @ H @ W, 5, "m")
    for j, th in enumerate(sel["values"]):
        x = W @ sel["X"][:, j]
        assert np.linalg.norm(W.T @ (H @ x - th * x)) <= 1e-12 * np.linalg.norm(H, 2)


@pytest.mark.parametrize("size", ["s", "l", "m"])
def test_harmonic_ritz_petrov_galerkin_and_inverse(size):
    n, t, s = 40, 10, 4
    eigs = np.geomspace(0.5, 80.0, n)
    H, _ = sym_known(n, eigs, 4)
    W, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((n, t)))
    Y = H @ W
    M = 0.5 * (W.T @ Y + Y.T @ W)
    sel = recycle.select_hritz(M, Y.T @ Y, s, size)
    for j, th in enumerate(sel["values"]):
        x = W @ sel["X"][:, j]
        assert np.linalg.norm(Y.T @ (H @ x - th * x)) <= 1e-10 * np.linalg.norm(Y) * np.linalg.norm(x) * eigs[-1]
    # reciprocals of the Ritz values of H^{-1} on range(HW)
    Vq, _ = np.linalg.qr(Y)
    ritz_inv = np.linalg.eigvalsh(Vq.T @ np.linalg.inv(H) @ Vq)
    allv = np.sort(1.0 / ritz_inv)
    want = allv[recycle.size_pick(t, s, size)]
    assert np.allclose(np.sort(sel["values"]), np.sort(want), rtol=1e-9)


def test_harmonic_ritz_exact_on_invariant_subspace():
    n = 30
    eigs = np.linspace(1.0, 20.0, n)
    H, Q = sym_known(n, eigs, 6)
    W = Q[:, [2, 7, 11, 20]]
    Y = H @ W
    sel = recycle.select_hritz(W.T @ Y, Y.T @ Y, 4, "s")
    assert np.allclose(np.sort(sel["values"]), eigs[[2, 7, 11, 20]], rtol=1e-12)


def test_rgen_sides():
    n, t, p, s = 50, 8, 12, 4
    H, _ = sym_known(n, np.geomspace(1.0, 40.0, n), 7)
    rng = np.random.default_rng(8)
    W, _ = np.linalg.qr(rng.standard_normal((n, t)))
    J = rng.standard_normal((p, n))
    M = W.T @ H @ W
    G = J @ W
    right = recycle.select(G, M, None, s, "rgen-l-r")
    left = recycle.select(G, M, None, s, "rgen-l-l")
    mid = recycle.select(G, M, None, s, "rgen-l-m")
    Xr = right["X"] / np.linalg.norm(right["X"], axis=0)
    D = (W @ left["X"]).T @ H @ (W @ Xr)
    assert np.abs(D - np.diag(np.diag(D))).max() <= 1e-12 * np.abs(np.diag(D)).max()
    assert np.all(np.diag(D) > 0)
    for j in range(s):
        xm = mid["X"][:, j] / np.linalg.norm(mid["X"][:, j])
        a = float(xm @ Xr[:, j])
        b = float(xm @ left["X"][:, j])
        assert abs(a - b) <= 1e-13 and a > 0
        # in the span of the pair
        P = np.stack([Xr[:, j], left["X"][:, j]], axis=1)
        assert np.linalg.norm(xm - P @ np.linalg.lstsq(P, xm, rcond=None)[0]) <= 1e-13
    assert np.array_equal(right["mu"], left["mu"]) and np.array_equal(right["V_H"], mid["V_H"])


@pytest.mark.parametrize("rule", recycle.SELECTIONS)
def test_refresh_invariants_every_rule(rule):
    n = 60
    H, _ = sym_known(n, np.geomspace(1.0, 50.0, n), 9)
    rng = np.random.default_rng(10)
    J = rng.standard_normal((6, n))
    V = np.linalg.qr(rng.standard_normal((n, 12)))[0]
    out = recycle.refresh(lambda v: H @ v, lambda v: J @ v, None, V, s=5, select_rule=rule)
    U, C = out["U"], out["C"]
    assert U.shape[1] == 5
    assert np.abs(C.T @ C - np.eye(5)).max() <= 1e-12
    assert np.linalg.norm(H @ U - C) <= 1e-11 * np.linalg.norm(C)
    if not rule.startswith("rgen"):
        assert np.all(out["mu"] == 0.0) and np.all(out["Z"] == 0.0)


@pytest.mark.parametrize("rule", recycle.SELECTIONS_FULL_RANK)
def test_rgen_small_and_mixed_sizes(rule):
    """p >= t: the chosen generalized singular values are the smallest (S) or both ends (M) of
    the full GSVD spectrum, and the chosen pairs still diagonalise the projected Hessian."""
    n, t, p, s = 50, 8, 12, 4
    H, _ = sym_known(n, np.geomspace(1.0, 40.0, n), 11)
    rng = np.random.default_rng(12)
    W, _ = np.linalg.qr(rng.standard_normal((n, t)))
    J = rng.standard_normal((p, n))
    M = W.T @ H @ W
    G = J @ W
    sel = recycle.select(G, M, None, s, rule)
    # generalized singular values: sigma(G M^{-1}) (eq. gritz-decomp), all t positive here
    allmu = np.sort(np.linalg.svd(G @ np.linalg.inv(M), compute_uv=False))
    size = rule.split("-")[1]
    want = allmu[recycle.size_pick(t, s, size)]
    assert np.allclose(np.sort(sel["mu"]), np.sort(want), rtol=1e-10)
    right = recycle.select(G, M, None, s, rule[:-1] + "r")
    Xr = right["X"] / np.linalg.norm(right["X"], axis=0)
    left = recycle.select(G, M, None, s, rule[:-1] + "l")
    D = (W @ left["X"]).T @ H @ (W @ Xr)
    assert np.abs(D - np.diag(np.diag(D))).max() <= 1e-12 * np.abs(np.diag(D)).max()
    assert np.all(np.diag(D) > 0)


def test_rgen_small_needs_full_rank():
    n, t = 40, 10
    H, _ = sym_known(n, np.geomspace(1.0, 20.0, n), 13)
    W, _ = np.linalg.qr(np.random.default_rng(14).standard_normal((n, t)))
    G = np.random.default_rng(15).standard_normal((3, n)) @ W     # p = 3 < t
    with pytest.raises(ValueError):
        recycle.select(G, W.T @ H @ W, None, 4, "rgen-s-r")
