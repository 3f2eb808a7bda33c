"""GPU parity of the recycle-space selections (Table 2) against the FP64 oracle: the refresh
from a stored Krylov basis with each rule gives the oracle's subspace (principal angles 1e-8),
C = H U with C^T C = I, and for the RGen sides the oracle's mu and Z.  On an indefinite Hessian
(filters away from the minimiser) the Ritz and harmonic Ritz rules work where RGen's projected
Cholesky fails, and RMINRES recycles the result."""
import numpy as np
import pytest

import synth
from oracle import krylov, problem, recycle, rminres

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08264_amd import bilevel
    return bilevel


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def tv_basis():
    wl = synth.custom("t", 48, "tv", 6, width=40, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=6, seed=61)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xh = inst["xstar"].ravel() + 0.05 * synth.unit_noise(prob.n, 62)
    th = inst["theta0"]
    g = xh - inst["xstar"].ravel()
    first = krylov.cg(lambda v: prob.hvp(xh, th, v), g, tol=1e-8, v_cap=24)
    return wl, prob, xh, th, first["V"]


@pytest.mark.parametrize("rule", list(recycle.SELECTIONS))
def test_refresh_every_selection(B, tv_basis, rule):
    wl, prob, xh, th, V = tv_basis
    hvp = lambda v: prob.hvp(xh, th, v)
    ref = recycle.refresh(hvp, lambda v: prob.jac_apply(xh, th, v), None, V, s=6, select_rule=rule)
    with B.Session(B.problem_from(wl), s_max=6, v_cap=24) as S:
        m = V.shape[1]
        S.V[:m] = dev(V.T)
        S.rs.v_cur = m
        st = S.refresh(th, dev(xh), s=6, select=rule)
        assert S.rs.s_cur == 6 and st.t == ref["t"]
        U = host(S.U[:6]).T
        C = host(S.Cm[:6]).T
        assert recycle.principal_angles(U, ref["U"]).max() <= 1e-8, rule
        assert np.abs(C.T @ C - np.eye(6)).max() <= 1e-13
        HU = np.stack([hvp(U[:, j]) for j in range(6)], axis=1)
        assert np.linalg.norm(HU - C) <= 1e-11 * np.linalg.norm(C)
        mu = host(S.mu[:6])
        if rule.startswith("rgen"):
            assert np.abs(mu[:2] - ref["mu"][:2]).max() <= 1e-10 * ref["mu"][0]
            Z = host(S.Z[:6]).T
            assert recycle.principal_angles(Z[:, :2], ref["Z"][:, :2]).max() <= 1e-8
        else:
            assert np.all(mu == 0.0) and float(S.Z[:6].abs().max()) == 0.0


@pytest.mark.parametrize("rule", ["ritz-s", "hritz-l"])
def test_indefinite_selection_then_rminres(B, rule):
    wl = synth.custom("f", 24, "filters", 6, rect_min=2, rect_max=6, seed=111)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"].copy()
    f2 = wl.filter_size ** 2
    for j in range(wl.n_filters):
        th[j * (1 + f2)] = np.log(50.0)
    x = 8.0 * synth.unit_noise(prob.n, 112)
    g = synth.unit_noise(prob.n, 113)
    hvp = lambda v: prob.hvp(x, th, v)
    V = np.linalg.qr(np.random.default_rng(114).standard_normal((prob.n, 20)))[0]
    ref = recycle.refresh(hvp, lambda v: prob.jac_apply(x, th, v), None, V, s=6, select_rule=rule)
    k = 12
    ref_s = rminres.rminres(hvp, g, None, ref["U"], ref["C"], tol=0.0, max_iter=k)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=20) as S:
        S.V[:20] = dev(V.T)
        S.rs.v_cur = 20
        with pytest.raises(B.BLError):
            S.refresh(th, dev(x), s=6)            # RGen: W^T H W is indefinite
        S.rs.v_cur = 20
        S.refresh(th, dev(x), s=6, select=rule)
        assert S.rs.s_cur == 6
        U = host(S.U[:6]).T
        assert recycle.principal_angles(U, ref["U"]).max() <= 1e-8
        # RMINRES with the GPU's own recycle space against the oracle's with the same space
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(x), dev(g), w, tol=0.0, max_iter=k, store_basis=False, method="rminres",
                     allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == k
        assert rel(host(w), ref_s["w"]) <= 1e-8


@pytest.mark.parametrize("rule", list(recycle.SELECTIONS_FULL_RANK))
def test_refresh_rgen_small_and_mixed_filters(B, rule):
    """Filters (p = 400 >= t): RGen of sizes S and M, every side, against the oracle."""
    wl = synth.custom("f", 40, "filters", 8, width=44, rect_min=2, rect_max=6, seed=71)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xh = inst["xstar"].ravel() + 0.02 * synth.unit_noise(prob.n, 72)
    th = inst["theta0"]
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    first = krylov.cg(hvp, g, tol=1e-8, v_cap=20)
    ref = recycle.refresh(hvp, lambda v: prob.jac_apply(xh, th, v), None, first["V"], s=8, select_rule=rule)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=8, v_cap=20) as S:
        m = first["V"].shape[1]
        S.V[:m] = dev(first["V"].T)
        S.rs.v_cur = m
        S.refresh(th, dev(xh), s=8, select=rule)
        assert S.rs.s_cur == 8
        mu = host(S.mu[:8])
        assert np.abs(np.sort(mu) - np.sort(ref["mu"])).max() <= 1e-9 * ref["mu"].max()
        U = host(S.U[:8]).T
        assert recycle.principal_angles(U, ref["U"]).max() <= 1e-8, rule


def test_rgen_small_refused_for_tv(B, tv_basis):
    wl, prob, xh, th, V = tv_basis
    with B.Session(B.problem_from(wl), s_max=6, v_cap=24) as S:
        m = V.shape[1]
        S.V[:m] = dev(V.T)
        S.rs.v_cur = m
        with pytest.raises(B.BLError):
            S.refresh(th, dev(xh), s=6, select="rgen-s-r")
