"""GPU parity of deflated CG (the O5 alternative: Saad, Yeung, Erhel and Guyomarc'h 2000, with the
refresh's U and C = H U as deflation space) against the oracle's deflated_cg: iterates after a
fixed number of steps (1e-10), the error estimate on tested iterations (1e-9), converged
solves (iteration counts within one, solution to the solve's accuracy), the record folds of a
384 x 384 image, plain CG when the space is empty, and the refusals (mixed precision, U^T C
not positive definite)."""
import numpy as np
import pytest

import synth
from oracle import krylov, problem, recycle

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


def case(reg, h, w, seed, s=6):
    if reg == "tv":
        wl = synth.custom("t", h, "tv", s, width=w, blur_radius=2, blur_sigma=1.5, rect_min=3, rect_max=8, seed=seed)
    else:
        wl = synth.custom("f", h, "filters", s, width=w, rect_min=3, rect_max=8, seed=seed)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xs = inst["xstar"].ravel()
    xh = (xs + 0.05 * synth.unit_noise(prob.n, seed + 1)) if reg == "tv" else (0.2 * xs + 0.01 * synth.unit_noise(prob.n, seed + 1))
    th = inst["theta0"]
    hvp = lambda v: prob.hvp(xh, th, v)
    first = krylov.cg(hvp, xh - xs, tol=1e-8, v_cap=20)
    rs = recycle.refresh(hvp, lambda v: prob.jac_apply(xh, th, v), None, first["V"], s=s)
    return wl, prob, xh, th, xs, hvp, rs


def upload(S, rs):
    s = rs["U"].shape[1]
    S.U[:s] = dev(rs["U"].T)
    S.Cm[:s] = dev(rs["C"].T)
    S.Z[:s] = dev(rs["Z"].T)
    S.mu[:s] = dev(rs["mu"])
    S.rs.s_cur = s


@pytest.mark.parametrize("reg,h,w,stop", [("tv", 40, 52, "resid"), ("tv", 40, 52, "hgerr"), ("filters", 36, 40, "resid")])
def test_deflated_fixed_steps(B, reg, h, w, stop):
    wl, prob, xh, th, xs, hvp, rs = case(reg, h, w, 201)
    g = xh - xs
    w0 = 0.3 * synth.unit_noise(prob.n, 202)
    k = 20
    ref = krylov.deflated_cg(hvp, g, w0, rs["U"], rs["C"], rs["Z"], rs["mu"], tol=0.0, stop=stop, hg_tol=0.0,
                             max_iter=k, check_every=4, record=True)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=24) as S:
        upload(S, rs)
        wd = dev(w0)
        st = S.solve(th, dev(xh), dev(g), wd, tol=0.0, stop=stop, hg_tol=0.0, max_iter=k, check_every=4,
                     store_basis=True, method="deflated", allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == k and st.status == B.BL_E_NOT_CONVERGED
        assert rel(host(wd), ref["w"]) <= 1e-10
        assert rel(host(S.V[:k]).T, ref["V"]) <= 1e-10
        assert S.rs.v_cur == k and S.rs.v_lz == 0
        if stop == "hgerr":
            assert abs(st.est - ref["hist_nsc"][k]) <= 1e-9 * ref["hist_nsc"][0]


@pytest.mark.parametrize("reg,h,w", [("tv", 40, 52), ("filters", 36, 40)])
def test_deflated_converged(B, reg, h, w):
    wl, prob, xh, th, xs, hvp, rs = case(reg, h, w, 211)
    g = xh - xs
    ref = krylov.deflated_cg(hvp, g, None, rs["U"], rs["C"], tol=1e-10)
    wref, _ = krylov.reference_solve(hvp, g)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=8) as S:
        upload(S, rs)
        wd = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), wd, tol=1e-10, store_basis=False, method="deflated")
        assert st.status == B.BL_OK and abs(st.iters - ref["iters"]) <= 1
        assert rel(host(wd), wref) <= 1e-7
        assert rel(S.hypergradient(th, dev(xh), wd), prob.jac_apply(xh, th, wref)) <= 1e-7


def test_deflated_folded_records_384(B):
    """384 x 384 (576 pixel blocks): update records of 1 + 20 + 20 values are folded before use."""
    wl, prob, xh, th, xs, hvp, _ = case("tv", 384, 384, 221, s=20)
    rng = np.random.default_rng(222)
    s = 20
    Ut = rng.standard_normal((prob.n, s))
    Cq, Rc = np.linalg.qr(np.stack([hvp(Ut[:, j]) for j in range(s)], axis=1))
    U = np.linalg.solve(Rc.T, Ut.T).T
    Z = np.linalg.qr(rng.standard_normal((prob.n, s)))[0]
    mu = np.geomspace(1.0, 1e-2, s)
    g = xh - xs
    k = 8
    ref = krylov.deflated_cg(hvp, g, None, U, Cq, Z, mu, tol=0.0, stop="hgerr", hg_tol=0.0, max_iter=k, record=True)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=s, v_cap=4) as S:
        S.U[:s] = dev(U.T)
        S.Cm[:s] = dev(Cq.T)
        S.Z[:s] = dev(Z.T)
        S.mu[:s] = dev(mu)
        S.rs.s_cur = s
        wd = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), wd, tol=0.0, stop="hgerr", hg_tol=0.0, max_iter=k, store_basis=False,
                     method="deflated", allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == k
        assert rel(host(wd), ref["w"]) <= 1e-10
        assert abs(st.est - ref["hist_nsc"][k]) <= 1e-9 * ref["hist_nsc"][0]


def test_deflated_empty_space_and_refusals(B):
    wl, prob, xh, th, xs, hvp, rs = case("tv", 24, 30, 231)
    g = xh - xs
    ref = krylov.cg(hvp, g, tol=0.0, max_iter=15)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=8) as S:
        wd = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), wd, tol=0.0, max_iter=15, store_basis=False, recycle=False,
                     method="deflated", allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == 15 and rel(host(wd), ref["w"]) <= 1e-10
        # U^T C not positive definite (U = -U flips its sign): refused before any iteration
        upload(S, rs)
        S.U[:6] = -S.U[:6]
        wd.zero_()
        with pytest.raises(B.BLError) as e:
            S.solve(th, dev(xh), dev(g), wd, tol=1e-8, method="deflated")
        assert e.value.status == B.BL_E_INDEFINITE
    with B.Session(B.problem_from(wl, prec="mixed"), s_max=6, v_cap=8) as S:
        wd = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        with pytest.raises(B.BLError) as e:
            S.solve(th, dev(xh), dev(g), wd, tol=1e-8, method="deflated")
        assert e.value.status == B.BL_E_ARG
