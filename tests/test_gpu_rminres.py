"""GPU parity of RMINRES (Section 2.2.2, Algorithm 3) against the FP64 oracle.

Tolerances: iterates after the same number of steps 1e-10 relative (the GPU sums in another
order and keeps the Appendix A residual in its one-vector form); converged solves: iteration
counts within max(2, 1%), solutions 1e-7 relative (both stop at a 1e-9 residual) and the true
residual within twice the tolerance; the error estimate 1e-9 relative.  Indefinite Hessians: both reach the tolerance, H w = g checked by the
oracle's operator.
"""
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


def tv_case(h, w, seed, r=2, sigma=1.5, noise_x=0.05):
    wl = synth.custom("t", h, "tv", 8, width=w, blur_radius=r, blur_sigma=sigma, rect_min=2, rect_max=6, seed=seed)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xh = inst["xstar"].ravel() + noise_x * synth.unit_noise(prob.n, seed + 1)
    return wl, inst, prob, xh


def upload_recycle(S, rs):
    s = rs["U"].shape[1]
    S.U[:s] = dev(rs["U"].T)
    S.Cm[:s] = dev(rs["C"].T)
    S.Z[:s] = dev(rs["Z"].T)
    S.mu[:s] = dev(rs["mu"])
    S.rs.s_cur = s


def tv_recycled(h, w, seed, s=6):
    wl, inst, prob, xh = tv_case(h, w, seed)
    th = inst["theta0"]
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    first = krylov.cg(hvp, g, tol=1e-6, v_cap=24)
    rs = recycle.refresh(hvp, lambda v: prob.jac_apply(xh, th, v), None, first["V"], s=s)
    return wl, inst, prob, xh, th, g, hvp, rs


@pytest.mark.parametrize("shape", [(37, 75), (64, 64)])
def test_plain_fixed_steps(B, shape):
    """U empty: the iterate after k steps (ragged tiles on 37 x 75)."""
    wl, inst, prob, xh = tv_case(*shape, seed=71)
    th = inst["theta0"]
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    w0 = 0.1 * synth.unit_noise(prob.n, 72)
    with B.Session(B.problem_from(wl), s_max=2, v_cap=8) as S:
        for k in (1, 2, 3, 9, 30):
            ref = rminres.rminres(hvp, g, w0, tol=0.0, max_iter=k)
            w = dev(w0)
            st = S.solve(th, dev(xh), dev(g), w, tol=0.0, max_iter=k, store_basis=False, recycle=False,
                         method="rminres", allow=(B.BL_E_NOT_CONVERGED,))
            assert st.iters == k and st.status == B.BL_E_NOT_CONVERGED
            assert rel(host(w), ref["w"]) <= 1e-10, k
            assert abs(st.res_norm - ref["res_norm"]) <= 1e-9 * ref["res_norm"]


def test_recycled_fixed_steps_and_estimate(B):
    """s = 6 recycle space from the oracle's refresh: iterates and the error estimate."""
    wl, inst, prob, xh, th, g, hvp, rs = tv_recycled(40, 52, seed=73)
    with B.Session(B.problem_from(wl), s_max=6, v_cap=24) as S:
        upload_recycle(S, rs)
        for k in (1, 2, 5, 17):
            ref = rminres.rminres(hvp, g, None, rs["U"], rs["C"], rs["Z"], rs["mu"], tol=0.0, max_iter=k,
                                  stop="hgerr", hg_tol=0.0, record=True)
            w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
            st = S.solve(th, dev(xh), dev(g), w, tol=0.0, max_iter=k, stop="hgerr", hg_tol=0.0, check_every=1,
                         store_basis=False, method="rminres", allow=(B.BL_E_NOT_CONVERGED,))
            assert st.iters == k
            assert rel(host(w), ref["w"]) <= 1e-10, k
            want = ref["hist_nsc"][k]
            assert abs(st.est - want) <= 1e-9 * want, (k, st.est, want)
            assert abs(st.res0_norm - ref["hist_res"][0]) <= 1e-12 * ref["hist_res"][0]


@pytest.mark.parametrize("stop,every", [("resid", 1), ("resid", 4), ("hgerr", 1), ("hgerr", 3)])
def test_recycled_converged(B, stop, every):
    wl, inst, prob, xh, th, g, hvp, rs = tv_recycled(48, 40, seed=75)
    kw = dict(tol=1e-9, stop=stop, hg_tol=1e-7, check_every=every)
    ref = rminres.rminres(hvp, g, None, rs["U"], rs["C"], rs["Z"], rs["mu"], **kw)
    assert ref["status"] == rminres.OK
    with B.Session(B.problem_from(wl), s_max=6, v_cap=24) as S:
        upload_recycle(S, rs)
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), w, store_basis=False, method="rminres", **kw)
        assert st.status == B.BL_OK and st.iters % every == 0
        if stop == "resid":
            assert abs(st.iters - ref["iters"]) <= max(2, ref["iters"] // 100)
            assert rel(host(w), ref["w"]) <= 1e-7
            assert np.linalg.norm(g - hvp(host(w))) <= 2e-9 * np.linalg.norm(g)
            return
        # the estimate is far from monotone, so its first passing iterate is rounding-sensitive:
        # the GPU stops inside the spread of the oracle's stopping iterates under one-ulp
        # perturbations of g, meets the test, and its hypergradient is as good as those runs'
        runs = [rminres.rminres(hvp, g * (1 + 2.0 ** -52 * synth.unit_noise(prob.n, 300 + k)), None, rs["U"],
                                rs["C"], rs["Z"], rs["mu"], **kw) for k in range(4)] + [ref]
        spread = [r_["iters"] for r_ in runs]
        lo, hi = min(spread), max(spread)
        assert lo - max(2 * every, hi - lo) <= st.iters <= hi + max(2 * every, hi - lo), (st.iters, spread)
        assert st.est <= kw["hg_tol"]
        wstar, _ = krylov.reference_solve(hvp, g)
        hg_star = prob.jac_apply(xh, th, wstar)
        worst = max(rel(prob.jac_apply(xh, th, r_["w"]), hg_star) for r_ in runs)
        assert rel(prob.jac_apply(xh, th, host(w)), hg_star) <= 10 * worst + 1e-12


def test_indefinite_filters_solved(B):
    """Filters at a point with large responses make H indefinite: CG stops with
    BL_E_INDEFINITE, RMINRES reaches the tolerance like the oracle."""
    wl = synth.custom("f", 24, "filters", 8, rect_min=2, rect_max=6, seed=111)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"].copy()
    f2 = wl.filter_size ** 2
    for j in range(wl.n_filters):
        th[j * (1 + f2)] = np.log(50.0)
    x = 8.0 * synth.unit_noise(prob.n, 112)
    g = synth.unit_noise(prob.n, 113)
    hvp = lambda v: prob.hvp(x, th, v)
    ref = rminres.rminres(hvp, g, tol=1e-9, max_iter=3000)
    assert ref["status"] == rminres.OK
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=2, v_cap=4) as S:
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(x), dev(g), w, tol=1e-9, max_iter=3000, store_basis=False,
                     allow=(B.BL_E_INDEFINITE,))
        assert st.status == B.BL_E_INDEFINITE
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(x), dev(g), w, tol=1e-9, max_iter=3000, store_basis=False, method="rminres")
        assert st.status == B.BL_OK
        assert abs(st.iters - ref["iters"]) <= max(3, ref["iters"] // 50)
        wh = host(w)
        assert np.linalg.norm(g - hvp(wh)) <= 2e-9 * np.linalg.norm(g)
        assert rel(wh, ref["w"]) <= 1e-6


def test_folded_records(B):
    """384 x 384 with s = 20: the apply records (576 tiles x 21 values) and the update records
    with Z^T r (576 blocks x 21) go through the fold; fixed steps against the oracle."""
    wl, inst, prob, xh = tv_case(384, 384, seed=77)
    th = inst["theta0"]
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    rng = np.random.default_rng(78)
    s = 20
    Ut = rng.standard_normal((prob.n, s))
    HU = np.stack([hvp(Ut[:, j]) for j in range(s)], axis=1)
    Cq, Rc = np.linalg.qr(HU)
    U = np.linalg.solve(Rc.T, Ut.T).T          # U = U~ R^{-1}
    Z = np.linalg.qr(rng.standard_normal((prob.n, s)))[0]
    mu = np.geomspace(1.0, 1e-3, s)
    rs = {"U": U, "C": Cq, "Z": Z, "mu": mu}
    k = 10
    ref = rminres.rminres(hvp, g, None, U, Cq, Z, mu, tol=0.0, max_iter=k, stop="hgerr", hg_tol=0.0, record=True)
    with B.Session(B.problem_from(wl), s_max=20, v_cap=4) as S:
        upload_recycle(S, rs)
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), w, tol=0.0, max_iter=k, stop="hgerr", hg_tol=0.0, check_every=2,
                     store_basis=False, method="rminres", allow=(B.BL_E_NOT_CONVERGED,))
        assert 576 * (1 + s) > 8192
        assert st.iters == k
        assert rel(host(w), ref["w"]) <= 1e-10
        want = ref["hist_nsc"][k]
        assert abs(st.est - want) <= 1e-9 * want


def test_basis_and_edge_cases(B):
    wl, inst, prob, xh = tv_case(33, 40, seed=79)
    th = inst["theta0"]
    g = xh - inst["xstar"].ravel()
    P = B.problem_from(wl)
    with B.Session(P, s_max=2, v_cap=6) as S:
        # stored Lanczos vectors are orthonormal
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), w, tol=1e-8, method="rminres")
        assert st.status == B.BL_OK and st.iters > 6 and S.rs.v_cur == 6
        V = host(S.V[:6]).T
        assert np.abs(V.T @ V - np.eye(6)).max() <= 1e-10
        # zero right-hand side: zero steps, w stays 0
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), torch.zeros_like(w), w, tol=1e-8, store_basis=False, method="rminres")
        assert st.iters == 0 and st.status == B.BL_OK and float(w.abs().max()) == 0.0
        # no steps allowed
        st = S.solve(th, dev(xh), dev(g), w, tol=1e-8, max_iter=0, store_basis=False, method="rminres",
                     allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == 0 and st.status == B.BL_E_NOT_CONVERGED
    # mixed precision is refused
    Pm = B.problem_from(wl, prec="mixed")
    with B.Session(Pm, s_max=2, v_cap=6) as S:
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        with pytest.raises(B.BLError):
            S.solve(th, dev(xh), dev(g), w, tol=1e-8, store_basis=False, method="rminres")
