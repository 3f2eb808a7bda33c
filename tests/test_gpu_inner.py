"""GPU parity of the inner refresh (eq. subtle-old; Section 5.1, "Inner versus outer recycling
strategies"): the recycle space for system i from the previous system's Krylov basis, with the
projected matrix W^T H^{(i-1)} W formed from the previous CG solve's coefficients and recycle
space (no products with either Hessian) and only the s selected vectors multiplied by H^{(i)}.
The oracle forms the same matrix from products with the previous Hessian.  Also: a GPU CG solve
records the CG coefficients of its stored residuals as the oracle computes them."""
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


def pair(reg, h, w, seed):
    """Systems i-1 and i of a sequence: nearby reconstructions and hyperparameters."""
    if reg == "tv":
        wl = synth.custom("t", h, "tv", 6, width=w, blur_radius=2, blur_sigma=1.5, rect_min=3, rect_max=8, seed=seed)
    else:
        wl = synth.custom("f", h, "filters", 6, width=w, rect_min=3, rect_max=8, seed=seed)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xs = inst["xstar"].ravel()
    if reg == "tv":
        x0 = xs + 0.05 * synth.unit_noise(prob.n, seed + 1)
        t0 = np.array(inst["theta0"])
        dt = np.array([0.05, -0.03])
    else:   # small responses: phi'' > 0 everywhere, so both Hessians are SPD
        x0 = 0.2 * xs + 0.01 * synth.unit_noise(prob.n, seed + 1)
        t0 = np.array(inst["theta0"])
        dt = 0.01 * synth.unit_noise(t0.size, seed + 3)
    x1 = x0 + 0.01 * synth.unit_noise(prob.n, seed + 2)
    return wl, prob, xs, (x0, t0), (x1, t0 + dt)


def lz_of(res):
    out = np.zeros(2 * len(res["rho"]))
    out[0::2] = res["alpha"]
    out[1::2] = res["rho"]
    return out


@pytest.mark.parametrize("reg,h,w", [("tv", 40, 52), ("filters", 36, 40)])
def test_inner_refresh_parity(B, reg, h, w):
    wl, prob, xs, (x0, t0), (x1, t1) = pair(reg, h, w, 171)
    h0 = lambda v: prob.hvp(x0, t0, v)
    h1 = lambda v: prob.hvp(x1, t1, v)
    first = krylov.cg(h0, x0 - xs, tol=1e-10, v_cap=20)
    rs0 = recycle.refresh(h0, lambda v: prob.jac_apply(x0, t0, v), None, first["V"], s=6)
    prev = krylov.recycled_cg(h0, x0 - xs + 0.1 * synth.unit_noise(prob.n, 9), first["w"], rs0["U"], rs0["C"],
                              tol=1e-12, v_cap=24)
    assert prev["V"].shape[1] == 24
    ref = recycle.refresh(h1, lambda v: prob.jac_apply(x1, t1, v), rs0["U"], prev["V"], s=6, hvp_old=h0)
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=24) as S:
        S.U[:6] = dev(rs0["U"].T)
        S.Cm[:6] = dev(rs0["C"].T)
        S.Z[:6] = dev(rs0["Z"].T)
        S.mu[:6] = dev(rs0["mu"])
        S.rs.s_cur = 6
        S.V[:24] = dev(prev["V"].T)
        S.lz[:48] = dev(lz_of(prev))
        S.rs.v_cur = S.rs.v_lz = 24
        st = S.refresh(t1, dev(x1), s=6, inner=True)
        assert S.rs.s_cur == 6 and st.t == ref["t"]
        k = ref["rank_G"] if reg == "tv" else 6
        mu = host(S.mu[:6])
        assert np.abs(mu[:k] - ref["mu"][:k]).max() <= 1e-8 * ref["mu"][0]
        U = host(S.U[:6]).T
        C = host(S.Cm[:6]).T
        assert recycle.principal_angles(U, ref["U"]).max() <= 1e-6
        assert np.abs(C.T @ C - np.eye(6)).max() <= 1e-13
        HU = np.stack([h1(U[:, j]) for j in range(6)], axis=1)
        assert np.linalg.norm(HU - C) <= 1e-11 * np.linalg.norm(C)
        Z = host(S.Z[:6]).T
        assert recycle.principal_angles(Z[:, :k], ref["Z"][:, :k]).max() <= 1e-6


def test_solve_records_cg_coefficients(B):
    """A recycled CG solve with store_basis writes alpha_j, rho_j of its stored residuals (the
    oracle's to 1e-10) and v_lz = v_cur; the inner refresh then runs on the GPU's own record."""
    wl, prob, xs, (x0, t0), (x1, t1) = pair("tv", 40, 52, 181)
    h0 = lambda v: prob.hvp(x0, t0, v)
    first = krylov.cg(h0, x0 - xs, tol=1e-10, v_cap=20)
    rs0 = recycle.refresh(h0, lambda v: prob.jac_apply(x0, t0, v), None, first["V"], s=6)
    g = x0 - xs
    ref = krylov.recycled_cg(h0, g, None, rs0["U"], rs0["C"], tol=0.0, max_iter=30, v_cap=24,
                             recurrence="single")   # the GPU's FP64 single-reduction form
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=24) as S:
        S.U[:6] = dev(rs0["U"].T)
        S.Cm[:6] = dev(rs0["C"].T)
        S.Z[:6] = dev(rs0["Z"].T)
        S.mu[:6] = dev(rs0["mu"])
        S.rs.s_cur = 6
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(t0, dev(x0), dev(g), w, tol=0.0, max_iter=30, store_basis=True,
                     allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == 30 and S.rs.v_cur == 24 and S.rs.v_lz == 24
        lz = host(S.lz[:48])
        assert rel(lz[0::2], ref["alpha"]) <= 1e-10 and rel(lz[1::2], ref["rho"]) <= 1e-10
        assert rel(host(S.V[:24]).T, ref["V"]) <= 1e-10
        st = S.refresh(t1, dev(x1), s=6, inner=True)
        assert S.rs.s_cur == 6
        # RMINRES stores Lanczos vectors without CG coefficients: the inner refresh refuses them
        w.zero_()
        S.solve(t0, dev(x0), dev(g), w, tol=1e-8, store_basis=True, method="rminres")
        assert S.rs.v_lz == 0 and S.rs.v_cur > 0
        with pytest.raises(B.BLError):
            S.refresh(t1, dev(x1), s=6, inner=True)


def test_inner_refresh_long_basis_takes_semiorthogonal_prefix(B):
    """A stored basis of 120 residuals from a long solve has lost orthogonality: both sides keep
    its semi-orthogonal leading part (the oracle from V^T V, the GPU from its Gram matrix), and
    the refreshes agree."""
    wl, prob, xs, (x0, t0), (x1, t1) = pair("tv", 40, 52, 191)
    h0 = lambda v: prob.hvp(x0, t0, v)
    h1 = lambda v: prob.hvp(x1, t1, v)
    prev = krylov.cg(h0, x0 - xs, tol=1e-13, v_cap=120)
    assert prev["V"].shape[1] == 120
    k = recycle.semiorthogonal_prefix(prev["V"])
    assert 6 < k < 120
    ref = recycle.refresh(h1, lambda v: prob.jac_apply(x1, t1, v), None, prev["V"], s=6, hvp_old=h0)
    assert ref["v_used"] == k and ref["t"] == k
    with B.Session(B.problem_from(wl, prec="fp64"), s_max=6, v_cap=120) as S:
        S.V[:120] = dev(prev["V"].T)
        S.lz[:240] = dev(lz_of(prev))
        S.rs.v_cur = S.rs.v_lz = 120
        st = S.refresh(t1, dev(x1), s=6, inner=True)
        assert st.t == k and S.rs.s_cur == 6
        U = host(S.U[:6]).T
        assert recycle.principal_angles(U, ref["U"]).max() <= 1e-6
        mu = host(S.mu[:2])
        assert np.abs(mu - ref["mu"][:2]).max() <= 1e-8 * ref["mu"][0]
