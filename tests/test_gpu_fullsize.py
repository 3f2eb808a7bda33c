"""GPU parity at the largest image size of the served workload (1024 x 1024, about 1 M pixels),
in the launch configuration the benchmark uses (the tile height of the library's table):

* recycled CG with an s = 10 recycle space, a fixed number of steps with the error-estimate
  records on tested iterations: iterate and estimate against the oracle (1e-10, 1e-9);
* the filter Hessian-vector product in FP64 (1e-13) and with FP32 stencils (1e-6).
The oracle's products at this size take about 1 s (TV) and 10 s (filters) each, so the solve
runs a few steps only."""
import numpy as np
import pytest

import synth
from oracle import krylov, problem

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


def test_recycled_cg_1024_tv(B):
    wl = synth.custom("big", 1024, "tv", 10, rect_min=8, rect_max=20, seed=91)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"]
    xh = inst["xstar"].ravel() + 0.05 * synth.unit_noise(prob.n, 92)
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    rng = np.random.default_rng(94)
    s = 10
    Ut = rng.standard_normal((prob.n, s))
    Cq, Rc = np.linalg.qr(np.stack([hvp(Ut[:, j]) for j in range(s)], axis=1))
    U = np.linalg.solve(Rc.T, Ut.T).T
    Z = np.linalg.qr(rng.standard_normal((prob.n, s)))[0]
    mu = np.geomspace(1.0, 1e-2, s)
    k = 6
    ref = krylov.recycled_cg(hvp, g, None, U, Cq, Z, mu, tol=0.0, max_iter=k, stop="hgerr", hg_tol=0.0,
                             record=True, recurrence="single")   # the GPU's FP64 single-reduction form
    with B.Session(B.problem_from(wl), s_max=s, v_cap=4) as S:
        S.U[:s] = dev(U.T)
        S.Cm[:s] = dev(Cq.T)
        S.Z[:s] = dev(Z.T)
        S.mu[:s] = dev(mu)
        S.rs.s_cur = s
        w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
        st = S.solve(th, dev(xh), dev(g), w, tol=0.0, max_iter=k, stop="hgerr", hg_tol=0.0, check_every=2,
                     store_basis=False, allow=(B.BL_E_NOT_CONVERGED,))
        assert st.iters == k
        assert rel(host(w), ref["w"]) <= 1e-10
        want = ref["hist_nsc"][k]
        assert abs(st.est - want) <= 1e-9 * want


def test_hvp_filters_1024(B):
    wl = synth.custom("big", 1024, "filters", 10, rect_min=8, rect_max=20, seed=95)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"]
    xh = inst["xstar"].ravel() + 0.02 * synth.unit_noise(prob.n, 96)
    v = synth.unit_noise(prob.n, 97)
    ref = prob.hvp(xh, th, v)
    for prec, tol in (("fp64", 1e-13), ("mixed", 1e-6)):
        with B.Session(B.problem_from(wl, prec=prec)) as S:
            out = torch.empty(prob.n, dtype=torch.float64, device=DEV)
            S.hvp(th, dev(xh), dev(v), out)
            assert rel(host(out), ref) <= tol, prec


def test_mixed_precision_converged_solve_filters_256(B):
    """Mixed precision (FP32 filter stencils, FP64 dots, projections and residual replacement)
    converged on a 256 x 256 filter problem (two 7 x 7 filters, the filter family's 11 x 11 blur):
    w and the hypergradient within 1e-6 of the oracle's FP64 reference solve (plain CG to 1e-13
    with true-residual replacement), with and without a recycle space.  The reconstruction is a
    stand-in point with small filter responses (|K_j x| < 1, so phi'' > 0 and H is SPD) and
    the filter weights are e^0 = 1; the oracle needs about 260 products (17 s)."""
    import math
    wl = synth.custom("f", 256, "filters", 8, n_filters=2, filter_size=7, seed=3101)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"].copy()
    for j in range(2):
        th[j * 50] = math.log(1.0)
    xh = 0.2 * inst["xstar"].ravel() + 0.01 * synth.unit_noise(prob.n, 3102)
    assert max(np.abs(k).max() for k in prob.responses(xh, th)[2]) < 1.0
    g = xh - inst["xstar"].ravel()
    hvp = lambda v: prob.hvp(xh, th, v)
    wref, _ = krylov.reference_solve(hvp, g)
    hgref = prob.jac_apply(xh, th, wref)
    # a recycle space: s random directions, C = H U orthonormalised by QR (oracle products)
    rng = np.random.default_rng(3103)
    s = 4
    Ut = rng.standard_normal((prob.n, s))
    Cq, Rc = np.linalg.qr(np.stack([hvp(Ut[:, j]) for j in range(s)], axis=1))
    U = np.linalg.solve(Rc.T, Ut.T).T
    with B.Session(B.problem_from(wl, prec="mixed"), s_max=s, v_cap=8) as S:
        for recycled in (False, True):
            if recycled:
                S.U[:s] = dev(U.T)
                S.Cm[:s] = dev(Cq.T)
                S.rs.s_cur = s
            w = torch.zeros(prob.n, dtype=torch.float64, device=DEV)
            st = S.solve(th, dev(xh), dev(g), w, tol=1e-10, rr_every=25, store_basis=False, recycle=recycled,
                         max_iter=5000)
            assert st.status == 0
            assert rel(host(w), wref) <= 1e-6, (recycled, rel(host(w), wref))
            assert rel(S.hypergradient(th, dev(xh), w), hgref) <= 1e-6
