"""GPU: batched and served recycled CG.

A solve advanced inside a batch (any mix of image sizes, recycle dimensions, stop rules and
arrival times) must give bitwise the iterate, iteration count, status and stored basis of the
same solve run alone; the solo path is pinned to the oracle in test_gpu_parity.  The batch
shares kernels between solves but never their reductions, so any difference would be a bug
(a record read from another slot, a wrong iteration index, a missed stop flag).
"""
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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def make_case(B, kind, h, w, s, seed, prec="fp64", v_cap=24):
    """A recycled system at theta + 0.01: the recycle space comes from a plain solve at theta
    (stored basis) and a refresh at the new theta; the warm start is the previous solution."""
    if kind == "tv":
        wl = synth.custom("t", h, "tv", 8, width=w, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=6,
                          seed=seed)
    else:
        wl = synth.custom("f", h, "filters", 8, width=w, rect_min=2, rect_max=6, seed=seed)
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xh = inst["xstar"].ravel() + 0.04 * synth.unit_noise(prob.n, seed + 1)
    th = inst["theta0"]
    th2 = th + 0.01
    P = B.problem_from(wl, prec=prec)
    S = B.Session(P, s_max=max(s, 1), v_cap=v_cap)
    xd, gd = dev(xh), dev(xh - inst["xstar"].ravel())
    w0 = torch.zeros_like(gd)
    S.solve(th, xd, gd, w0, tol=1e-8, store_basis=True, recycle=False)
    if s > 0:
        S.refresh(th2, xd, s=s)
    return dict(P=P, S=S, th=th2, xh=xd, g=gd, w0=w0, rec=S.rec if s > 0 else None, n=prob.n, prob=prob,
                theta_np=th2, xh_np=xh, g_np=xh - inst["xstar"].ravel())


def solo(B, c, **kw):
    w = c["w0"].clone()
    st = c["S"].solve(c["th"], c["xh"], c["g"], w, recycle=c["rec"] is not None,
                      allow=(B.BL_OK, B.BL_E_NOT_CONVERGED), **kw)
    return w, st


def same(st_a, st_b):
    return (st_a.iters, st_a.status, st_a.res_norm, st_a.res0_norm, st_a.g_norm) == \
           (st_b.iters, st_b.status, st_b.res_norm, st_b.res0_norm, st_b.g_norm)


def test_batched_tv_fp64_bitwise_equals_solo(B):
    cases = [make_case(B, "tv", 40, 56, 6, 101), make_case(B, "tv", 64, 64, 8, 102),
             make_case(B, "tv", 24, 100, 0, 103), make_case(B, "tv", 33, 33, 4, 104),
             make_case(B, "tv", 9, 300, 5, 105)]
    opts = B.solve_opts(tol=1e-9, store_basis=False)
    ref = [solo(B, c, tol=1e-9, store_basis=False) for c in cases]
    ws = [c["w0"].clone() for c in cases]
    code, stats = B.hessian_solve_batched([c["P"] for c in cases], [c["th"] for c in cases],
                                          [c["xh"] for c in cases], [c["g"] for c in cases], ws,
                                          [c["rec"] for c in cases], opts)
    assert code == B.BL_OK
    for c, (w_ref, st_ref), w, st in zip(cases, ref, ws, stats):
        assert st_ref.status == B.BL_OK
        assert same(st, st_ref), (c["P"].h, c["P"].w, st.iters, st_ref.iters)
        assert torch.equal(w, w_ref)
    # and the batched answers solve the systems (oracle FP64 solve)
    for c, w in zip(cases[:2], ws[:2]):
        prob = c["prob"]
        ref_w, _ = krylov.reference_solve(lambda v: prob.hvp(c["xh_np"], c["theta_np"], v), c["g_np"])
        assert rel(w.cpu().numpy(), ref_w) <= 1e-7


def test_batched_filters_mixed_bitwise_equals_solo(B):
    """Mixed precision with residual replacement every 8 iterations: replacements fall at
    different global steps in every slot, and each converged slot is re-tested on its FP64
    residual; both must follow the slot's own iteration index."""
    cases = [make_case(B, "filters", 48, 40, 6, 201, prec="mixed"),
             make_case(B, "filters", 40, 72, 0, 202, prec="mixed"),
             make_case(B, "filters", 64, 64, 8, 203, prec="mixed")]
    opts = B.solve_opts(tol=1e-10, rr_every=8, store_basis=False)
    ref = [solo(B, c, tol=1e-10, rr_every=8, store_basis=False) for c in cases]
    ws = [c["w0"].clone() for c in cases]
    code, stats = B.hessian_solve_batched([c["P"] for c in cases], [c["th"] for c in cases],
                                          [c["xh"] for c in cases], [c["g"] for c in cases], ws,
                                          [c["rec"] for c in cases], opts)
    assert code == B.BL_OK
    for c, (w_ref, st_ref), w, st in zip(cases, ref, ws, stats):
        assert st_ref.status == B.BL_OK
        assert same(st, st_ref)
        assert torch.equal(w, w_ref)
        prob = c["prob"]
        ref_w, _ = krylov.reference_solve(lambda v: prob.hvp(c["xh_np"], c["theta_np"], v), c["g_np"])
        assert rel(w.cpu().numpy(), ref_w) <= 1e-6


@pytest.mark.parametrize("kind,prec", [("tv", "fp64"), ("filters", "mixed")])
def test_engine_continuous_admission_bitwise(B, kind, prec):
    """Requests arrive while others run: two are admitted, advanced, a third is refused for
    want of arena space, admitted after the first completes, and each result (iterate, stats,
    stored basis) equals the solo run; the arena is whole again at the end."""
    cases = [make_case(B, kind, 56, 48, 6, 301, prec=prec), make_case(B, kind, 40, 40, 4, 302, prec=prec),
             make_case(B, kind, 64, 72, 8, 303, prec=prec)]
    per = [dict(stop="hgerr", hg_tol=1e-9, tol=1e-12, rr_every=8, store_basis=False),
           dict(stop="resid", tol=1e-9, rr_every=8, store_basis=False),
           dict(stop="resid", tol=1e-9, rr_every=16, store_basis=True)]
    ref = []
    for c, kw in zip(cases, per):
        w, st = solo(B, c, **kw)
        basis = c["rec"].V[: c["rec"].rs.v_cur].clone() if kw["store_basis"] else None
        ref.append((w, st, basis, c["rec"].rs.v_cur))
    sizes = [B.Engine.slot_bytes(c["P"], c["rec"].rs.s_cur if c["rec"] else 0) for c in cases]
    arena = max(sizes[0] + sizes[1], sizes[2])     # the first two fit together, never all three
    eng = B.Engine(cap=3, arena_bytes=arena)
    try:
        ws = [c["w0"].clone() for c in cases]
        slots = {}
        for k in (0, 1):
            sl = eng.admit(cases[k]["P"], cases[k]["th"], cases[k]["xh"], cases[k]["g"], ws[k], cases[k]["rec"],
                           B.solve_opts(**per[k]))
            assert sl is not None
            slots[sl] = k
        # arena full: refused without side effects
        assert eng.admit(cases[2]["P"], cases[2]["th"], cases[2]["xh"], cases[2]["g"], ws[2], cases[2]["rec"],
                         B.solve_opts(**per[2])) is None
        done = eng.step(max_iters=5, return_on_done=False)
        assert done == []
        stats = {}
        pending = [2]
        while slots:
            for sl in eng.step():
                k = slots.pop(sl)
                stats[k] = eng.retire(sl)
            while pending:
                k = pending[0]
                sl = eng.admit(cases[k]["P"], cases[k]["th"], cases[k]["xh"], cases[k]["g"], ws[k], cases[k]["rec"],
                               B.solve_opts(**per[k]))
                if sl is None:
                    break
                slots[sl] = k
                pending.pop(0)
        assert not pending
        running, free_slots, free_bytes, largest = eng.query()
        assert running == 0 and free_slots == 3 and free_bytes == largest >= arena
    finally:
        eng.close()
    for k, c in enumerate(cases):
        w_ref, st_ref, basis, vcur = ref[k]
        assert st_ref.status == B.BL_OK
        assert same(stats[k], st_ref), (k, stats[k].iters, st_ref.iters)
        assert torch.equal(ws[k], w_ref)
        if basis is not None:
            assert c["rec"].rs.v_cur == vcur
            assert torch.equal(c["rec"].V[:vcur], basis)


def test_engine_mixes_operator_classes(B):
    """TV and filter solves in FP64 and mixed precision, each class at two tile heights, with
    and without recycle spaces, share one engine (one apply launch per (class, height,
    recycling) group, one update launch for all) and each equals its solo run bitwise; a 17th
    group is refused while sixteen are admitted.  The shared update launch is the variant with
    recycle-space registers while any recycled solve runs; a plain solve's solo run uses the
    variant without them, so the bitwise match also covers the two variants' agreement."""
    base = [("tv", 36, 44, "fp64"), ("filters", 40, 36, "fp64"), ("filters", 32, 48, "mixed"),
            ("tv", 50, 30, "mixed"), ("tv", 64, 70, "fp64"), ("filters", 70, 66, "fp64"),
            ("filters", 66, 72, "mixed"), ("tv", 72, 64, "mixed")]
    # each shape once with a recycle space (s = 2..5) and once without (s = 0)
    cases = [make_case(B, kind, h, w, s, 401 + 2 * k + (s == 0), prec=prec)
             for k, (kind, h, w, prec) in enumerate(base) for s in (2 + k % 4, 0)]
    # the first eight (size class 10) on 8-row tiles, the last eight (size class 12) on 32
    heights = [8] * 8 + [32] * 8
    kw = dict(tol=1e-9, rr_every=8, store_basis=False)
    extra = B.bl_problem(32, 32, 3, 1.5, B.BL_REG_TV, 0, 0, 0.0, 0, 0)   # another blur radius
    try:
        for c, rows in zip(cases, heights):
            B.bl_tile_rows_set(c["P"], rows)
        assert [B.bl_tile_rows(c["P"]) for c in cases] == heights
        ref = [solo(B, c, **kw) for c in cases]
        arena = sum(B.Engine.slot_bytes(c["P"], c["rec"].rs.s_cur if c["rec"] else 0) for c in cases) + \
            B.Engine.slot_bytes(extra, 0)
        with B.Engine(cap=17, arena_bytes=arena) as eng:
            ws = [c["w0"].clone() for c in cases]
            slots = {}
            for k, c in enumerate(cases):
                sl = eng.admit(c["P"], c["th"], c["xh"], c["g"], ws[k], c["rec"], B.solve_opts(**kw))
                slots[sl] = k
            w9 = torch.zeros(32 * 32, dtype=torch.float64, device=DEV)
            with pytest.raises(B.BLError):
                eng.admit(extra, np.zeros(2), w9, w9, w9, None, B.solve_opts())
            with pytest.raises(B.BLError):
                eng.retire(16)                       # nothing there
            stats = {}
            while slots:
                for sl in eng.step():
                    stats[slots.pop(sl)] = eng.retire(sl)
    finally:
        for c in cases:
            B.bl_tile_rows_set(c["P"], 0)
    for k in range(len(cases)):
        w_ref, st_ref = ref[k]
        assert st_ref.status == B.BL_OK
        assert same(stats[k], st_ref), k
        assert torch.equal(ws[k], w_ref)


def test_graph_replay_bitwise_equals_direct_launches(B):
    """Repeated chunks of iterations replayed from captured graphs give bitwise the iterates,
    counts and statuses of direct launches: a long FP64 TV solve (error-estimate stop tested
    every 4 iterations), a mixed-precision filter solve (scheduled residual replacements every
    16 iterations and the final re-test change the chunks' launch sequences), a plain solve, and
    a batch of three with continuous admission; the replay path is taken (the context's
    counters: chunks alternate between two header buffers, so the first two chunks are
    captured and the later ones replayed)."""
    cases = [make_case(B, "tv", 64, 72, 6, 701), make_case(B, "filters", 48, 40, 4, 702, prec="mixed"),
             make_case(B, "tv", 40, 36, 0, 703)]
    kws = [dict(tol=1e-11, stop="hgerr", hg_tol=0.0, check_every=4, max_iter=300, store_basis=True),
           dict(tol=1e-12, rr_every=16, store_basis=False), dict(tol=1e-12, store_basis=False)]
    for c, kw in zip(cases, kws):
        S = c["S"]
        cap0, rep0 = S.graph_counts()
        w_g, st_g = solo(B, c, **kw)
        cap1, rep1 = S.graph_counts()
        S.set_graphs(False)
        try:
            w_d, st_d = solo(B, c, **kw)
        finally:
            S.set_graphs(True)
        assert S.graph_counts() == (cap1, rep1)
        assert rep1 - rep0 >= 2 and cap1 > cap0, (cap0, rep0, cap1, rep1, st_g.iters, st_g.status, st_d.iters,
                                                  B.lib.bl_last_error(S.ctx).decode())
        assert same(st_g, st_d) and st_g.iters == st_d.iters
        assert torch.equal(w_g, w_d)
        if c["rec"] is not None and kw.get("store_basis"):
            assert c["rec"].rs.v_cur > 0
    # engine: graphs on and off over the same admissions
    outs = []
    for graphs in (True, False):
        ctx = B.Context([c["P"] for c in cases], s_max=6, v_cap=24)
        ctx.set_graphs(graphs)
        arena = sum(B.Engine.slot_bytes(c["P"], c["rec"].rs.s_cur if c["rec"] else 0) for c in cases)
        ws = [c["w0"].clone() for c in cases]
        with B.Engine(cap=2, arena_bytes=arena, ctx=ctx.ctx) as eng:
            pending, slots, stats = list(range(3)), {}, {}
            while pending or slots:
                while pending:
                    k = pending[0]
                    sl = eng.admit(cases[k]["P"], cases[k]["th"], cases[k]["xh"], cases[k]["g"], ws[k],
                                   cases[k]["rec"], B.solve_opts(tol=1e-11, store_basis=False))
                    if sl is None:
                        break
                    slots[sl] = pending.pop(0)
                for sl in eng.step(max_iters=24):
                    stats[slots.pop(sl)] = eng.retire(sl)
        outs.append((ws, stats, ctx.graph_counts()))
        ctx.close()
    (wg, sg, cg), (wd, sd, _) = outs
    assert cg[1] > 0
    for k in range(3):
        assert same(sg[k], sd[k]) and torch.equal(wg[k], wd[k]), k
