"""GPU: the served form.  Requests of several samples (TV and filters, different sizes and
recycle dimensions, mixed precision) served concurrently by continuous batching give bitwise the
hypergradients, iteration counts and statuses that the same requests give when each sample is
served alone; and the served hypergradients match an FP64 reference solve to 1e-6."""
import time

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


def build(B, ctx, specs, T):
    """Frozen outer steps per sample: a drifting theta path and lower-level solutions."""
    out = []
    for kind, h, w, s, seed in specs:
        if kind == "tv":
            wl = synth.custom("t", h, "tv", s, width=w, blur_radius=2, blur_sigma=1.5, rect_min=2, rect_max=6,
                              seed=seed)
        else:
            wl = synth.custom("f", h, "filters", s, width=w, rect_min=2, rect_max=6, seed=seed)
        inst = synth.instance(wl)
        P64 = B.problem_from(wl, prec="fp64")
        xs = torch.as_tensor(inst["xstar"].ravel(), device=DEV)
        e = torch.as_tensor(inst["e"].ravel(), device=DEV)
        y = torch.empty_like(xs)
        ctx.forward_p(P64, xs, e, wl.noise, y)
        path = synth.theta_drift(wl, T, seed + 5, scale=0.01)
        x = y.clone()
        xhats = []
        for th in path:
            ctx.lower_solve_p(P64, th, y, x, gtol=1e-7, max_iter=2000)
            xhats.append(x.clone())
        out.append((wl, path, xhats, xs, inst))
    return out


def serve_all(B, ctx, data, order, prec, pool=None):
    from paper_2412_08264_amd import serve
    Ps = [B.problem_from(wl, prec=prec) for wl, *_ in data]
    arena = sum(B.Engine.slot_bytes(P, wl.s) for P, (wl, *_) in zip(Ps, data))
    srv = serve.Server(ctx, cap=8, arena_bytes=arena, hg_rel=1e-10, iters_per_turn=8, pool=pool)
    keys = sorted(set(order))
    for k in keys:
        wl, path, xhats, xs, _ = data[k]
        srv.add_sample(serve.Sample(k, Ps[k], path, xhats, xs, wl.s, 32, torch.device(DEV)))
    for i, k in enumerate(order):
        srv.submit(k, float(i))
    # a stuck server fails here; a bound on turns instead would also count the idle turns
    # spent waiting for a refresh on the pool's threads
    deadline = time.monotonic() + 90.0
    while not srv.idle():
        srv.turn()
        assert time.monotonic() < deadline
    res = {}
    for r in srv.completed:
        res[(r.sample.key, r.step)] = (r.hg, r.stats.iters, r.stats.status)
    srv.close()
    return res


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_served_results_same_alone_and_in_mix(B, prec):
    specs = [("tv", 40, 48, 4, 601), ("filters", 36, 36, 6, 602), ("tv", 64, 32, 5, 603), ("filters", 28, 44, 3, 604)]
    T = 3
    P64s = [B.problem_from(synth.custom("x", h, kind, s, width=w), prec="fp64") for kind, h, w, s, _ in specs]
    ctx = B.Context(P64s, s_max=6, v_cap=32, device=torch.device(DEV))
    try:
        data = build(B, ctx, specs, T)
        order = [k for _ in range(T) for k in range(len(specs))]      # interleaved arrivals
        # in the mix, refreshes and hypergradients run on other streams and host threads
        with B.ContextPool(P64s, 6, 32, 3, torch.device(DEV)) as pool:
            mix = serve_all(B, ctx, data, order, prec, pool)
        assert len(mix) == len(specs) * T
        for k in range(len(specs)):
            alone = serve_all(B, ctx, data, [k] * T, prec)
            for step in range(T):
                hg_a, it_a, st_a = alone[(k, step)]
                hg_m, it_m, st_m = mix[(k, step)]
                assert st_a == 0 and st_m == 0
                assert it_a == it_m, (k, step, it_a, it_m)
                assert np.array_equal(hg_a, hg_m), (k, step)
        # served hypergradients against FP64 reference solves (oracle-grade CG on the GPU's inputs)
        for k in (0, 1):
            wl, path, xhats, xs, inst = data[k]
            prob = problem.make_problem(wl, inst["xstar"], inst["e"])
            xh = xhats[T - 1].cpu().numpy()
            th = path[T - 1]
            g = xh - inst["xstar"].ravel()
            wref, _ = krylov.reference_solve(lambda v: prob.hvp(xh, th, v), g)
            ref = prob.jac_apply(xh, th, wref)
            got = mix[(k, T - 1)][0]
            assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)
    finally:
        ctx.close()
