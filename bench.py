"""Benchmark: hypergradient Hessian solves/s (recycled vs plain CG) at hypergradient rel err 1e-6.

Default workload (tv256): 256x256 smoothed-TV deblurring, FP64, recycle dimension s = 20, a
frozen sequence of 30 outer (upper-level) iterations.  Inputs are synthetic (seeded rectangles,
9x9 Gaussian blur sigma 2.5, noise 0.01), generated on the GPU before timing: measurement y, the
30-step gradient-descent trajectory {theta_i, x_hat_i} and reference hypergradients (plain CG to
relative residual 1e-13).  One step = one pass of the hot path over the whole sequence: for
every system the Ritz-GSV refresh (RGen-L(R)), the recycled CG solve with the
hypergradient-error stop, and the hypergradient.  A solve counts towards ``value`` only if its
hypergradient is within 1e-6 (relative) of the reference.  Plain warm-started CG, recycling
with the residual stop, RMINRES with the error-estimate stop and MINRES (the paper's solver)
are timed on the same sequence and reported beside the headline.

Other workloads (``--workload``):
  tv32     the same protocol on the 32x32 TV recipe;
  foe512   512x512, eight 7x7 filters, mixed precision (FP32 stencils) against FP64, s = 30;
  batch64  64 filter images of sides {128..512}, shared theta, one engine advancing all 64 solves
           per launch; one step = one outer iteration of the whole training set;
  serve    Poisson request stream over resident samples (TV and filters, sides 64..1024,
           s in {10, 30, 50}) served by continuous batching; p50/p99 latency, mixed and FP64;
  selections  the tv256 sequence refreshed by every selection rule of Table 2 (Ritz, harmonic
           Ritz, sides of RGen-L), recycled CG with the residual stop;
  train    tv256 trained end to end (not a frozen sequence) with recycled CG, RMINRES and plain
           CG hypergradients; wall time per outer iteration and its split;
  sweep    tv256 over recycle dimensions s and stored-basis capacities v_cap, outer and inner
           refreshes, with plain CG beside them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hypergradient Hessian solves/sec (recycled vs plain CG) at rel err 1e-6; p99 ms"
V_CAP = 64
RESID_TOL = 1e-10      # residual tolerance of the workload recipe (upper end of the sweep)
# Each variant is timed at the loosest stopping threshold of its sweep for which every
# hypergradient of the sequence is within 1e-6 of the reference (untimed selection pass).
SWEEP_RESID = (1e-6, 3e-7, 1e-7, 3e-8, 1e-8, 1e-9, 1e-10)
SWEEP_HG = (1e-7, 3e-8, 1e-8, 3e-9, 1e-9, 3e-10, 1e-10, 1e-11)   # relative to the previous hypergradient norm
LBFGS_CAP = 1500       # L-BFGS iterations per lower solve of a trajectory (warm started)
HBM_PEAK = 8000.0      # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def upper_loss(x, xs):
    d = x - xs
    return 0.5 * float((d * d).sum())


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def step_bytes_per_pixel(reg: str, prec: str, s: int, nf: int, z_cols: float = 0.0) -> float:
    """Algorithmic HBM bytes per pixel of the launch the library times in each Krylov step.
    FP64 (one fused launch per iteration): read r, q, p, w and write r, p, q, w (FP64), read the s
    columns of C and of H C, z_cols columns of Z on average (the error-estimate test reads all of
    Z on the iterations it runs), and the Hessian state: x_hat for TV, the nf phi'' maps for
    filters.  Mixed precision (the apply launch of the two-launch step): read r and p, write p and
    q (FP64), read the s columns of C and the state (FP32 phi'' maps)."""
    if prec == "mixed":
        b = 8 * 4 + 8 * s
        b += 8 if reg == "tv" else 4 * nf
        return b
    b = 8 * 8 + 16 * s + 8 * z_cols
    b += 8 if reg == "tv" else 8 * nf
    return b


def step_kernel(prec: str, radius: int, reg: str, rows: int, rec: bool = True, single: bool = True) -> str:
    """Name of the timed launch's kernel (the template arguments as rocprofv3 prints them); `single`:
    the FP64 step of a launch that holds one solve (its descriptor passed by value)."""
    cls = 0 if reg == "tv" else 1
    if prec == "mixed":
        return f"k_b_apply<float, {radius}, {cls}, {rows // 8}, {'true' if rec else 'false'}>"
    return f"k_f_step<{radius}, {cls}, {rows // 8}, {'true' if rec else 'false'}, {'true' if single else 'false'}>"


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("tile.h", "common.h", "batch_tile.h"):
        with open(os.path.join(ROOT, "paper_2412_08264_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM traffic per launch from committed rocprofv3 counter summaries, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh).get(f"{kernel}@{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


KT_SAMPLE = 8   # the library records kernel events on one Krylov step in eight


def roofline(kernel, bytes_per_launch, kt, workload):
    """Achieved HBM rate of the apply kernel: algorithmic bytes per launch over its mean duration,
    the duration from HIP events the library records around sampled launches of the timed run."""
    apply_ms = kt[0] / max(kt[1], 1.0)
    achieved = bytes_per_launch / max(apply_ms * 1e-3, 1e-30) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s", "frac": achieved / HBM_PEAK,
            "traffic": measured_traffic(kernel, workload), "kernel": kernel, "avg_launch_us": apply_ms * 1e3,
            "timed_launches": int(kt[1]), "algorithmic_bytes_per_launch": bytes_per_launch,
            "update_avg_us": kt[2] / max(kt[3], 1.0) * 1e3}


def autotune_tiles(ctx, B, items, iters=100):
    """Tile heights from the library's autotuner, one run per (operator class, size class):
    items are (P, theta, xhat, s).  Returns {label: {"rows": r, "us_per_iter": [8, 16, 32 rows]}}."""
    out = {}
    for P, th, xh, s in items:
        lg = int(np.floor(np.log2(P.h * P.w)))
        label = (f"{'tv' if P.reg == B.BL_REG_TV else 'filters'} r{P.blur_radius} "
                 f"{'mixed' if P.prec == B.BL_PREC_MIXED else 'fp64'} n~2^{lg}")
        if label in out:
            continue
        rows, us = ctx.autotune_tiles(P, th, xh, s, iters)
        out[label] = {"rows": rows, "us_per_iter": [round(u, 2) for u in us]}
        log(f"[bench] autotune {label}: {rows} rows ({', '.join(f'{u:.1f}' for u in us)} us/iteration)")
    return out


def base_line(args, value, el, dtype, config, **extra):
    out = {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    return out


def threads_used():
    from threadpoolctl import threadpool_info
    return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])


# =============================================================================== sequence workloads
def make_trajectory(ctx, P, B, wl, torch, y, xs, theta0, outer, gtol=1e-8):
    """Gradient descent with backtracking on theta (frozen sequence), all on the GPU.

    Lower solves stop at ||grad Phi|| <= 1e-8 or after LBFGS_CAP iterations (the smoothing
    weight the descent reaches makes 1e-8 unreachable in reasonable time at 256x256); the
    gradient norms reached are logged.  The Hessian systems of the sequence are SPD at any
    point, so the frozen sequence is a valid workload either way.
    """
    th = np.array(theta0, dtype=np.float64)
    x = y.clone()
    ctx.lower_solve_p(P, th, y, x, gtol=gtol, max_iter=LBFGS_CAP)
    c1 = upper_loss(x, xs)
    beta = 1.0
    thetas, xhats = [], []
    w = torch.zeros_like(x)
    nl = []
    for i in range(outer):
        thetas.append(th.copy())
        xhats.append(x.clone())
        g = x - xs
        w.zero_()
        ctx.solve_p(P, None, th, x, g, w, tol=1e-12, store_basis=False, recycle=False, max_iter=50000,
                    allow=(B.BL_OK, B.BL_E_NOT_CONVERGED))
        grad = ctx.hypergradient_p(P, th, x, w)
        d = -grad
        c2 = float(grad @ d)
        xprev = x
        for j in range(1, 31):
            tau = beta * 0.5 ** (j - 1)
            thj = th + tau * d
            xj = xprev.clone()
            lst = ctx.lower_solve_p(P, thj, y, xj, gtol=gtol, max_iter=LBFGS_CAP)
            nl.append((lst.iters, float(f"{lst.res_norm:.1e}")))
            c0 = upper_loss(xj, xs)
            if c0 <= c1 + 1e-4 * tau * c2:
                th, x, c1, beta = thj, xj, c0, 2.0 * tau
                break
            xprev = xj
        log(f"  trajectory step {i + 1}/{outer}: loss {c1:.6e} L-BFGS (iterations, |grad|) {nl}")
        nl.clear()
    return thetas, xhats


def run_sequence(S, B, torch, thetas, xhats, xs, mode, refs, lat=None, thr=RESID_TOL, rr_every=50,
                 first_tol=RESID_TOL, check_every=1, inner=False):
    """One pass over the sequence.  mode: 'rgen_hg' | 'rgen_res' | 'plain' (recycled CG, or CG)
    | 'rminres_hg' | 'minres' (RMINRES with the error-estimate stop, or MINRES); thr: the stopping
    threshold (residual tolerance, or the error-estimate threshold relative to the previous
    hypergradient norm); first_tol: residual tolerance of the error-estimate variant's first
    system, which has no recycle space yet (the threshold of the variant without recycling);
    inner: refreshes by the inner variant (eq. subtle-old) instead of the outer one.
    Returns per-solve records."""
    method = "rminres" if mode in ("rminres_hg", "minres") else "cg"
    kind = {"rminres_hg": "rgen_hg", "minres": "plain"}.get(mode, mode)
    S.reset()
    w = torch.zeros_like(xs)
    prev_hg = None
    recs = []
    for i, (th, x) in enumerate(zip(thetas, xhats)):
        t0 = time.perf_counter()
        g = x - xs
        if kind != "plain" and i > 0:
            S.refresh(th, x, s=S.rs.s_max, inner=inner)
        if kind == "rgen_hg" and S.rs.s_cur > 0 and prev_hg is not None:
            st = S.solve(th, x, g, w, stop="hgerr", hg_tol=thr * prev_hg, tol=RESID_TOL, store_basis=True,
                         rr_every=rr_every, check_every=check_every, method=method)
        else:
            # first system of the error-estimate variant (no recycle space yet): residual test
            st = S.solve(th, x, g, w, tol=first_tol if kind == "rgen_hg" else thr,
                         store_basis=(kind != "plain"), recycle=(kind != "plain"), rr_every=rr_every,
                         method=method)
        hg = S.hypergradient(th, x, w)
        t1 = time.perf_counter()
        if lat is not None:
            lat.append((t1 - t0) * 1e3)
        prev_hg = float(np.linalg.norm(hg))
        recs.append({"iters": st.iters, "err": rel_err(hg, refs[i]), "status": st.status, "hg": hg})
    return recs


def choose_threshold(S, B, torch, thetas, xhats, xs, mode, refs, sweep, first_tol=RESID_TOL, check_every=1,
                     inner=False):
    for thr in sweep:
        rr = run_sequence(S, B, torch, thetas, xhats, xs, mode, refs, thr=thr, first_tol=first_tol,
                          check_every=check_every, inner=inner)
        if all(r["err"] <= 1e-6 and r["status"] == 0 for r in rr):
            return thr
    return sweep[-1]


def timed_passes(S, B, torch, thetas, xhats, xs, mode, refs, thr, steps, lat=None, first_tol=RESID_TOL,
                 check_every=1, inner=False):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [run_sequence(S, B, torch, thetas, xhats, xs, mode, refs, lat, thr=thr, first_tol=first_tol,
                         check_every=check_every, inner=inner) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ok = sum(1 for rr in recs for r in rr if r["err"] <= 1e-6 and r["status"] == 0)
    total = sum(len(rr) for rr in recs)
    return recs, el, ok, total


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_sequence(wl, thetas, xhats, xs_t, ftol, thr, check_every, gpu_iters_per_solve, budget_s=12.0):
    """The CPU oracle on the benchmark's own systems with the headline's stop rules, over a bounded
    sample scaled to solves/s.

    One tv256 system takes the oracle longer than the sample's budget, so the sample is: the
    first system's solve (plain CG, residual stop ftol) cut at the iteration count that fits the
    budget, timed per iteration; the refresh of the second system from that run's basis (outer
    RGen-L(R): t products, projected GSVD, U, C, Z) and one hypergradient, timed once.  The
    oracle's time per solve is then refresh + hypergradient + (the GPU headline's mean
    iterations per solve) x (time per iteration).  Run twice: with the BLAS threads of every
    affinity core, and with one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import krylov, problem, recycle
    import synth
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xs = xs_t.detach().cpu().numpy()
    th0, x0 = thetas[0], xhats[0].detach().cpu().numpy()
    th1, x1 = thetas[1], xhats[1].detach().cpu().numpy()

    def one(limit):
        with threadpool_limits(limits=limit):
            hvp0 = lambda v: prob.hvp(x0, th0, v)
            t0 = time.perf_counter()
            for _ in range(5):
                hvp0(x0)
            per = (time.perf_counter() - t0) / 5
            k = max(10, int(0.7 * budget_s / per))
            t0 = time.perf_counter()
            res = krylov.recycled_cg(hvp0, x0 - xs, None, tol=ftol, max_iter=k, v_cap=V_CAP)
            t_it = (time.perf_counter() - t0) / max(res["iters"], 1)
            t0 = time.perf_counter()
            rs = recycle.refresh(lambda v: prob.hvp(x1, th1, v), lambda v: prob.jac_apply(x1, th1, v), None, res["V"],
                                 wl.s)
            t_ref = time.perf_counter() - t0
            t0 = time.perf_counter()
            prob.jac_apply(x1, th1, res["w"])
            t_hg = time.perf_counter() - t0
            per_solve = t_ref + t_hg + gpu_iters_per_solve * t_it
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
            return 1.0 / per_solve, res["iters"], t_it, t_ref, t_hg, threads

    v_all, it_all, tit_all, tref_all, thg_all, thr_all = one(None)
    v_one, _, tit_one, tref_one, _, _ = one(1)
    ncores = len(os.sched_getaffinity(0))
    return {"value": v_all, "unit": "solves/s", "cores": ncores, "kind": "oracle",
            "sample": (f"oracle on the bench's own {wl.h}x{wl.w} systems: {it_all} CG iterations of system 0 "
                       f"({tit_all * 1e3:.1f} ms each), the outer RGen-L(R) refresh of system 1 ({tref_all:.2f} s) "
                       f"and a hypergradient ({thg_all * 1e3:.0f} ms), scaled to one solve of the headline's mean "
                       f"{gpu_iters_per_solve:.0f} iterations (the threshold rule {thr:g} x previous |grad| "
                       f"decides those on the GPU); NumPy FP64"),
            "blas_threads": int(thr_all), "cpu_model": cpu_model(),
            "value_1thread": v_one, "ms_per_iter_1thread": tit_one * 1e3, "refresh_s_1thread": tref_one}


def oracle_reference_worker(inp: str, outp: str) -> None:
    """Child process of the benchmark: the oracle's reference hypergradients (plain CG to relative
    residual 1e-13 with true-residual replacement, Section 5's reference) for the listed systems."""
    import synth
    from oracle import krylov, problem
    d = np.load(inp, allow_pickle=False)
    wl = synth.WORKLOADS[str(d["workload"])]
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    xs = inst["xstar"].ravel()
    hgs, its = [], []
    for th, xh in zip(d["thetas"], d["xhats"]):
        w, it = krylov.reference_solve(lambda v: prob.hvp(xh, th, v), xh - xs, tol=1e-13)
        hgs.append(prob.jac_apply(xh, th, w))
        its.append(it)
    np.savez(outp, hg=np.stack(hgs), iters=np.array(its))


def start_oracle_gate(wl, thetas, xhats, idx):
    import subprocess
    import tempfile
    d = tempfile.mkdtemp(prefix="bench_oracle_")
    inp, outp = os.path.join(d, "in.npz"), os.path.join(d, "out.npz")
    np.savez(inp, workload=np.array(wl.name), thetas=np.stack([thetas[i] for i in idx]),
             xhats=np.stack([xhats[i].detach().cpu().numpy() for i in idx]))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-ref", inp, outp],
                            stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, env=env)
    return {"proc": proc, "out": outp, "idx": list(idx), "t0": time.perf_counter()}


def finish_oracle_gate(gate, hgs_by_variant, timeout_s=300.0):
    """Relative error of each listed variant's hypergradients against the oracle's references."""
    try:
        gate["proc"].wait(timeout=max(1.0, timeout_s - (time.perf_counter() - gate["t0"])))
    except Exception:
        gate["proc"].kill()
        return {"systems": gate["idx"], "error": "oracle reference timed out"}
    if gate["proc"].returncode != 0 or not os.path.exists(gate["out"]):
        err = gate["proc"].stderr.read().decode()[-400:] if gate["proc"].stderr else ""
        return {"systems": gate["idx"], "error": f"oracle reference failed: {err}"}
    d = np.load(gate["out"], allow_pickle=False)
    out = {"systems": gate["idx"], "oracle_cg_iters": [int(v) for v in d["iters"]],
           "seconds": round(time.perf_counter() - gate["t0"], 1)}
    for name, hgs in hgs_by_variant.items():
        out[f"{name}_vs_oracle"] = [rel_err(np.asarray(h), o) for h, o in zip(hgs, d["hg"])]
    return out


def bench_selections(args, B, torch, synth):
    """tv256 with every recycle-space selection of Table 2: recycled CG with the residual stop,
    each rule at the loosest threshold of SWEEP_RESID that keeps every hypergradient within 1e-6;
    reports solves/s, iterations per pass and the mean refresh time of each rule."""
    wl = synth.WORKLOADS["tv256"]
    outer = args.outer or wl.outer
    dev = torch.device("cuda:0")
    inst = synth.instance(wl)
    P64 = B.problem_from(wl, prec="fp64")
    S = B.Session(P64, s_max=wl.s, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs, e = t(inst["xstar"]), t(inst["e"])
    y = torch.empty_like(xs)
    S.forward(xs, e, wl.noise, y)
    thetas, xhats = make_trajectory(S, P64, B, wl, torch, y, xs, inst["theta0"], outer)
    refs = []
    w = torch.zeros_like(xs)
    for th, x in zip(thetas, xhats):
        w.zero_()
        S.solve(th, x, x - xs, w, tol=1e-13, store_basis=False, recycle=False, max_iter=100000,
                allow=(B.BL_OK, B.BL_E_NOT_CONVERGED))
        refs.append(S.hypergradient(th, x, w))
    tiles = autotune_tiles(S, B, [(S.P, thetas[0], xhats[0], wl.s)])

    def one_pass(rule, thr, refresh_ms=None):
        S.reset()
        w = torch.zeros_like(xs)
        recs = []
        for i, (th, x) in enumerate(zip(thetas, xhats)):
            if i > 0:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.refresh(th, x, s=wl.s, select=rule)
                torch.cuda.synchronize()
                if refresh_ms is not None:
                    refresh_ms.append((time.perf_counter() - t0) * 1e3)
            st = S.solve(th, x, x - xs, w, tol=thr, store_basis=True)
            hg = S.hypergradient(th, x, w)
            recs.append({"iters": st.iters, "err": rel_err(hg, refs[i]), "status": st.status})
        return recs

    out_rules = {}
    # RGen of sizes S and M needs p >= t; TV has p = 2
    for rule in [r for r in B.SELECTIONS if not r.startswith(("rgen-s", "rgen-m"))]:
        thr = SWEEP_RESID[-1]
        for cand in SWEEP_RESID:
            rr = one_pass(rule, cand)
            if all(r["err"] <= 1e-6 and r["status"] == 0 for r in rr):
                thr = cand
                break
        one_pass(rule, thr)
        ref_ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = [one_pass(rule, thr, ref_ms) for _ in range(args.steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ok = sum(1 for rr in recs for r in rr if r["err"] <= 1e-6 and r["status"] == 0)
        total = sum(len(rr) for rr in recs)
        out_rules[rule] = {"solves_per_s": ok / el, "threshold": thr, "iters_per_sequence": sum(r["iters"] for r in recs[0]),
                           "refresh_ms": float(np.mean(ref_ms)), "passing": f"{ok}/{total}",
                           "max_rel_err": max(r["err"] for r in recs[0])}
        log(f"[bench] {rule}: {out_rules[rule]}")
    head = out_rules["rgen-l-r"]
    desc = (f"selections: tv256 ({wl.h}x{wl.w} smoothed-TV, s={wl.s}, {outer} frozen outer steps), recycled CG "
            f"with the residual stop after a refresh by each rule of Table 2")
    return base_line(args, head["solves_per_s"], 0.0, "f64", {"workload": desc, "outer_steps": outer, "s": wl.s,
                                                              "tiles": tiles},
                     selections=out_rules)


SWEEP_GRID = ((20, 64), (10, 64), (50, 64), (20, 128), (20, 236), (10, 246), (50, 206))


def bench_sweep(args, B, torch, synth):
    """tv256: recycled CG with RGen-L(R) and the error-estimate stop (Section 5.1, "Dimension of the
    recycle space") at recycle dimensions s and stored-basis capacities v_cap (s + v_cap <= 256, the
    refresh's limit), outer and inner refreshes, each at the loosest threshold of SWEEP_HG that
    keeps every hypergradient within 1e-6; plain CG beside them.  Reports iterations per pass,
    solves/s and the mean refresh time of each setting."""
    wl = synth.WORKLOADS["tv256"]
    outer = args.outer or wl.outer
    dev = torch.device("cuda:0")
    inst = synth.instance(wl)
    P64 = B.problem_from(wl, prec="fp64")
    S0 = B.Session(P64, s_max=wl.s, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs, e = t(inst["xstar"]), t(inst["e"])
    y = torch.empty_like(xs)
    S0.forward(xs, e, wl.noise, y)
    thetas, xhats = make_trajectory(S0, P64, B, wl, torch, y, xs, inst["theta0"], outer)
    refs = []
    w = torch.zeros_like(xs)
    for th, x in zip(thetas, xhats):
        w.zero_()
        S0.solve(th, x, x - xs, w, tol=1e-13, store_basis=False, recycle=False, max_iter=100000,
                 allow=(B.BL_OK, B.BL_E_NOT_CONVERGED))
        refs.append(S0.hypergradient(th, x, w))
    tiles = autotune_tiles(S0, B, [(S0.P, thetas[0], xhats[0], wl.s)])
    ftol = choose_threshold(S0, B, torch, thetas, xhats, xs, "plain", refs, SWEEP_RESID)
    rr, el, ok, tot = timed_passes(S0, B, torch, thetas, xhats, xs, "plain", refs, ftol, args.steps)
    rows = [{"s": 0, "v_cap": 0, "refresh": "-", "threshold": ftol, "iters_per_sequence": sum(r["iters"] for r in rr[0]),
             "solves_per_s": ok / el, "passing": f"{ok}/{tot}"}]
    log(f"[bench] sweep plain: {rows[-1]}")
    S0.close()
    for s_, vc in SWEEP_GRID:
        S = B.Session(P64, s_max=s_, v_cap=vc, device=dev)
        for inner in (False, True):
            thr = choose_threshold(S, B, torch, thetas, xhats, xs, "rgen_hg", refs, SWEEP_HG, first_tol=ftol,
                                   check_every=args.check_every, inner=inner)
            S.set_timing(1)
            ref_ms = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs = []
            for _ in range(args.steps):
                S.reset()
                wv = torch.zeros_like(xs)
                prev_hg = None
                rec = []
                for i, (th, x) in enumerate(zip(thetas, xhats)):
                    if i > 0:
                        st = S.refresh(th, x, s=s_, inner=inner)
                        ref_ms.append(st.ms[3])
                    if S.rs.s_cur > 0 and prev_hg is not None:
                        st = S.solve(th, x, x - xs, wv, stop="hgerr", hg_tol=thr * prev_hg, tol=RESID_TOL,
                                     check_every=args.check_every)
                    else:
                        st = S.solve(th, x, x - xs, wv, tol=ftol)
                    hg = S.hypergradient(th, x, wv)
                    prev_hg = float(np.linalg.norm(hg))
                    rec.append({"iters": st.iters, "err": rel_err(hg, refs[i]), "status": st.status})
                recs.append(rec)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            S.set_timing(0)
            ok = sum(1 for rr in recs for r in rr if r["err"] <= 1e-6 and r["status"] == 0)
            tot = sum(len(rr) for rr in recs)
            rows.append({"s": s_, "v_cap": vc, "refresh": "inner" if inner else "outer", "threshold": thr,
                         "iters_per_sequence": sum(r["iters"] for r in recs[0]), "solves_per_s": ok / el,
                         "passing": f"{ok}/{tot}", "refresh_ms": float(np.mean(ref_ms)) if ref_ms else 0.0})
            log(f"[bench] sweep: {rows[-1]}")
        S.close()
    best = max(rows[1:], key=lambda r: r["solves_per_s"])
    desc = (f"sweep: tv256 ({wl.h}x{wl.w} smoothed-TV, {outer} frozen outer steps), recycled CG with RGen-L(R) and "
            f"the error-estimate stop over recycle dimension s and stored-basis capacity v_cap, outer and inner "
            f"refreshes; plain CG beside them")
    return base_line(args, best["solves_per_s"], 0.0, "f64", {"workload": desc, "outer_steps": outer, "tiles": tiles},
                     sweep=rows, best=best, plain_cg=rows[0])


def bench_train(args, B, torch, synth):
    """tv256 trained end to end (Algorithm 2 with Algorithm 1's backtracking, `outer` steps from
    theta0): hypergradients by recycled CG with RGen-L(R) and the error-estimate stop, by RMINRES
    likewise, and by plain CG; reports the wall time split into lower-level solves, refreshes,
    Hessian solves and hypergradients, and the final upper loss."""
    from paper_2412_08264_amd import train as T
    wl = synth.WORKLOADS["tv256"]
    outer = args.outer or 10
    dev = torch.device("cuda:0")
    inst = synth.instance(wl)
    P64 = B.problem_from(wl, prec="fp64")
    S = B.Session(P64, s_max=wl.s, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs, e = t(inst["xstar"]), t(inst["e"])
    y = torch.empty_like(xs)
    S.forward(xs, e, wl.noise, y)
    autotune_tiles(S, B, [(S.P, inst["theta0"], y, wl.s)])
    runs = {}
    for name, kw in (("recycled_cg", dict(s=wl.s, solver="cg", stop="hgerr")),
                     ("rminres", dict(s=wl.s, solver="rminres", stop="hgerr")),
                     ("plain_cg", dict(s=0, solver="cg", stop="resid"))):
        t0 = time.perf_counter()
        hist = T.train(S, y, xs, inst["theta0"], outer, tol=1e-8, hg_rel=1e-8, check_every=args.check_every,
                       lbfgs_iters=LBFGS_CAP, **kw)
        el = time.perf_counter() - t0
        runs[name] = {"seconds": el, "outer_per_s": outer / el, "final_loss": hist["loss"][-1],
                      "hessian_iters": sum(hist["iters"]), "lbfgs_iters": sum(hist["lbfgs_iters"]),
                      "split_s": {k: round(v, 3) for k, v in hist["seconds"].items()}}
        log(f"[bench] train {name}: {runs[name]}")
    desc = (f"train: tv256 ({wl.h}x{wl.w} smoothed-TV) trained end to end for {outer} outer steps from theta0, "
            f"s={wl.s}, error-estimate stop 1e-8 x previous |grad| (first system and plain CG: residual 1e-8)")
    head = runs["recycled_cg"]
    return base_line(args, head["outer_per_s"], head["seconds"], "f64", {"workload": desc, "outer_steps": outer},
                     unit_note="outer iterations per second", train=runs)


def bench_sequence(args, B, torch, synth):
    wl = synth.WORKLOADS[args.workload]
    outer = args.outer or wl.outer
    dev = torch.device("cuda:0")
    inst = synth.instance(wl)
    P64 = B.problem_from(wl, prec="fp64")
    S = B.Session(P64, s_max=wl.s, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs, e = t(inst["xstar"]), t(inst["e"])
    y = torch.empty_like(xs)
    S.forward(xs, e, wl.noise, y)
    log(f"[bench] {args.workload}: {wl.h}x{wl.w} {wl.reg}, s={wl.s}, outer={outer}; building the trajectory")
    tt = time.perf_counter()
    thetas, xhats = make_trajectory(S, P64, B, wl, torch, y, xs, inst["theta0"], outer)
    log(f"[bench] trajectory built in {time.perf_counter() - tt:.1f} s; reference hypergradients")
    refs, ref_ok = [], 0
    w = torch.zeros_like(xs)
    for th, x in zip(thetas, xhats):
        w.zero_()
        st = S.solve(th, x, x - xs, w, tol=1e-13, store_basis=False, recycle=False, max_iter=100000,
                     allow=(B.BL_OK, B.BL_E_NOT_CONVERGED))
        ref_ok += st.status == B.BL_OK
        refs.append(S.hypergradient(th, x, w))
    if ref_ok < len(refs):
        log(f"[bench] WARNING: {len(refs) - ref_ok} reference solves stopped at the iteration limit "
            "before relative residual 1e-13: the run is marked failed")
    mixed = wl.prec == "mixed"
    Sh = B.Session(B.problem_from(wl, prec="mixed"), s_max=wl.s, v_cap=V_CAP, device=dev) if mixed else S
    if args.rows:   # a fixed tile height (profiling runs repeat the height a timed run chose)
        for PP in (Sh.P, S.P):
            B.bl_tile_rows_set(PP, args.rows)
        tiles = {"fixed": args.rows}
    else:
        tiles = autotune_tiles(S, B, [(Sh.P, thetas[0], xhats[0], wl.s), (S.P, thetas[0], xhats[0], wl.s)])
    # threshold selection (untimed): loosest setting with every hypergradient within 1e-6
    variants = [("rgen_hg", Sh, SWEEP_HG), ("rgen_res", Sh, SWEEP_RESID), ("plain", S, SWEEP_RESID),
                ("rgen_hg_inner", Sh, SWEEP_HG)]
    if mixed:
        variants.append(("rgen_hg_fp64", S, SWEEP_HG))
    # the paper's own solver (FP64): RMINRES with the error-estimate stop, and MINRES
    variants += [("minres", S, SWEEP_RESID), ("rminres_hg", S, SWEEP_HG)]
    chosen = {}
    # variants without recycling first: their thresholds are the first-system tolerances of
    # the estimate variants of the same solver
    first_of = lambda name: chosen.get("minres" if name == "rminres_hg" else "plain", RESID_TOL)
    order = [v for v in variants if v[0] in ("plain", "minres")] + [v for v in variants
                                                                    if v[0] not in ("plain", "minres")]
    mode_of = lambda name: name.replace("_fp64", "").replace("_inner", "")
    for name, SS, sweep in order:
        chosen[name] = choose_threshold(SS, B, torch, thetas, xhats, xs, mode_of(name), refs, sweep,
                                        first_tol=first_of(name), check_every=args.check_every,
                                        inner=name.endswith("_inner"))
        log(f"[bench] {name}: threshold {chosen[name]:g}")
    ftol = chosen["plain"]
    for _ in range(args.warmup):
        run_sequence(Sh, B, torch, thetas, xhats, xs, "rgen_hg", refs, thr=chosen["rgen_hg"], first_tol=ftol,
                     check_every=args.check_every)
    # timed: headline (recycled + error-estimate stop), per-kernel events on the library's stream
    Sh.set_timing(2)
    Sh.kernel_times(reset=True)
    lat = []
    recs, el, ok, total = timed_passes(Sh, B, torch, thetas, xhats, xs, "rgen_hg", refs, chosen["rgen_hg"],
                                       args.steps, lat, first_tol=ftol, check_every=args.check_every)
    kt = Sh.kernel_times(reset=True)
    Sh.set_timing(0)
    value = ok / el
    extra, hg_of = {}, {}
    for name, SS, _ in variants[1:]:
        mode, inner = mode_of(name), name.endswith("_inner")
        run_sequence(SS, B, torch, thetas, xhats, xs, mode, refs, thr=chosen[name], first_tol=first_of(name),
                     check_every=args.check_every, inner=inner)
        rr, elm, okm, totm = timed_passes(SS, B, torch, thetas, xhats, xs, mode, refs, chosen[name], args.steps,
                                          first_tol=first_of(name), check_every=args.check_every, inner=inner)
        extra[name] = {"solves_per_s": okm / elm, "threshold": chosen[name],
                       "iters_per_sequence": sum(r["iters"] for r in rr[0]),
                       "max_rel_err": max(r["err"] for r in rr[0]), "passing": f"{okm}/{totm}"}
        hg_of[name] = rr[0]
    head = recs[0]
    iters_seq = sum(r["iters"] for r in head)
    prec = "mixed" if mixed else "fp64"
    # the error-estimate test reads the s columns of Z on one iteration in check_every
    bpp = step_bytes_per_pixel(wl.reg, prec, wl.s, wl.n_filters, z_cols=wl.s / args.check_every)
    kname = step_kernel(prec, wl.blur_radius, wl.reg, B.bl_tile_rows(Sh.P))
    desc = (f"{args.workload}: {wl.h}x{wl.w} {'smoothed-TV' if wl.reg == 'tv' else '8 x 7x7 filter'} deblurring, "
            f"blur r={wl.blur_radius} sigma={wl.blur_sigma}, noise {wl.noise}, {outer} frozen outer steps, "
            f"RGen-L(R) s={wl.s}, error-estimate stop {chosen['rgen_hg']:g} x previous |grad| tested every "
            f"{args.check_every} iterations (first system: "
            f"residual {ftol:g}, as plain CG)"
            + (", FP32 stencils + FP64 rest with residual replacement" if mixed else ""))
    out = base_line(args, value, el, "f32+f64" if mixed else "f64",
                    {"workload": desc, "outer_steps": outer, "s": wl.s, "v_cap": V_CAP, "n": wl.n, "tiles": tiles},
                    passing=f"{ok}/{total}",
                    latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                    iters_per_sequence={"rgen_hg": iters_seq, **{k: v["iters_per_sequence"] for k, v in extra.items()}},
                    max_rel_err=max(r["err"] for r in head),
                    speedup_vs_plain_cg=value / extra["plain"]["solves_per_s"],
                    reference_converged=f"{ref_ok}/{len(refs)}",
                    plain_cg=extra["plain"], rgen_resid=extra["rgen_res"], rgen_inner=extra["rgen_hg_inner"],
                    roofline=roofline(kname, bpp * wl.n, kt, args.workload))
    if ref_ok < len(refs):
        out["status"] = "failed: reference solves did not converge"
    if mixed:
        out["rgen_hg_fp64"] = extra["rgen_hg_fp64"]
    out["rminres"] = extra["rminres_hg"]
    out["minres"] = extra["minres"]
    if not args.no_micro and args.workload == "tv256":
        log("[bench] HBM microbenchmark (4096 x 4096)")
        out["hbm_micro"] = hbm_micro(args, B, torch, synth)
    if not args.no_cpu:
        # the CPU leg, after every GPU timing (host work beside the timed GPU runs would slow their
        # launches): the oracle timed on the same systems, and its reference hypergradients of the
        # first and last systems (in a child process) as a gate on the GPU's own references and on
        # the headline's results
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline_sequence(wl, thetas, xhats, xs, ftol, chosen["rgen_hg"], args.check_every,
                                                    iters_seq / len(thetas))
        log("[bench] the oracle's reference hypergradients of the first and last systems")
        gate = start_oracle_gate(wl, thetas, xhats, [0, len(thetas) - 1])
        idx = gate["idx"]
        pick = lambda recs: [recs[i]["hg"] for i in idx]
        out["cpu_baseline"]["oracle_gate"] = finish_oracle_gate(
            gate, {"reference": [refs[i] for i in idx], "headline": pick(head), "plain_cg": pick(hg_of["plain"])})
    S.close()
    if Sh is not S:
        Sh.close()
    return out


# =============================================================================== batched training set
def bench_batch(args, B, torch, synth):
    """64 filter images, shared theta: per outer step a refresh of every image's recycle space,
    one engine advancing all 64 recycled solves together, and the summed hypergradient."""
    from paper_2412_08264_amd import train as train_mod
    wls = synth.batch_set(args.batch, 4000, s=20)
    T = args.outer or 4
    dev = torch.device("cuda:0")
    prec = args.prec
    Ps = [B.problem_from(wl, prec=prec) for wl in wls]
    P64 = [B.problem_from(wl, prec="fp64") for wl in wls]
    ctx = B.Context(P64, s_max=20, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs, ys, xcur = [], [], []
    for wl, P in zip(wls, P64):
        inst = synth.instance(wl)
        xsk, ek = t(inst["xstar"]), t(inst["e"])
        yk = torch.empty_like(xsk)
        ctx.forward_p(P, xsk, ek, wl.noise, yk)
        xs.append(xsk)
        ys.append(yk)
        xcur.append(yk.clone())
    theta = synth.instance(wls[0])["theta0"].copy()   # shared theta (filters seeded alike)
    nf, f2 = wls[0].n_filters, wls[0].filter_size ** 2
    log(f"[bench] batch{len(wls)}: sum n = {sum(w.n for w in wls)}, {T} Adam steps to build the frozen sequence")
    # frozen sequence: Adam (lr 1e-2) on the summed upper loss; tap updates kept zero-mean
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    thetas, xhats, refs = [], [], []
    opts_ref = B.solve_opts(tol=1e-12, max_iter=100000, store_basis=False)
    tt = time.perf_counter()
    for i in range(T):
        its = []
        for k, P in enumerate(P64):
            st = ctx.lower_solve_p(P, theta, ys[k], xcur[k], gtol=1e-6, max_iter=400)
            its.append(st.iters)
        thetas.append(theta.copy())
        xhats.append([x.clone() for x in xcur])
        wref = [torch.zeros_like(x) for x in xcur]
        code, _ = B.hessian_solve_batched(P64, [theta] * len(P64), xcur, [x - s for x, s in zip(xcur, xs)], wref,
                                          [None] * len(P64), opts_ref, device=dev, ctx=ctx.ctx)
        hgs = [ctx.hypergradient_p(P, theta, x, w) for P, x, w in zip(P64, xcur, wref)]
        refs.append(hgs)
        grad = np.sum(hgs, axis=0)
        theta, m, v = train_mod.adam_update(theta, grad, m, v, i + 1, 1e-2, zero_mean_blocks=(nf, wls[0].filter_size))
        log(f"  step {i + 1}/{T}: L-BFGS iterations max {max(its)} mean {np.mean(its):.0f}, "
            f"|grad| {np.linalg.norm(grad):.3e} ({time.perf_counter() - tt:.1f} s)")
    recs = [B.Recycle(w.n, 20, V_CAP, dev) for w in wls]
    arena = int(lib_batched_bytes(B, Ps, [20] * len(Ps)) * 1.02)
    eng = B.Engine(cap=min(len(Ps), 64), arena_bytes=arena, device=dev, ctx=ctx.ctx)
    # refreshes and hypergradients of the images run concurrently on a pool of contexts
    pool = B.ContextPool(P64, 20, V_CAP, args.workers, dev)

    phase_ms = {"refresh": 0.0, "solve": 0.0, "hypergradient": 0.0}

    def one_pass(mode, thr, stats=None, first_tol=RESID_TOL, phases=None):
        """The sequence once: mode 'rgen_hg' (refresh + error-estimate stop; first step: residual
        stop at first_tol, as plain CG), 'plain' (residual stop at thr)."""
        for r in recs:
            r.rs.s_cur = 0
            r.rs.v_cur = 0
        ws = [torch.zeros_like(x) for x in xs]
        prev = [None] * len(Ps)
        errs, iters = [], []

        def mark(name, t0):
            if phases is not None:
                torch.cuda.synchronize()
                phases[name] += (time.perf_counter() - t0) * 1e3
            return time.perf_counter()
        for i in range(T):
            xh = xhats[i]
            tp = time.perf_counter()
            if mode != "plain" and i > 0:
                pool.map(lambda c, k: c.refresh_p(P64[k], recs[k], thetas[i], xh[k], s=20),
                         [(k,) for k in range(len(P64))])
            tp = mark("refresh", tp)
            slot_of = {}
            for k, P in enumerate(Ps):
                use_hg = mode == "rgen_hg" and recs[k].rs.s_cur > 0 and prev[k] is not None
                o = B.solve_opts(stop="hgerr" if use_hg else "resid", hg_tol=thr * prev[k] if use_hg else 0.0,
                                 tol=first_tol if mode != "plain" else thr, store_basis=mode != "plain",
                                 rr_every=50, check_every=args.check_every if use_hg else 1)
                sl = eng.admit(P, thetas[i], xh[k], xh[k] - xs[k], ws[k], recs[k] if mode != "plain" else None, o)
                assert sl is not None, "engine arena too small"
                slot_of[sl] = k
            while slot_of:
                for sl in eng.step(return_on_done=False):
                    k = slot_of.pop(sl)
                    st = eng.retire(sl)
                    iters.append(st.iters)
                    if stats is not None:
                        stats.append((k, st.iters))
            tp = mark("solve", tp)
            hg = pool.map(lambda c, k: c.hypergradient_p(P64[k], thetas[i], xh[k], ws[k]),
                          [(k,) for k in range(len(P64))])
            mark("hypergradient", tp)
            for k in range(len(Ps)):
                prev[k] = float(np.linalg.norm(hg[k]))
                errs.append(rel_err(hg[k], refs[i][k]))
        return errs, iters

    chosen = {}
    for mode, sweep in (("plain", SWEEP_RESID), ("rgen_hg", SWEEP_HG)):
        chosen[mode] = sweep[-1]
        for thr in sweep:
            errs, _ = one_pass(mode, thr, first_tol=chosen.get("plain", RESID_TOL))
            if max(errs) <= 1e-6:
                chosen[mode] = thr
                break
        log(f"[bench] batch {mode}: threshold {chosen[mode]:g}")
    ftol = chosen["plain"]
    # tile heights: the whole batch shares the chip, so the autotuner times whole passes, one
    # per height for every image (untimed)
    search = {}
    for rows in ((args.rows,) if args.rows else (8, 16, 32)):
        for P in Ps:
            B.bl_tile_rows_set(P, rows)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        one_pass("rgen_hg", chosen["rgen_hg"], first_tol=ftol)
        torch.cuda.synchronize()
        search[rows] = (time.perf_counter() - ts) * 1e3
    best_rows = min(search, key=search.get)
    for P in Ps:
        B.bl_tile_rows_set(P, best_rows)
    log(f"[bench] batch tile heights: {best_rows} rows (ms per pass {search})")
    for _ in range(args.warmup):
        one_pass("rgen_hg", chosen["rgen_hg"], first_tol=ftol)
    one_pass("rgen_hg", chosen["rgen_hg"], first_tol=ftol, phases=phase_ms)   # phase split (untimed)
    ctx.set_timing(2)
    ctx.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    allerr, alliters, stats = [], [], []
    for _ in range(args.steps):
        errs, its = one_pass("rgen_hg", chosen["rgen_hg"], stats, first_tol=ftol)
        allerr += errs
        alliters += its
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = ctx.kernel_times(reset=True)
    ctx.set_timing(0)
    ok = sum(1 for e in allerr if e <= 1e-6)
    value = ok / el
    total_bytes = sum(step_bytes_per_pixel("filters", prec, 20, nf, z_cols=20 / args.check_every) * wls[k].n * it
                      for k, it in stats)
    launches = max(kt[1] * KT_SAMPLE, 1.0)   # apply launches of the timed passes (sampled 1 in 8)
    one_pass("plain", chosen["plain"])
    torch.cuda.synchronize()
    tp = time.perf_counter()
    perr, piters = [], []
    for _ in range(args.steps):
        e_, i_ = one_pass("plain", chosen["plain"])
        perr += e_
        piters += i_
    torch.cuda.synchronize()
    elp = time.perf_counter() - tp
    okp = sum(1 for e in perr if e <= 1e-6)
    kname = step_kernel(prec, 5, "filters", best_rows)
    out = base_line(args, value, el, "f32+f64" if prec == "mixed" else "f64",
                    {"workload": f"batch{len(wls)}: {len(wls)} filter images (8 x 7x7, blur r=5 sigma=3, noise 0.02), "
                                 f"sides {sorted(set(w.h for w in wls))}, sum n = {sum(w.n for w in wls)}, shared theta, "
                                 f"{T} frozen Adam steps, RGen-L(R) s=20 per image, one engine for all solves",
                     "images": len(wls), "outer_steps": T, "s": 20, "sum_n": sum(w.n for w in wls),
                     "tiles": {"rows": best_rows, "ms_per_pass": {str(k): round(v, 2) for k, v in search.items()}}},
                    passing=f"{ok}/{len(allerr)}", max_rel_err=max(allerr),
                    iters_per_pass={"rgen_hg": sum(alliters) // args.steps, "plain": sum(piters) // args.steps},
                    plain_cg={"solves_per_s": okp / elp, "threshold": chosen["plain"], "passing": f"{okp}/{len(perr)}"},
                    speedup_vs_plain_cg=value / max(okp / elp, 1e-30),
                    phase_ms_per_pass={k: round(v, 1) for k, v in phase_ms.items()},
                    roofline=roofline(kname, total_bytes / launches, kt, "batch64"))
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline_batch(wls)
    eng.close()
    pool.close()
    ctx.close()
    return out


def lib_batched_bytes(B, Ps, s):
    import ctypes as C
    arr = (B.bl_problem * len(Ps))(*Ps)
    sv = (C.c_int * len(Ps))(*s)
    return int(B.lib.bl_batched_workspace_bytes(len(Ps), arr, sv))


def cpu_baseline_batch(wls, seconds_budget=25.0):
    """The oracle on images of the batch taken smallest first (stand-in points x* + 0.05 e'),
    each a plain-start recycled CG solve (no recycle space yet) + hypergradient."""
    import synth
    from oracle import krylov, problem
    order = sorted(range(len(wls)), key=lambda k: wls[k].n)
    done, px = 0, 0
    t0 = time.perf_counter()
    for k in order:
        wl = wls[k]
        inst = synth.instance(wl)
        prob = problem.make_problem(wl, inst["xstar"], inst["e"])
        xs = inst["xstar"].ravel()
        xh = xs + 0.05 * synth.unit_noise(prob.n, wl.seed + 77)
        th = inst["theta0"]
        res = krylov.recycled_cg(lambda v: prob.hvp(xh, th, v), xh - xs, None, None, None, tol=RESID_TOL, v_cap=0)
        prob.jac_apply(xh, th, res["w"])
        done += 1
        px += wl.n
        if time.perf_counter() - t0 > seconds_budget:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "solves/s", "cores": int(threads_used()), "kind": "oracle",
            "sample": f"{done} of the {len(wls)} images, smallest first ({px} pixels; the batch has "
                      f"{sum(w.n for w in wls)}), CG 1e-10 + hypergradient at stand-in points x*+0.05e', numpy FP64, "
                      f"{el:.1f} s; host {len(os.sched_getaffinity(0))} affinity cores"}


# =============================================================================== served stream
def bench_serve(args, B, torch, synth):
    """Poisson request stream over resident samples served by continuous batching."""
    from paper_2412_08264_amd import serve
    dev = torch.device("cuda:0")
    wls = synth.serve_samples(256, 5000)[: args.samples]
    T = args.outer or 4
    P64 = [B.problem_from(wl, prec="fp64") for wl in wls]
    ctx = B.Context(P64, s_max=max(w.s for w in wls), v_cap=args.v_cap, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    log(f"[bench] serve: {len(wls)} samples, sum n = {sum(w.n for w in wls)}, {T} frozen outer steps each")
    tt = time.perf_counter()
    data = []
    for k, (wl, P) in enumerate(zip(wls, P64)):
        inst = synth.instance(wl)
        xs, e = t(inst["xstar"]), t(inst["e"])
        y = torch.empty_like(xs)
        ctx.forward_p(P, xs, e, wl.noise, y)
        path = synth.theta_drift(wl, T, wl.seed + 99)
        x = y.clone()
        xhats = []
        for th in path:
            ctx.lower_solve_p(P, th, y, x, gtol=1e-6, max_iter=300)
            xhats.append(x.clone())
        data.append((path, xhats, xs))
    log(f"[bench] frozen steps built in {time.perf_counter() - tt:.1f} s")
    pool = B.ContextPool(P64, max(w.s for w in wls), args.v_cap, args.workers, dev)
    modes = {}
    tiles = {}
    # the offered rate in both precisions, then (mixed) a rate below the measured capacity, where
    # latency is service time rather than queueing
    # last: plain warm-started FP64 CG on the same stream (no recycle space, no refresh; every
    # solve on the residual test at --serve-tol), the baseline of the recycled forms
    runs = ([("mixed", args.rate), ("fp64", args.rate)] + ([("mixed", args.rate2)] if args.rate2 > 0 else [])
            + [("fp64_plain", args.rate)])
    for mode, rate in runs:
        prec = "fp64" if mode == "fp64_plain" else mode
        arrivals = synth.poisson_arrivals(rate, args.warm_s + args.duration, len(wls), seed=5001)
        Ps = [B.problem_from(wl, prec=prec) for wl in wls]
        tiles.update(autotune_tiles(ctx, B, [(P, data[k][0][0], data[k][1][0], wl.s)
                                             for k, (P, wl) in enumerate(zip(Ps, wls))]))
        arena = sum(B.Engine.slot_bytes(P, wl.s) for P, wl in zip(Ps, wls))
        srv = serve.Server(ctx, cap=64, arena_bytes=arena, hg_rel=args.hg_rel, tol=args.serve_tol, pool=pool,
                           check_every=args.check_every, recycle=mode != "fp64_plain")
        for k, (wl, P) in enumerate(zip(wls, Ps)):
            path, xhats, xs = data[k]
            srv.add_sample(serve.Sample(k, P, path, xhats, xs, wl.s, args.v_cap, dev))
        ctx.set_timing(2)
        ctx.kernel_times(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srv.clock = lambda: time.perf_counter() - t0
        i = 0
        end = args.warm_s + args.duration
        while True:
            now = srv.clock()
            while i < len(arrivals) and arrivals[i][0] <= now:
                srv.submit(arrivals[i][1], arrivals[i][0])
                i += 1
            if now >= end:
                break
            if srv.idle():
                if i < len(arrivals):
                    time.sleep(max(0.0, min(arrivals[i][0] - now, 1e-3)))
                continue
            srv.turn()
        backlog = len(srv.queue) + len(srv.preparing) + len(srv.ready) + len(srv.running) + len(srv.finishing)
        for req in srv.preparing + srv.finishing:   # drain the pool before the next run
            if req.fut is not None:
                req.fut.result()
        kt = ctx.kernel_times(reset=True)
        ctx.set_timing(0)
        win = [r for r in srv.completed if r.t_arrival >= args.warm_s]
        # references for every (sample, step) served in the window: FP64 CG to 1e-12
        refs = {}
        for r in win:
            key = (r.sample.key, r.step)
            if key in refs:
                continue
            smp = r.sample
            w = torch.zeros_like(smp.xstar)
            ctx.solve_p(smp.P64, None, smp.thetas[r.step], smp.xhats[r.step], smp.xhats[r.step] - smp.xstar, w,
                        tol=1e-12, recycle=False, store_basis=False, max_iter=100000,
                        allow=(B.BL_OK, B.BL_E_NOT_CONVERGED))
            refs[key] = ctx.hypergradient_p(smp.P64, smp.thetas[r.step], smp.xhats[r.step], w)
        errs = [rel_err(r.hg, refs[(r.sample.key, r.step)]) for r in win]
        ok = sum(1 for r, e in zip(win, errs) if e <= 1e-6 and r.stats.status == 0)
        lat = [(r.t_done - r.t_arrival) * 1e3 for r in win]
        stage = lambda a, b: float(np.mean([(getattr(r, b) - getattr(r, a)) * 1e3 for r in win])) if win else None
        stages = {"queue": stage("t_arrival", "t_start"), "refresh": stage("t_start", "t_ready"),
                  "wait_engine": stage("t_ready", "t_admit"), "solve": stage("t_admit", "t_solved"),
                  "hypergradient": stage("t_solved", "t_done")}
        sc = 0 if mode == "fp64_plain" else None   # plain CG reads no recycle columns
        bpp = lambda smp: step_bytes_per_pixel("tv" if smp.P.reg == B.BL_REG_TV else "filters", prec,
                                               smp.s if sc is None else sc, smp.P.n_filters,
                                               z_cols=smp.s / args.check_every if sc is None else 0.0)
        total_bytes = sum(bpp(r.sample) * r.sample.P.h * r.sample.P.w * r.stats.iters for r in srv.completed)
        launches = max(kt[1] * KT_SAMPLE, 1.0)
        key = mode if rate == args.rate else f"{mode}_at_{rate:g}_per_s"
        modes[key] = {"rate_per_s": rate, "solves_per_s": ok / args.duration, "completed": len(win),
                       "passing": f"{ok}/{len(win)}",
                       "arrived": sum(1 for a in arrivals if args.warm_s <= a[0] < end),
                       "backlog_at_end": backlog,
                       "latency_ms": {"p50": float(np.percentile(lat, 50)) if lat else None,
                                      "p99": float(np.percentile(lat, 99)) if lat else None},
                       "max_rel_err": max(errs) if errs else None,
                       "mean_iters": float(np.mean([r.stats.iters for r in win])) if win else None,
                       "mean_stage_ms": {k: (round(v, 2) if v is not None else None) for k, v in stages.items()},
                       "roofline": roofline("k_b_apply<float, *> (all classes)" if prec == "mixed" else
                                            "k_f_step<*> (all classes)", total_bytes / launches, kt, "serve")}
        log(f"[bench] serve {key}: {modes[key]['solves_per_s']:.1f} solves/s, p50 "
            f"{modes[key]['latency_ms']['p50']} ms, p99 {modes[key]['latency_ms']['p99']} ms, backlog {backlog}")
        srv.close()
    head = modes["mixed"]
    out = base_line(args, head["solves_per_s"], args.duration * 1e3 * args.steps, "f32+f64",
                    {"workload": f"serve: {len(wls)} resident samples (sides {sorted(set(w.h for w in wls))}, TV or "
                                 f"8 x 7x7 filters, s in {sorted(set(w.s for w in wls))}), {T} frozen outer steps each, "
                                 f"Poisson arrivals {args.rate:g}/s, {args.duration:g} s window after {args.warm_s:g} s, "
                                 f"continuous batching (engine cap 64), error-estimate stop {args.hg_rel:g} x previous "
                                 f"|grad| tested every {args.check_every} iterations, residual stop {args.serve_tol:g} "
                                 f"without a recycle space, mixed precision; recycled FP64 and plain warm-started "
                                 f"FP64 CG (residual stop {args.serve_tol:g}, no refresh) on the same stream beside it",
                     "samples": len(wls), "rate_per_s": args.rate, "window_s": args.duration, "tiles": tiles},
                    latency_ms=head["latency_ms"], passing=head["passing"], mixed=head, fp64=modes["fp64"],
                    roofline=head["roofline"], **{k: v for k, v in modes.items() if k not in ("mixed", "fp64")})
    out["steps"] = 1
    out["ms_per_step"] = args.duration * 1e3
    plain = modes["fp64_plain"]
    out["vs_plain_fp64_cg"] = {
        "solves_per_s": [head["solves_per_s"], plain["solves_per_s"]],
        "p99_ms": [head["latency_ms"]["p99"], plain["latency_ms"]["p99"]],
        "ratio": head["solves_per_s"] / max(plain["solves_per_s"], 1e-30)}
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline_serve(wls, data_steps=T)
    pool.close()
    ctx.close()
    return out


def cpu_baseline_serve(wls, data_steps, seconds_budget=25.0):
    """The oracle serving requests serially on the smallest samples (stand-in points
    x* + 0.05 e'): per request a recycled CG solve (refresh after the first) + hypergradient."""
    import synth
    from oracle import krylov, problem, recycle
    order = sorted(range(len(wls)), key=lambda k: wls[k].n)
    done = 0
    t0 = time.perf_counter()
    for k in order:
        wl = wls[k]
        inst = synth.instance(wl)
        prob = problem.make_problem(wl, inst["xstar"], inst["e"])
        xs = inst["xstar"].ravel()
        xh = xs + 0.05 * synth.unit_noise(prob.n, wl.seed + 77)
        U = V = w = None
        for th in synth.theta_drift(wl, min(data_steps, 2), wl.seed + 99):
            hvp = lambda v, th=th: prob.hvp(xh, th, v)
            jac = lambda v, th=th: prob.jac_apply(xh, th, v)
            rs = recycle.refresh(hvp, jac, U, V, wl.s) if V is not None else {"U": None, "C": None}
            res = krylov.recycled_cg(hvp, xh - xs, w, rs["U"], rs["C"], tol=RESID_TOL, v_cap=V_CAP)
            jac(res["w"])
            U, V, w = rs["U"], res["V"], res["w"]
            done += 1
        if time.perf_counter() - t0 > seconds_budget:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "solves/s", "cores": int(threads_used()), "kind": "oracle",
            "sample": f"{done} requests served serially on the smallest samples (2 outer steps each, refresh + "
                      f"recycled CG 1e-10 + hypergradient) at stand-in points x*+0.05e', numpy FP64, {el:.1f} s; host "
                      f"{len(os.sched_getaffinity(0))} affinity cores"}


# =============================================================================== HBM microbenchmark
def hbm_micro(args, B, torch, synth, side=4096, s=20, iters=63):
    """HBM rate of the iteration kernels where the working set is far above the 256 MB Infinity
    Cache: a 4096 x 4096 TV problem (16.8 M pixels, FP64) solved for a fixed number of iterations
    (stop test off) with s recycle columns that are zero (plain-CG arithmetic with every projection
    read and written as in a recycled solve), then without a recycle space.  The fused step's
    durations come from the library's sampled HIP events; rates use algorithmic bytes."""
    wl = synth.custom("tv4096", side, "tv", s, blur_radius=4, blur_sigma=2.5, rect_min=8, rect_max=20, seed=6001)
    inst = synth.instance(wl)
    dev = torch.device("cuda:0")
    n = wl.n
    P = B.problem_from(wl, prec="fp64")
    S = B.Session(P, s_max=s, v_cap=0, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs = t(inst["xstar"])
    xh = xs + 0.05 * t(synth.unit_noise(n, 6002))
    g = xh - xs
    th = inst["theta0"]
    if args.rows:
        B.bl_tile_rows_set(P, args.rows)
    out = {"workload": f"{side}x{side} smoothed-TV (r=4), FP64, {iters} iterations, s={s} zero recycle columns "
                       f"(recycled) or none (plain), residual stop off; tile height "
                       + (f"{args.rows} rows" if args.rows else "tuned per variant"),
           "n": n}
    for name, sc in (("recycled", s), ("plain", 0)):
        # each variant at the tile height its own autotune picks (the plain step has a fraction
        # of the recycled one's registers, so the two need not agree)
        tuned = None if args.rows else S.autotune_tiles(P, th, xh, sc, 24)[1]
        S.rs.s_cur = sc
        w = torch.zeros_like(xs)
        # iteration counts of whole chunks (the launch of iteration k tests iterate k - 1: k + 1
        # launches), so that no launch of a stopped solve enters the kernel statistics
        S.solve(th, xh, g, w, tol=0.0, max_iter=15, store_basis=False, recycle=sc > 0, allow=(B.BL_E_NOT_CONVERGED,))
        S.set_timing(2)
        S.kernel_times(reset=True)
        w.zero_()
        S.solve(th, xh, g, w, tol=0.0, max_iter=iters, store_basis=False, recycle=sc > 0,
                allow=(B.BL_E_NOT_CONVERGED,))
        kt = S.kernel_times(reset=True)
        S.set_timing(0)
        a_us = kt[0] / max(kt[1], 1.0) * 1e3
        a_bytes = int(step_bytes_per_pixel("tv", "fp64", sc, 0) * n)
        out[name] = {"step": {"kernel": step_kernel("fp64", 4, "tv", B.bl_tile_rows(P), sc > 0),
                              "avg_us": round(a_us, 2), "algorithmic_bytes": a_bytes,
                              "GBps": round(a_bytes / (a_us * 1e3), 1),
                              "frac": round(a_bytes / (a_us * 1e3) / HBM_PEAK, 3), "launches": int(kt[1])},
                     "tile_rows": B.bl_tile_rows(P),
                     "autotune_us_per_iter": [round(u, 1) for u in tuned] if tuned else None}
    S.close()
    torch.cuda.empty_cache()
    return out


# =============================================================================== kernels-only
def kernels_only_batch(args, B, torch, synth):
    """batch64 shapes at stand-in points x* + 0.05 e': 100 plain iterations of all images in one
    engine (basis stored), a refresh of every image, 100 recycled iterations, then the copy."""
    dev = torch.device("cuda:0")
    wls = synth.batch_set(args.batch, 4000, s=20)
    Ps = [B.problem_from(wl, prec=args.prec) for wl in wls]
    for P in Ps:
        B.bl_tile_rows_set(P, args.rows or 32)
    P64 = [B.problem_from(wl, prec="fp64") for wl in wls]
    ctx = B.Context(P64, s_max=20, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs, xh, recs = [], [], []
    for wl in wls:
        inst = synth.instance(wl)
        xs.append(t(inst["xstar"]))
        xh.append(xs[-1] + 0.05 * t(synth.unit_noise(wl.n, wl.seed + 77)))
        recs.append(B.Recycle(wl.n, 20, V_CAP, dev))
    th = synth.instance(wls[0])["theta0"]
    eng = B.Engine(cap=len(Ps), arena_bytes=int(lib_batched_bytes(B, Ps, [20] * len(Ps)) * 1.02), device=dev,
                   ctx=ctx.ctx)
    for phase in range(2):
        ws = [torch.zeros_like(x) for x in xs]
        if phase == 1:
            for k, P in enumerate(P64):
                ctx.refresh_p(P, recs[k], th, xh[k], s=20)
        slots = set()
        for k, P in enumerate(Ps):
            o = B.solve_opts(tol=0.0, max_iter=100, store_basis=phase == 0)
            slots.add(eng.admit(P, th, xh[k], xh[k] - xs[k], ws[k], recs[k], o))
        while slots:
            for sl in eng.step(return_on_done=False):
                eng.retire(sl)
                slots.discard(sl)
    a = torch.empty(8 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    eng.close()
    ctx.close()
    print(json.dumps({"kernels_only": True, "workload": "batch64", "copy_bytes": a.numel() * 8}))


def kernels_only(args, B, torch, synth):
    """Short run for hardware counters: 200 plain and 200 recycled CG iterations on the
    workload's shape at a stand-in point, then 200 RMINRES steps with the same recycle space and
    200 without (FP64 problems), and one 64 MiB device-to-device copy (counter calibration: its
    FETCH_SIZE / WRITE_SIZE should read 64 MiB each)."""
    if args.workload == "batch64":
        kernels_only_batch(args, B, torch, synth)
        return
    wl = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    inst = synth.instance(wl)
    S = B.Session(B.problem_from(wl), s_max=wl.s, v_cap=V_CAP, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1)
    xs = t(inst["xstar"])
    xh = xs + 0.05 * t(synth.unit_noise(wl.n, wl.seed + 77))
    th = inst["theta0"]
    if args.rows:
        B.bl_tile_rows_set(S.P, args.rows)
    else:
        autotune_tiles(S, B, [(S.P, th, xh, wl.s)])
    w = torch.zeros_like(xs)
    S.solve(th, xh, xh - xs, w, tol=0.0, max_iter=200, store_basis=True, allow=(B.BL_E_NOT_CONVERGED,))
    S.refresh(th, xh, s=wl.s)
    w.zero_()
    S.solve(th, xh, xh - xs, w, tol=0.0, max_iter=200, store_basis=False, allow=(B.BL_E_NOT_CONVERGED,))
    if wl.prec == "fp64":
        for rec in (True, False):
            w.zero_()
            S.solve(th, xh, xh - xs, w, tol=0.0, max_iter=200, store_basis=False, recycle=rec, method="rminres",
                    allow=(B.BL_E_NOT_CONVERGED,))
    a = torch.empty(8 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    S.close()
    print(json.dumps({"kernels_only": True, "workload": wl.name, "copy_bytes": a.numel() * 8,
                      "rows": B.bl_tile_rows(S.P)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tv256", choices=("tv256", "tv32", "foe512", "batch64", "serve", "selections", "train",
                                                      "sweep"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-micro", dest="no_micro", action="store_true",
                    help="skip the 4096 x 4096 HBM microbenchmark of the default workload")
    ap.add_argument("--micro-only", dest="micro_only", action="store_true",
                    help="run only the 4096 x 4096 HBM microbenchmark (profiling aid)")
    ap.add_argument("--outer", type=int, default=0, help="override the number of outer steps")
    ap.add_argument("--batch", type=int, default=64, help="batch64: number of images")
    ap.add_argument("--prec", default="mixed", choices=("mixed", "fp64"), help="batch64: precision")
    ap.add_argument("--workers", type=int, default=8, help="batch64 / serve: contexts (streams) for refreshes "
                    "and hypergradients running beside the engine")
    ap.add_argument("--samples", type=int, default=64, help="serve: resident samples (of the 256-sample recipe)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--rate2", type=float, default=40.0,
                    help="serve: second, sub-capacity arrival rate (mixed precision; 0: skip)")
    ap.add_argument("--duration", type=float, default=20.0, help="serve: measured window (s)")
    ap.add_argument("--warm-s", dest="warm_s", type=float, default=3.0, help="serve: warm-up part of the stream (s)")
    ap.add_argument("--hg-rel", dest="hg_rel", type=float, default=1e-9, help="serve: error-estimate threshold "
                    "relative to the sample's previous hypergradient norm")
    ap.add_argument("--v-cap", dest="v_cap", type=int, default=V_CAP, help="serve: stored Krylov vectors per sample")
    ap.add_argument("--serve-tol", dest="serve_tol", type=float, default=1e-8,
                    help="serve: residual tolerance of solves without a recycle space (first step of a pass)")
    ap.add_argument("--check-every", dest="check_every", type=int, default=8,
                    help="iterations between error-estimate tests (Z^T r is formed on tested iterations only)")
    ap.add_argument("--rows", type=int, default=0, choices=(0, 8, 16, 32),
                    help="tile height of the solves (0: autotune; kernels-only batch64: 0 means 32)")
    ap.add_argument("--oracle-ref", dest="oracle_ref", nargs=2, metavar=("IN", "OUT"),
                    help="internal: the oracle's reference hypergradients for the systems in IN (host only)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profiling aid: a few recycled-CG iterations on the workload's shape at stand-in points "
                         "x* + 0.05 e' (no trajectory) plus a 64 MiB device copy for counter calibration")
    args = ap.parse_args()
    if args.oracle_ref:
        oracle_reference_worker(*args.oracle_ref)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the per-sample solves are "
              "independent: several GPUs would each hold and solve their own samples.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2412_08264_amd import bilevel as B
    torch.cuda.set_device(torch.device("cuda:0"))
    if args.kernels_only:
        kernels_only(args, B, torch, synth)
        return
    if args.micro_only:
        print(json.dumps({"hbm_micro": hbm_micro(args, B, torch, synth)}), flush=True)
        return
    if args.workload == "batch64":
        out = bench_batch(args, B, torch, synth)
    elif args.workload == "serve":
        out = bench_serve(args, B, torch, synth)
    elif args.workload == "selections":
        out = bench_selections(args, B, torch, synth)
    elif args.workload == "train":
        out = bench_train(args, B, torch, synth)
    elif args.workload == "sweep":
        out = bench_sweep(args, B, torch, synth)
    else:
        out = bench_sequence(args, B, torch, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
