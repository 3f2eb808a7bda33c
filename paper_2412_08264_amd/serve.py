"""Served hypergradient requests with continuous batching on one GPU.

A Server keeps every training sample's recycle state (U, C = H U, Z, mu and the stored Krylov
basis V) resident in device memory, keyed by the sample.  A request asks for the hypergradient
of one sample at its next outer step: the Ritz-GSV refresh of the sample's recycle space
(RGen-L(R), Section 3.2), the recycled Hessian solve (Section 2.2.2) with the
hypergradient-error stop (Section 4), and the hypergradient J w (Section 2.1).  The solves of
all requests in progress share one engine (bl_engine): a request is admitted as soon as the
engine has a free slot and an arena block for the solve's scratch (admission by bytes), its
iterations then run in the same kernel launches as everyone else's, and it retires when its
own stop test passes; its result does not depend on what else runs.  Requests of one sample
are served in arrival order (each needs the recycle space the previous one left behind).
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import bilevel as B


class Sample:
    """One resident training sample: its frozen outer steps and its recycle state."""

    def __init__(self, key, P, thetas, xhats, xstar, s: int, v_cap: int, device):
        self.key = key
        self.P = P                 # problem in the served precision
        self.P64 = B.bl_problem(*[getattr(P, f) for f, _ in B.bl_problem._fields_])
        self.P64.prec = B.BL_PREC_FP64
        self.thetas = thetas       # per outer step (host arrays)
        self.xhats = xhats         # per outer step (device tensors)
        self.xstar = xstar
        self.s = s
        self.rec = B.Recycle(P.h * P.w, s, v_cap, device, P)
        self.w = xstar.new_zeros(xstar.shape)
        self.step = 0              # next outer step to serve
        self.prev_hg = None
        self.busy = False

    def resident_bytes(self) -> int:
        return self.rec.nbytes() + self.w.numel() * 8


class Request:
    __slots__ = ("sample", "t_arrival", "step", "t_start", "t_ready", "t_admit", "t_solved", "t_done", "slot", "hg",
                 "stats", "g", "fut", "opts")

    def __init__(self, sample, t_arrival):
        self.sample = sample
        self.t_arrival = t_arrival
        self.step = -1
        self.t_start = self.t_ready = self.t_admit = self.t_solved = self.t_done = None
        self.slot = None
        self.hg = None
        self.stats = None
        self.g = None
        self.fut = None
        self.opts = None


class Server:
    """Continuous-batching server over resident samples: one engine (on the context's stream)
    for the solves; refreshes and hypergradients on `pool` (a ContextPool: other streams,
    other host threads) so that they overlap the engine's iterations, or inline without one."""

    def __init__(self, ctx: B.Context, cap: int, arena_bytes: int, hg_rel: float = 1e-9, tol: float = 1e-10,
                 rr_every: int = 50, iters_per_turn: int = 16, clock=time.perf_counter, pool=None,
                 check_every: int = 1, recycle: bool = True):
        """recycle=False serves plain warm-started CG: no refresh, every solve on the residual
        test at `tol` (the baseline the recycled form is compared with)."""
        self.ctx = ctx
        self.recycle = recycle
        self.engine = B.Engine(cap=cap, arena_bytes=arena_bytes, device=ctx.device, ctx=ctx.ctx)
        self.hg_rel = hg_rel
        self.tol = tol
        self.rr_every = rr_every
        self.check_every = check_every
        self.iters_per_turn = iters_per_turn
        self.clock = clock
        self.pool = pool
        self.samples = {}
        self.queue = collections.deque()   # arrived, not started
        self.preparing = []                # refresh submitted
        self.ready = collections.deque()   # refreshed, waiting for engine room
        self.running = {}                  # slot -> request
        self.finishing = []                # hypergradient submitted
        self.completed = []

    def add_sample(self, sample: Sample):
        self.samples[sample.key] = sample

    def resident_bytes(self) -> int:
        return sum(s.resident_bytes() for s in self.samples.values())

    def submit(self, key, t_arrival: float):
        self.queue.append(Request(self.samples[key], t_arrival))

    def _run(self, fn, *args):
        if self.pool is None:
            fn(self.ctx, *args)
            return None
        return self.pool.submit(fn, *args)

    # ---- stages
    def _prepare(self, req: Request):
        """Refresh the sample's recycle space for its next outer step (an empty space at the
        start of a pass over the sample's steps) and fix the solve options."""
        smp = req.sample
        step = smp.step % len(smp.thetas)
        req.step = step
        if step == 0:
            smp.rec.rs.s_cur = 0
            smp.rec.rs.v_cur = 0
            smp.prev_hg = None
            smp.w.zero_()
        req.t_start = self.clock()
        if step > 0 and self.recycle:
            req.fut = self._run(lambda c, P, rec, th, xh, s: c.refresh_p(P, rec, th, xh, s=s),
                                smp.P64, smp.rec, smp.thetas[step], smp.xhats[step], smp.s)

    def _admit(self, req: Request) -> bool:
        smp = req.sample
        use_hg = smp.rec.rs.s_cur > 0 and smp.prev_hg is not None
        opts = B.solve_opts(stop="hgerr" if use_hg else "resid", hg_tol=self.hg_rel * smp.prev_hg if use_hg else 0.0,
                            tol=self.tol, store_basis=self.recycle, rr_every=self.rr_every,
                            check_every=self.check_every if use_hg else 1)
        xh = smp.xhats[req.step]
        req.g = xh - smp.xstar
        slot = self.engine.admit(smp.P, smp.thetas[req.step], xh, req.g, smp.w, smp.rec, opts)
        if slot is None:
            return False
        req.slot = slot
        req.t_admit = self.clock()
        self.running[slot] = req
        return True

    def _complete(self, req: Request):
        smp = req.sample
        req.t_done = self.clock()
        smp.prev_hg = float(np.linalg.norm(req.hg))
        smp.step += 1
        smp.busy = False
        self.completed.append(req)

    def turn(self):
        """Start refreshes of queued requests whose sample is idle; admit refreshed ones while the
        engine has room; advance the engine a few iterations; finish completed solves."""
        out = []
        blocked = set()
        for req in list(self.queue):
            smp = req.sample
            if smp.busy or smp.key in blocked:
                blocked.add(smp.key)
                continue
            self.queue.remove(req)
            smp.busy = True
            self._prepare(req)
            self.preparing.append(req)
        for req in list(self.preparing):
            if req.fut is None or req.fut.done():
                if req.fut is not None:
                    req.fut.result()
                self.preparing.remove(req)
                req.t_ready = self.clock()
                self.ready.append(req)
        while self.ready:
            if not self._admit(self.ready[0]):
                break
            self.ready.popleft()
        if self.running:
            for slot in self.engine.step(max_iters=self.iters_per_turn, return_on_done=True):
                req = self.running.pop(slot)
                req.t_solved = self.clock()
                req.stats = self.engine.retire(slot)
                smp = req.sample
                if self.pool is None:
                    req.hg = self.ctx.hypergradient_p(smp.P64, smp.thetas[req.step], smp.xhats[req.step], smp.w)
                    self._complete(req)
                    out.append(req)
                else:
                    req.fut = self.pool.submit(lambda c, P, th, xh, w: c.hypergradient_p(P, th, xh, w),
                                               smp.P64, smp.thetas[req.step], smp.xhats[req.step], smp.w)
                    self.finishing.append(req)
        for req in list(self.finishing):
            if req.fut.done():
                req.hg = req.fut.result()
                self.finishing.remove(req)
                self._complete(req)
                out.append(req)
        return out

    def idle(self) -> bool:
        return not (self.queue or self.preparing or self.ready or self.running or self.finishing)

    def close(self):
        self.engine.close()
