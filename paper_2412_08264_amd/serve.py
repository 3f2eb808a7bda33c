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
        self.rec = B.Recycle(P.h * P.w, s, v_cap, device)
        self.w = xstar.new_zeros(xstar.shape)
        self.step = 0              # next outer step to serve
        self.prev_hg = None
        self.busy = False

    def resident_bytes(self) -> int:
        return self.rec.nbytes() + self.w.numel() * 8


class Request:
    __slots__ = ("sample", "t_arrival", "step", "t_start", "t_done", "slot", "hg", "stats", "g")

    def __init__(self, sample, t_arrival):
        self.sample = sample
        self.t_arrival = t_arrival
        self.step = -1
        self.t_start = self.t_done = None
        self.slot = None
        self.hg = None
        self.stats = None
        self.g = None


class Server:
    """Continuous-batching server over resident samples (one context, one engine, one stream)."""

    def __init__(self, ctx: B.Context, cap: int, arena_bytes: int, hg_rel: float = 1e-9, tol: float = 1e-10,
                 rr_every: int = 50, iters_per_turn: int = 16, clock=time.perf_counter):
        self.ctx = ctx
        self.engine = B.Engine(cap=cap, arena_bytes=arena_bytes, device=ctx.device, ctx=ctx.ctx)
        self.hg_rel = hg_rel
        self.tol = tol
        self.rr_every = rr_every
        self.iters_per_turn = iters_per_turn
        self.clock = clock
        self.samples = {}
        self.queue = collections.deque()
        self.running = {}
        self.completed = []

    def add_sample(self, sample: Sample):
        self.samples[sample.key] = sample

    def resident_bytes(self) -> int:
        return sum(s.resident_bytes() for s in self.samples.values())

    def submit(self, key, t_arrival: float):
        self.queue.append(Request(self.samples[key], t_arrival))

    def _start(self, req: Request) -> bool:
        """Refresh and admit; False (nothing changed) when the engine has no room."""
        smp = req.sample
        step = smp.step % len(smp.thetas)
        if step == 0:   # a new pass over the sample's outer steps starts from an empty space
            smp.rec.rs.s_cur = 0
            smp.rec.rs.v_cur = 0
            smp.prev_hg = None
            smp.w.zero_()
        need = B.Engine.slot_bytes(smp.P, smp.s if step > 0 else 0)
        _, free_slots, _, largest = self.engine.query()
        if free_slots == 0 or largest < need:
            return False
        th, xh = smp.thetas[step], smp.xhats[step]
        if step > 0:
            self.ctx.refresh_p(smp.P64, smp.rec, th, xh, s=smp.s)
        use_hg = smp.rec.rs.s_cur > 0 and smp.prev_hg is not None
        opts = B.solve_opts(stop="hgerr" if use_hg else "resid", hg_tol=self.hg_rel * smp.prev_hg if use_hg else 0.0,
                            tol=self.tol, store_basis=True, rr_every=self.rr_every)
        req.g = xh - smp.xstar
        slot = self.engine.admit(smp.P, th, xh, req.g, smp.w, smp.rec, opts)
        if slot is None:   # the refresh changed s_cur: retry later
            return False
        req.step = step
        req.slot = slot
        req.t_start = self.clock()
        smp.busy = True
        self.running[slot] = req
        return True

    def admit_waiting(self):
        """Start queued requests whose sample is idle, in arrival order, as far as room allows."""
        blocked = set()
        for req in list(self.queue):
            smp = req.sample
            if smp.busy or smp.key in blocked:
                blocked.add(smp.key)
                continue
            if not self._start(req):
                blocked.add(smp.key)
                continue
            self.queue.remove(req)

    def turn(self):
        """Admit what fits, advance the engine a few iterations, finish completed requests."""
        self.admit_waiting()
        if not self.running:
            return []
        done = self.engine.step(max_iters=self.iters_per_turn, return_on_done=True)
        out = []
        for slot in done:
            req = self.running.pop(slot)
            req.stats = self.engine.retire(slot)
            smp = req.sample
            req.hg = self.ctx.hypergradient_p(smp.P64, smp.thetas[req.step], smp.xhats[req.step], smp.w)
            req.t_done = self.clock()
            smp.prev_hg = float(np.linalg.norm(req.hg))
            smp.step += 1
            smp.busy = False
            out.append(req)
        self.completed += out
        return out

    def idle(self) -> bool:
        return not self.running and not self.queue

    def close(self):
        self.engine.close()
