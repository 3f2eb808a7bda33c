"""ctypes binding of libbilevel_hip.so (same names as the C ABI in include/bilevel.h).

Argument marshalling only: torch tensors provide device memory and the stream, every
step of the computation runs in the library's HIP kernels.  Importing this module
loads the library and fails loudly when it is missing or was built without GPU code.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: the library's HIP runtime dependency (libamdhip64.so.7) then resolves to the
# runtime torch has loaded, so the process holds one HIP runtime whatever the import order
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbilevel_hip.so")

BL_OK, BL_E_ARG, BL_E_SHAPE, BL_E_WORKSPACE, BL_E_NOT_CONVERGED = 0, 1, 2, 3, 4
BL_E_INDEFINITE, BL_E_BREAKDOWN, BL_E_RANK, BL_E_NONFINITE, BL_E_HIP = 5, 6, 7, 8, 9
BL_REG_TV, BL_REG_FILTERS = 0, 1
BL_PEN_LOG, BL_PEN_QUAD = 0, 1
BL_PREC_FP64, BL_PREC_MIXED = 0, 1
BL_STOP_RESID, BL_STOP_HGERR = 0, 1


class bl_problem(C.Structure):
    _fields_ = [("h", C.c_int), ("w", C.c_int), ("blur_radius", C.c_int), ("blur_sigma", C.c_double),
                ("reg", C.c_int), ("n_filters", C.c_int), ("filter_size", C.c_int), ("eps", C.c_double),
                ("penalty", C.c_int), ("prec", C.c_int)]


class bl_recycle(C.Structure):
    _fields_ = [("U", C.c_void_p), ("C", C.c_void_p), ("Z", C.c_void_p), ("mu", C.c_void_p), ("V", C.c_void_p),
                ("s_max", C.c_int), ("s_cur", C.c_int), ("v_cap", C.c_int), ("v_cur", C.c_int),
                ("lz", C.c_void_p), ("v_lz", C.c_int)]


class bl_solve_opts(C.Structure):
    _fields_ = [("stop", C.c_int), ("tol", C.c_double), ("hg_tol", C.c_double), ("max_iter", C.c_int),
                ("check_every", C.c_int), ("rr_every", C.c_int), ("store_basis", C.c_int)]


class bl_recycle_opts(C.Structure):
    _fields_ = [("s", C.c_int), ("rank_tol", C.c_double), ("select", C.c_int), ("inner", C.c_int)]


# selection rules of bl_select, by name
SELECTIONS = {"rgen-l-r": 0, "rgen-l-l": 1, "rgen-l-m": 2, "ritz-s": 3, "ritz-l": 4, "ritz-m": 5,
              "hritz-s": 6, "hritz-l": 7, "hritz-m": 8,
              "rgen-s-r": 9, "rgen-s-l": 10, "rgen-s-m": 11, "rgen-m-r": 12, "rgen-m-l": 13, "rgen-m-m": 14}


class bl_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("status", C.c_int), ("t", C.c_int), ("s_cur", C.c_int),
                ("res_norm", C.c_double), ("res0_norm", C.c_double), ("g_norm", C.c_double), ("est", C.c_double),
                ("ms", C.c_double * 4)]


_P = C.POINTER
_vp = C.c_void_p
_SIGS = {
    "bl_create": (C.c_int, [_P(_vp), _vp]),
    "bl_destroy": (C.c_int, [_vp]),
    "bl_status_string": (C.c_char_p, [C.c_int]),
    "bl_last_error": (C.c_char_p, [_vp]),
    "bl_num_params": (C.c_int, [_P(bl_problem)]),
    "bl_workspace_bytes": (C.c_size_t, [_P(bl_problem), C.c_int, C.c_int]),
    "bl_forward": (C.c_int, [_vp, _P(bl_problem), _vp, _vp, C.c_double, _vp, _vp, C.c_size_t]),
    "bl_lower_solve": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, C.c_double, C.c_int, C.c_int,
                                 _vp, C.c_size_t, _P(bl_stats)]),
    "bl_recycle_update": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _P(bl_recycle),
                                    _P(bl_recycle_opts), _vp, C.c_size_t, _P(bl_stats)]),
    "bl_hessian_solve": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, _P(bl_recycle),
                                   _P(bl_solve_opts), _vp, C.c_size_t, _P(bl_stats)]),
    "bl_hessian_solve_noalloc": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, _P(bl_recycle),
                                           _P(bl_solve_opts), _P(bl_stats)]),
    "bl_hessian_solve_deflated": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, _P(bl_recycle),
                                            _P(bl_solve_opts), _vp, C.c_size_t, _P(bl_stats)]),
    "bl_hessian_solve_rminres": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, _P(bl_recycle),
                                           _P(bl_solve_opts), _vp, C.c_size_t, _P(bl_stats)]),
    "bl_hypergradient": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _P(C.c_double), C.c_int,
                                   _vp, C.c_size_t]),
    "bl_hvp": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, C.c_int, _vp, C.c_size_t]),
    "bl_lower_grad": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, _P(C.c_double), _vp,
                                C.c_size_t]),
    "bl_set_timing": (C.c_int, [_vp, C.c_int]),
    "bl_set_graphs": (C.c_int, [_vp, C.c_int]),
    "bl_graph_counts": (C.c_int, [_vp, _P(C.c_longlong), _P(C.c_longlong)]),
    "bl_kernel_times": (C.c_int, [_vp, _P(C.c_double), C.c_int]),
    "bl_engine_slot_bytes": (C.c_size_t, [_P(bl_problem), C.c_int]),
    "bl_engine_workspace_bytes": (C.c_size_t, [C.c_int, C.c_size_t]),
    "bl_engine_create": (C.c_int, [_vp, C.c_int, _vp, C.c_size_t, _P(_vp)]),
    "bl_engine_destroy": (C.c_int, [_vp]),
    "bl_engine_admit": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, _vp, _vp, _P(bl_recycle),
                                  _P(bl_solve_opts), _P(C.c_int)]),
    "bl_engine_step": (C.c_int, [_vp, C.c_int, C.c_int, _P(C.c_int), _P(C.c_int)]),
    "bl_engine_retire": (C.c_int, [_vp, C.c_int, _P(bl_stats)]),
    "bl_engine_query": (C.c_int, [_vp, _P(C.c_int), _P(C.c_int), _P(C.c_size_t), _P(C.c_size_t)]),
    "bl_batched_workspace_bytes": (C.c_size_t, [C.c_int, _P(bl_problem), _P(C.c_int)]),
    "bl_hessian_solve_batched": (C.c_int, [_vp, C.c_int, _P(bl_problem), _P(_P(C.c_double)), _P(_vp), _P(_vp),
                                           _P(_vp), _P(bl_recycle), _P(bl_solve_opts), _vp, C.c_size_t,
                                           _P(bl_stats)]),
    "bl_tile_rows_set": (C.c_int, [_P(bl_problem), C.c_int]),
    "bl_tile_rows": (C.c_int, [_P(bl_problem)]),
    "bl_autotune_workspace_bytes": (C.c_size_t, [_P(bl_problem), C.c_int]),
    "bl_autotune": (C.c_int, [_vp, _P(bl_problem), _P(C.c_double), _vp, C.c_int, C.c_int, C.c_char_p, _vp,
                              C.c_size_t, _P(C.c_int), _P(C.c_double)]),
    "bl_tile_cache_load": (C.c_int, [C.c_char_p, _P(C.c_int)]),
    "bl_recycle_bytes": (C.c_size_t, [_P(bl_problem), C.c_int, C.c_int]),
    "bl_recycle_init": (C.c_int, [_P(bl_problem), C.c_int, C.c_int, _vp, C.c_size_t, _P(bl_recycle)]),
}
EXPORTED = tuple(_SIGS)


def load_library(path: str = _LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load_library()


class BLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{lib.bl_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _theta(theta) -> C.Array:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    return (C.c_double * th.size)(*th.tolist())


def problem_from(wl, prec: str | None = None, penalty: str = "log") -> bl_problem:
    """bl_problem of a synthetic workload recipe."""
    prec = prec or wl.prec
    return bl_problem(wl.h, wl.w, wl.blur_radius, wl.blur_sigma,
                      BL_REG_TV if wl.reg == "tv" else BL_REG_FILTERS,
                      wl.n_filters, wl.filter_size, wl.eps,
                      BL_PEN_LOG if penalty == "log" else BL_PEN_QUAD,
                      BL_PREC_MIXED if prec == "mixed" else BL_PREC_FP64)


# --------------------------------------------------------------------------- same-name wrappers
def bl_create(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    ctx = C.c_void_p()
    st = lib.bl_create(C.byref(ctx), C.c_void_p(s.cuda_stream))
    if st != BL_OK:
        raise BLError(st, "bl_create")
    return ctx


def bl_destroy(ctx) -> None:
    lib.bl_destroy(ctx)


def bl_workspace_bytes(P: bl_problem, s_max: int, v_cap: int) -> int:
    return int(lib.bl_workspace_bytes(C.byref(P), s_max, v_cap))


def bl_num_params(P: bl_problem) -> int:
    return int(lib.bl_num_params(C.byref(P)))


def _check(ctx, st: int, name: str, ok=(BL_OK,)) -> int:
    if st not in ok:
        raise BLError(st, f"{name}: {lib.bl_last_error(ctx).decode()}")
    return st


def bl_tile_rows_set(P: bl_problem, rows: int) -> None:
    """Tile height (8, 16, 32; 0 clears) of the solves of P's operator class and size class."""
    st = lib.bl_tile_rows_set(C.byref(P), int(rows))
    if st != BL_OK:
        raise BLError(st, "bl_tile_rows_set")


def bl_tile_rows(P: bl_problem) -> int:
    return int(lib.bl_tile_rows(C.byref(P)))


def bl_tile_cache_load(path: str) -> int:
    """Entries of a tile cache file (written by bl_autotune) into the tile table; their count."""
    k = C.c_int(0)
    st = lib.bl_tile_cache_load(path.encode(), C.byref(k))
    if st != BL_OK:
        raise BLError(st, f"bl_tile_cache_load({path})")
    return k.value


class Context:
    """Context + workspace for problems up to the given shapes; every call names its problem
    and recycle storage explicitly (torch tensors on one device)."""

    def __init__(self, problems, s_max: int = 0, v_cap: int = 0, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ctx = bl_create(self.stream)
            sizes = [bl_workspace_bytes(P, s_max, v_cap) for P in problems]
            if not sizes or min(sizes) == 0:
                raise BLError(BL_E_ARG, "bl_workspace_bytes rejected a shape")
            nbytes = max(sizes)
            self.ws, self.ws_ptr = _aligned_workspace(nbytes, self.device)
            self.ws_bytes = nbytes

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def close(self):
        if getattr(self, "ctx", None) is not None:
            bl_destroy(self.ctx)
            self.ctx = None

    def set_timing(self, mode: int = 1):
        lib.bl_set_timing(self.ctx, int(mode))

    def set_graphs(self, enable: bool = True):
        """Replay repeated chunks of Krylov iterations from captured HIP graphs (default on)."""
        lib.bl_set_graphs(self.ctx, 1 if enable else 0)

    def graph_counts(self):
        """(chunks captured, chunk replays) on this context."""
        cap, rep = C.c_longlong(), C.c_longlong()
        lib.bl_graph_counts(self.ctx, C.byref(cap), C.byref(rep))
        return cap.value, rep.value

    def kernel_times(self, reset: bool = True):
        """(apply ms total, apply launches, update ms total, update launches)."""
        out = (C.c_double * 4)()
        lib.bl_kernel_times(self.ctx, out, 1 if reset else 0)
        return tuple(out[:])

    def autotune_tiles(self, P, theta, xhat, s: int, iters: int = 100, cache_path: str | None = None):
        """bl_autotune: time every tile height on a solve of P at (theta, xhat) and keep the fastest
        for P's operator class and size class (or take the stored height from cache_path, and store
        a new result there).  Returns (rows, microseconds per iteration at 8/16/32; zeros when the
        height came from the cache)."""
        us = (C.c_double * 3)()
        best = C.c_int()
        nbytes = int(lib.bl_autotune_workspace_bytes(C.byref(P), int(s)))
        if nbytes == 0:
            raise BLError(BL_E_ARG, "bl_autotune_workspace_bytes rejected the shape")
        with self.torch.cuda.device(self.device):
            ws, wsp = _aligned_workspace(nbytes, self.device)
        path = cache_path.encode() if cache_path is not None else None
        _check(self.ctx, lib.bl_autotune(self.ctx, C.byref(P), _theta(theta), _ptr(xhat), int(s), int(iters), path,
                                         wsp, nbytes, C.byref(best), us), "bl_autotune")
        del ws
        return best.value, tuple(us[:])

    # -- calls
    def forward_p(self, P, x, e, noise, y):
        _check(self.ctx, lib.bl_forward(self.ctx, C.byref(P), _ptr(x), _ptr(e), noise, _ptr(y),
                                        self.ws_ptr, self.ws_bytes), "bl_forward")

    def hvp_p(self, P, theta, xhat, v, out, ncols: int = 1):
        _check(self.ctx, lib.bl_hvp(self.ctx, C.byref(P), _theta(theta), _ptr(xhat), _ptr(v), _ptr(out),
                                    ncols, self.ws_ptr, self.ws_bytes), "bl_hvp")

    def lower_grad_p(self, P, theta, y, x, grad) -> float:
        phi = C.c_double()
        _check(self.ctx, lib.bl_lower_grad(self.ctx, C.byref(P), _theta(theta), _ptr(y), _ptr(x), _ptr(grad),
                                           C.byref(phi), self.ws_ptr, self.ws_bytes), "bl_lower_grad")
        return phi.value

    def lower_solve_p(self, P, theta, y, x, gtol=1e-8, max_iter=20000, m=10) -> bl_stats:
        st = bl_stats()
        _check(self.ctx, lib.bl_lower_solve(self.ctx, C.byref(P), _theta(theta), _ptr(y), _ptr(x), gtol,
                                            max_iter, m, self.ws_ptr, self.ws_bytes, C.byref(st)),
               "bl_lower_solve", ok=(BL_OK, BL_E_NOT_CONVERGED))
        return st

    def refresh_p(self, P, rec, theta, xhat, s: int, rank_tol: float = 1e-8, select: str = "rgen-l-r",
                  inner: bool = False) -> bl_stats:
        st = bl_stats()
        o = bl_recycle_opts(s, rank_tol, SELECTIONS[select], 1 if inner else 0)
        _check(self.ctx, lib.bl_recycle_update(self.ctx, C.byref(P), _theta(theta), _ptr(xhat),
                                               C.byref(rec.rs), C.byref(o), self.ws_ptr, self.ws_bytes,
                                               C.byref(st)), "bl_recycle_update", ok=(BL_OK, BL_E_RANK))
        return st

    def solve_p(self, P, rec, theta, xhat, g, w, tol=1e-10, stop: str = "resid", hg_tol: float = 0.0,
                max_iter: int = 20000, check_every: int = 1, rr_every: int = 50, store_basis: bool = True,
                recycle: bool = True, allow=(BL_OK,), method: str = "cg") -> bl_stats:
        """Hessian solve by recycled CG (``method="cg"``), RMINRES (``method="rminres"``) or
        deflated CG (``method="deflated"``)."""
        fns = {"cg": (lib.bl_hessian_solve, "bl_hessian_solve"),
               "rminres": (lib.bl_hessian_solve_rminres, "bl_hessian_solve_rminres"),
               "deflated": (lib.bl_hessian_solve_deflated, "bl_hessian_solve_deflated")}
        if method not in fns:
            raise ValueError(f"unknown method {method!r}")
        fn, name = fns[method]
        st = bl_stats()
        o = bl_solve_opts(BL_STOP_HGERR if stop == "hgerr" else BL_STOP_RESID, tol, hg_tol, max_iter, check_every,
                          rr_every, 1 if store_basis else 0)
        rs = rec.rs if rec is not None and (recycle or store_basis) else None
        saved = None
        if rs is not None and not recycle:
            saved, rs.s_cur = rs.s_cur, 0
        try:
            code = fn(self.ctx, C.byref(P), _theta(theta), _ptr(xhat), _ptr(g), _ptr(w),
                      C.byref(rs) if rs is not None else None, C.byref(o), self.ws_ptr, self.ws_bytes, C.byref(st))
        finally:
            if saved is not None:
                rs.s_cur = saved
        _check(self.ctx, code, name, ok=allow)
        return st

    def hypergradient_p(self, P, theta, xhat, w, project: bool = True) -> np.ndarray:
        out = (C.c_double * bl_num_params(P))()
        _check(self.ctx, lib.bl_hypergradient(self.ctx, C.byref(P), _theta(theta), _ptr(xhat), _ptr(w), out,
                                              1 if project else 0, self.ws_ptr, self.ws_bytes), "bl_hypergradient")
        return np.array(out[:], dtype=np.float64)


class Session(Context):
    """Context + workspace + recycle storage of one problem shape."""

    def __init__(self, P: bl_problem, s_max: int = 0, v_cap: int = 0, device=None, stream=None):
        super().__init__([P], s_max, v_cap, device, stream)
        self.P = P
        self.n = P.h * P.w
        self.p = bl_num_params(P)
        self.rec = Recycle(self.n, s_max, v_cap, self.device, P)
        self.U, self.Cm, self.Z, self.mu, self.V = self.rec.U, self.rec.Cm, self.rec.Z, self.rec.mu, self.rec.V
        self.lz = self.rec.lz
        self.rs = self.rec.rs

    def reset(self):
        self.rs.s_cur = 0
        self.rs.v_cur = 0
        self.rs.v_lz = 0

    def forward(self, x, e, noise, y):
        self.forward_p(self.P, x, e, noise, y)

    def hvp(self, theta, xhat, v, out, ncols: int = 1):
        self.hvp_p(self.P, theta, xhat, v, out, ncols)

    def lower_grad(self, theta, y, x, grad) -> float:
        return self.lower_grad_p(self.P, theta, y, x, grad)

    def lower_solve(self, theta, y, x, gtol=1e-8, max_iter=20000, m=10) -> bl_stats:
        return self.lower_solve_p(self.P, theta, y, x, gtol, max_iter, m)

    def refresh(self, theta, xhat, s: int, rank_tol: float = 1e-8, select: str = "rgen-l-r",
                inner: bool = False) -> bl_stats:
        return self.refresh_p(self.P, self.rec, theta, xhat, s, rank_tol, select, inner)

    def solve(self, theta, xhat, g, w, **kw) -> bl_stats:
        return self.solve_p(self.P, self.rec, theta, xhat, g, w, **kw)

    def hypergradient(self, theta, xhat, w, project: bool = True) -> np.ndarray:
        return self.hypergradient_p(self.P, theta, xhat, w, project)


# --------------------------------------------------------------------------- recycle storage
class Recycle:
    """Device storage of one sample's recycle state, one buffer of bl_recycle_bytes() carved by
    bl_recycle_init: U, C, Z (s_max x n), mu, V (v_cap x n), exposed as tensor views."""

    def __init__(self, n: int, s_max: int, v_cap: int, device, P: bl_problem | None = None):
        import torch
        if P is None:   # the layout depends on n only: any valid problem of n pixels
            if n % 2:
                raise ValueError("Recycle: pass the problem P for an odd pixel count")
            P = bl_problem(2, n // 2, 0, 1.0, BL_REG_TV, 0, 0, 0.0, BL_PEN_LOG, BL_PREC_FP64)
        elif P.h * P.w != n:
            raise ValueError("Recycle: n differs from P.h * P.w")
        self.n = n
        nbytes = int(lib.bl_recycle_bytes(C.byref(P), int(s_max), int(v_cap)))
        if nbytes == 0:
            raise BLError(BL_E_SHAPE, f"bl_recycle_bytes rejected s_max={s_max}, v_cap={v_cap}")
        self.buf, base = _aligned_workspace(nbytes, device)
        self.rs = bl_recycle()
        st = lib.bl_recycle_init(C.byref(P), int(s_max), int(v_cap), base, nbytes, C.byref(self.rs))
        if st != BL_OK:
            raise BLError(st, "bl_recycle_init")
        self.buf.zero_()
        off = lambda p: (p or base) - self.buf.data_ptr()
        view = lambda p, rows: self.buf[off(p):off(p) + 8 * rows * n].view(torch.float64).view(rows, n)
        self.U = view(self.rs.U, s_max)
        self.Cm = view(self.rs.C, s_max)
        self.Z = view(self.rs.Z, s_max)
        self.mu = self.buf[off(self.rs.mu):off(self.rs.mu) + 8 * s_max].view(torch.float64)
        self.V = view(self.rs.V, v_cap) if v_cap > 0 else self.buf[:0].view(torch.float64).view(0, n)
        self.lz = (self.buf[off(self.rs.lz):off(self.rs.lz) + 16 * v_cap].view(torch.float64) if v_cap > 0
                   else self.buf[:0].view(torch.float64))
        self._nbytes = nbytes

    def nbytes(self) -> int:
        return self._nbytes


def solve_opts(tol=1e-10, stop: str = "resid", hg_tol: float = 0.0, max_iter: int = 20000, check_every: int = 1,
               rr_every: int = 50, store_basis: bool = True) -> bl_solve_opts:
    return bl_solve_opts(BL_STOP_HGERR if stop == "hgerr" else BL_STOP_RESID, tol, hg_tol, max_iter, check_every,
                         rr_every, 1 if store_basis else 0)


def _aligned_workspace(nbytes: int, device):
    import torch
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return ws, ws.data_ptr() + (-ws.data_ptr()) % 256


# --------------------------------------------------------------------------- batched / served solves
class Engine:
    """bl_engine: up to `cap` concurrent solves (up to 16 groups of operator class, tile height and
    recycling) advanced together."""

    def __init__(self, cap: int, arena_bytes: int, device=None, stream=None, ctx=None):
        import torch
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.cap = cap
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._own_ctx = ctx is None
            self.ctx = ctx if ctx is not None else bl_create(self.stream)
            nbytes = int(lib.bl_engine_workspace_bytes(cap, arena_bytes))
            if nbytes == 0:
                raise BLError(BL_E_ARG, "bl_engine_workspace_bytes rejected the capacity")
            self.ws, self.ws_ptr = _aligned_workspace(nbytes, self.device)
        self.handle = C.c_void_p()
        _check(self.ctx, lib.bl_engine_create(self.ctx, cap, self.ws_ptr, nbytes, C.byref(self.handle)),
               "bl_engine_create")
        self._held = {}
        self._done = (C.c_int * cap)()

    @staticmethod
    def slot_bytes(P: bl_problem, s: int) -> int:
        return int(lib.bl_engine_slot_bytes(C.byref(P), s))

    def admit(self, P: bl_problem, theta, xhat, g, w, rec: Recycle | None, opts: bl_solve_opts) -> int | None:
        """Slot of the admitted solve, or None when no slot or arena block is free."""
        slot = C.c_int(-1)
        code = lib.bl_engine_admit(self.handle, C.byref(P), _theta(theta), _ptr(xhat), _ptr(g), _ptr(w),
                                   C.byref(rec.rs) if rec is not None else None, C.byref(opts), C.byref(slot))
        if code == BL_E_WORKSPACE:
            return None
        _check(self.ctx, code, "bl_engine_admit")
        self._held[slot.value] = (P, xhat, g, w, rec)
        return slot.value

    def step(self, max_iters: int = 1 << 30, return_on_done: bool = True) -> list:
        nd = C.c_int(0)
        _check(self.ctx, lib.bl_engine_step(self.handle, max_iters, 1 if return_on_done else 0, self._done,
                                            C.byref(nd)), "bl_engine_step")
        return list(self._done[:nd.value])

    def retire(self, slot: int) -> bl_stats:
        st = bl_stats()
        code = lib.bl_engine_retire(self.handle, slot, C.byref(st))
        if code in (BL_E_ARG,):
            _check(self.ctx, code, "bl_engine_retire")
        self._held.pop(slot, None)
        return st

    def query(self):
        r, f = C.c_int(), C.c_int()
        fb, lf = C.c_size_t(), C.c_size_t()
        _check(self.ctx, lib.bl_engine_query(self.handle, C.byref(r), C.byref(f), C.byref(fb), C.byref(lf)),
               "bl_engine_query")
        return r.value, f.value, fb.value, lf.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.bl_engine_destroy(self.handle)
            self.handle = None
        if getattr(self, "_own_ctx", False) and getattr(self, "ctx", None) is not None:
            bl_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def hessian_solve_batched(problems, thetas, xhats, gs, ws_, recs, opts: bl_solve_opts, device=None, stream=None,
                          ctx=None):
    """bl_hessian_solve_batched over lists of problems / thetas / tensors (recs: list of Recycle or None).
    Returns (status, [bl_stats])."""
    import torch
    k = len(problems)
    device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    Parr = (bl_problem * k)(*problems)
    svals = (C.c_int * k)(*[(r.rs.s_cur if r is not None else 0) for r in recs])
    nbytes = int(lib.bl_batched_workspace_bytes(k, Parr, svals))
    if nbytes == 0:
        raise BLError(BL_E_ARG, "bl_batched_workspace_bytes rejected the batch")
    with torch.cuda.device(device):
        stream = stream if stream is not None else torch.cuda.current_stream(device)
        own = ctx is None
        ctx = ctx if ctx is not None else bl_create(stream)
        ws, wsp = _aligned_workspace(nbytes, device)
    try:
        th = [_theta(t) for t in thetas]
        tharr = (_P(C.c_double) * k)(*[C.cast(t, _P(C.c_double)) for t in th])
        xa = (_vp * k)(*[_ptr(t) for t in xhats])
        ga = (_vp * k)(*[_ptr(t) for t in gs])
        wa = (_vp * k)(*[_ptr(t) for t in ws_])
        any_rec = any(r is not None for r in recs)
        empty = bl_recycle(None, None, None, None, None, 0, 0, 0, 0, None, 0)
        rsarr = (bl_recycle * k)(*[(r.rs if r is not None else empty) for r in recs]) if any_rec else None
        out = (bl_stats * k)()
        code = lib.bl_hessian_solve_batched(ctx, k, Parr, tharr, xa, ga, wa, rsarr, C.byref(opts), wsp, nbytes, out)
        if code in (BL_E_ARG, BL_E_SHAPE, BL_E_WORKSPACE, BL_E_HIP):
            _check(ctx, code, "bl_hessian_solve_batched")
        if rsarr is not None:   # v_cur written into the array copies
            for r, rr in zip(recs, rsarr):
                if r is not None:
                    r.rs.v_cur = rr.v_cur
                    r.rs.v_lz = rr.v_lz
        return code, list(out)
    finally:
        if own:
            bl_destroy(ctx)


class ContextPool:
    """Several contexts, each with its own HIP stream (default priority) and workspace, driven by
    as many host threads: independent per-sample calls (refreshes, hypergradients, lower solves)
    run concurrently on the GPU.  Every call synchronises its own stream before it returns, so a
    result is complete when its future is."""

    def __init__(self, problems, s_max: int, v_cap: int, workers: int, device=None):
        import queue
        from concurrent.futures import ThreadPoolExecutor

        import torch
        device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ctxs = [Context(problems, s_max, v_cap, device, stream=torch.cuda.Stream(device)) for _ in range(workers)]
        self._free = queue.Queue()
        for c in self.ctxs:
            self._free.put(c)
        self._ex = ThreadPoolExecutor(max_workers=workers)

    def submit(self, fn, *args):
        """fn(context, *args) on a free context; returns a future."""
        def run():
            c = self._free.get()
            try:
                return fn(c, *args)
            finally:
                self._free.put(c)
        return self._ex.submit(run)

    def map(self, fn, arg_tuples) -> list:
        futs = [self.submit(fn, *a) for a in arg_tuples]
        return [f.result() for f in futs]

    def close(self):
        self._ex.shutdown(wait=True)
        for c in self.ctxs:
            c.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
