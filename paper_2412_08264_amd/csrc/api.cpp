// Host side of the C ABI: argument validation, workspace carving and kernel orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "host.h"
#include "tile.h"

using namespace bl;
using namespace blh;

namespace {

constexpr int LBFGS_MMAX = 20;

// Workspace layout (all offsets in bytes from the workspace base).
struct Layout {
    size_t state, mstate, slots, ctr, fold, part, vec, maps, taps, mhc, W0, W1, Ut, Ct, small, lb, total;
    size_t part_doubles;
    int n, p, s_max, v_cap, t_max, nf;
};

// solve_only: the part a Hessian solve uses (state, records, vectors, filter maps and taps);
// the refresh and lower-level scratch after it has size zero.
Layout layout(const bl_problem* P, int s_max, int v_cap, bool solve_only = false) {
    Layout L{};
    L.n = P->h * P->w;
    L.p = nparams(P);
    L.s_max = s_max;
    L.v_cap = v_cap;
    L.t_max = s_max + v_cap;
    L.nf = P->reg == BL_REG_FILTERS ? P->n_filters : 0;
    const int tiles = ((P->w + TW - 1) / TW) * ((P->h + TH - 1) / TH);
    size_t pd = (size_t)std::max(tiles, (L.n + NT - 1) / NT) * (size_t)NV_RED;
    pd = std::max(pd, (size_t)gram_chunks(L.n) * L.t_max * L.t_max);
    pd = std::max(pd, (size_t)256 * L.t_max * std::max(L.p, 2));
    pd = std::max(pd, (size_t)RED_BLOCKS * 4);
    L.part_doubles = pd;
    size_t o = 0;
    L.state = o;    o += al(sizeof(SolveState));
    L.mstate = o;   o += al(sizeof(MinresState));
    L.slots = o;    o += al(sizeof(Slot));
    L.ctr = o;      o += al(sizeof(int));
    L.fold = o;     o += al((size_t)3 * FOLD_BLOCKS * NV_RED * sizeof(double));
    L.part = o;     o += al(4 * pd * sizeof(double));   // records: residual / apply / update / apply of odd fused steps
    L.vec = o;      o += al(((size_t)8 * L.n + 2 * L.p) * sizeof(double));   // 8 vectors + a p-vector
    L.maps = o;     o += al((size_t)L.nf * L.n * (2 * sizeof(double) + sizeof(float)));
    L.taps = o;     o += al(TAPS_BYTES);
    L.mhc = o;      o += al((size_t)s_max * s_max * sizeof(double));   // the solve's C^T H C
    if (solve_only) {   // the solve's H C (n x s_max) in the place of the refresh's U~
        L.W0 = L.W1 = L.Ct = L.small = L.lb = L.Ut = o;
        o += al((size_t)L.n * std::max(s_max, 1) * sizeof(double));
        L.total = o;
        return L;
    }
    L.W0 = o;       o += al((size_t)L.n * L.t_max * sizeof(double));
    L.W1 = o;       o += al((size_t)L.n * L.t_max * sizeof(double));
    L.Ut = o;       o += al((size_t)L.n * std::max(s_max, 1) * sizeof(double));
    L.Ct = o;       o += al((size_t)L.n * std::max(s_max, 1) * sizeof(double));
    const size_t T2 = (size_t)L.t_max * L.t_max;
    L.small = o;
    o += al((9 * T2 + (size_t)L.p * L.t_max + 2 * (size_t)L.t_max * std::max(s_max, 1) + 256 +
             gsvd_scratch_doubles(L.t_max, L.p)) * sizeof(double) + 4 * L.t_max * sizeof(int));
    L.lb = o;       o += al(((size_t)2 * (LBFGS_MMAX + 1) * L.n + (size_t)(LBFGS_MMAX + 6) * 1024 + 64) * sizeof(double));
    L.total = o;
    return L;
}

struct WS {
    Layout L;
    char* base;
    SolveState* st() const { return (SolveState*)(base + L.state); }
    MinresState* mst() const { return (MinresState*)(base + L.mstate); }
    Slot* slots() const { return (Slot*)(base + L.slots); }
    int* ctr() const { return (int*)(base + L.ctr); }
    double* part() const { return (double*)(base + L.part); }
    double* part_res() const { return part(); }
    double* part_app() const { return part() + L.part_doubles; }
    double* part_upd() const { return part() + 2 * L.part_doubles; }
    double* part_app2() const { return part() + 3 * L.part_doubles; }
    double* part_fold(int k) const { return (double*)(base + L.fold) + (size_t)k * FOLD_BLOCKS * NV_RED; }
    double* vec(int k) const { return (double*)(base + L.vec) + (size_t)k * L.n; }
    double* d1() const { return (double*)(base + L.maps); }
    double* d2() const { return d1() + (size_t)L.nf * L.n; }
    float* d2f() const { return (float*)(d2() + (size_t)L.nf * L.n); }
    double* taps() const { return (double*)(base + L.taps); }
    double* mhc() const { return (double*)(base + L.mhc); }
    double* W0() const { return (double*)(base + L.W0); }
    double* W1() const { return (double*)(base + L.W1); }
    double* Ut() const { return (double*)(base + L.Ut); }
    double* Ct() const { return (double*)(base + L.Ct); }
    double* small(size_t off) const { return (double*)(base + L.small) + off; }
    double* lb() const { return (double*)(base + L.lb); }
};

bl_status check_ws(bl_ctx* c, const Layout& L, void* ws, size_t ws_bytes, WS& out) {
    if (!ws) return c->err = "null workspace", BL_E_WORKSPACE;
    if (ws_bytes < L.total) return c->err = "workspace smaller than bl_workspace_bytes()", BL_E_WORKSPACE;
    if ((uintptr_t)ws % ALIGN) return c->err = "workspace must be 256-byte aligned", BL_E_WORKSPACE;
    out.L = L;
    out.base = (char*)ws;
    return BL_OK;
}

// Stencil description at (theta); filters: taps and weights copied to the workspace.
bl_status make_stencil(bl_ctx* c, const bl_problem* P, const double* theta, const WS& ws, Stencil& S) {
    class_stencil(P, S);
    S.h = P->h;
    S.w = P->w;
    S.n = P->h * P->w;
    S.tiles_x = (P->w + TW - 1) / TW;
    S.tiles_y = (P->h + TH - 1) / TH;
    TRY(theta_values(c, P, theta, S.lam, S.gam2, c->h_buf));
    if (P->reg == BL_REG_FILTERS) {
        const int f2 = S.fs * S.fs;
        HIPCHK(hipMemcpyAsync(ws.taps(), c->h_buf, TAPS_MAX * sizeof(double) + (S.nf * f2 + S.nf) * sizeof(float),
                              hipMemcpyHostToDevice, c->stream));
        // the staging buffer is reused by later calls: make the copy complete
        HIPCHK(hipStreamSynchronize(c->stream));
        S.taps = ws.taps();
        S.tapsf = reinterpret_cast<const float*>(ws.taps() + TAPS_MAX);
        S.lamj = ws.taps() + S.nf * f2;
        S.d2 = ws.d2();
        S.d2f = ws.d2f();
    }
    return BL_OK;
}

bl_status filter_state(bl_ctx* c, const Stencil& S, const double* xhat, const WS& ws) {
    if (S.reg != BL_REG_FILTERS) return BL_OK;
    HIPCHK(launch_filter_state(S, xhat, ws.d1(), ws.d2(), ws.d2f(), c->stream));
    return BL_OK;
}

void mark(bl_ctx* c, int k) {
    if (c->timing) hipEventRecord(c->ev[k], c->stream);
}

float elapsed(bl_ctx* c, int a, int b) {
    float ms = 0.f;
    if (c->timing) hipEventElapsedTime(&ms, c->ev[a], c->ev[b]);
    return ms;
}

}  // namespace

extern "C" {

bl_status bl_create(bl_ctx** ctx, void* hip_stream) {
    if (!ctx) return BL_E_ARG;
    bl_ctx* c = new bl_ctx();
    c->stream = (hipStream_t)hip_stream;
    if (hipHostMalloc((void**)&c->h_state, sizeof(SolveState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_buf, 8192 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_info, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_hdr, 2 * HDR_BYTES, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return BL_E_HIP;
    }
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return BL_E_HIP;
    for (auto& e : c->poll_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return BL_E_HIP;
    *ctx = c;
    return BL_OK;
}

bl_status bl_destroy(bl_ctx* c) {
    if (!c) return BL_E_ARG;
    hipStreamSynchronize(c->stream);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    for (auto& e : c->ev)
        if (e) hipEventDestroy(e);
    for (auto& e : c->kev) hipEventDestroy(e);
    for (auto& e : c->poll_ev)
        if (e) hipEventDestroy(e);
    if (c->h_hdr) hipHostFree(c->h_hdr);
    if (c->h_state) hipHostFree(c->h_state);
    if (c->h_buf) hipHostFree(c->h_buf);
    if (c->h_info) hipHostFree(c->h_info);
    delete c;
    return BL_OK;
}

const char* bl_status_string(int s) {
    switch (s) {
        case BL_OK: return "ok";
        case BL_E_ARG: return "invalid argument";
        case BL_E_SHAPE: return "inconsistent shape";
        case BL_E_WORKSPACE: return "workspace too small or missing";
        case BL_E_NOT_CONVERGED: return "iteration limit reached";
        case BL_E_INDEFINITE: return "non-positive curvature (indefinite Hessian)";
        case BL_E_BREAKDOWN: return "breakdown";
        case BL_E_RANK: return "rank deficiency: columns dropped";
        case BL_E_NONFINITE: return "non-finite value";
        case BL_E_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* bl_last_error(const bl_ctx* c) { return c ? c->err.c_str() : "null context"; }

int bl_num_params(const bl_problem* P) { return P ? nparams(P) : -1; }

size_t bl_workspace_bytes(const bl_problem* P, int s_max, int v_cap) {
    if (!P || s_max < 0 || v_cap < 0 || s_max > S_MAX || s_max + v_cap > 256) return 0;
    return layout(P, s_max, v_cap).total;
}

bl_status bl_set_graphs(bl_ctx* c, int enable) {
    if (!c) return BL_E_ARG;
    c->graphs = enable ? 1 : 0;
    return BL_OK;
}

bl_status bl_graph_counts(const bl_ctx* c, long long* captured, long long* replayed) {
    if (!c) return BL_E_ARG;
    if (captured) *captured = c->graph_captures;
    if (replayed) *replayed = c->graph_replays;
    return BL_OK;
}

bl_status bl_set_timing(bl_ctx* c, int enable) {
    if (!c) return BL_E_ARG;
    c->timing = enable < 0 ? 0 : (enable > 2 ? 2 : enable);
    return BL_OK;
}

bl_status bl_kernel_times(bl_ctx* c, double* out4, int reset) {
    if (!c || !out4) return BL_E_ARG;
    for (int k = 0; k < 4; ++k) out4[k] = c->kt[k];
    if (reset)
        for (double& v : c->kt) v = 0.0;
    return BL_OK;
}

bl_status bl_forward(bl_ctx* c, const bl_problem* P, const double* x, const double* e, double noise, double* y,
                     void* wsp, size_t ws_bytes) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!x || !e || !y) return c->err = "null vector", BL_E_ARG;
    WS ws;
    TRY(check_ws(c, layout(P, 0, 0), wsp, ws_bytes, ws));
    double th[2] = {0.0, 0.0};
    bl_problem Q = *P;
    Q.reg = BL_REG_TV;
    Stencil S;
    TRY(make_stencil(c, &Q, th, ws, S));
    HIPCHK(launch_forward(S, x, e, noise, y, c->stream));
    return BL_OK;
}

bl_status bl_hvp(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, const double* v,
                 double* out, int ncols, void* wsp, size_t ws_bytes) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !v || !out || ncols < 1) return c->err = "null vector or ncols < 1", BL_E_ARG;
    WS ws;
    TRY(check_ws(c, layout(P, 0, 0), wsp, ws_bytes, ws));
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    TRY(filter_state(c, S, xhat, ws));
    HIPCHK(launch_hvp(S, P->prec == BL_PREC_MIXED, xhat, v, out, ncols, tile_rows(P), c->stream));
    return BL_OK;
}

bl_status bl_lower_grad(bl_ctx* c, const bl_problem* P, const double* theta, const double* y, const double* x,
                        double* grad, double* phi_host, void* wsp, size_t ws_bytes) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!y || !x || !grad) return c->err = "null vector", BL_E_ARG;
    WS ws;
    TRY(check_ws(c, layout(P, 0, 0), wsp, ws_bytes, ws));
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    double* out = ws.vec(8);
    HIPCHK(launch_lower_grad(S, x, y, grad, ws.part(), c->stream));
    HIPCHK(launch_finish_sum(ws.part(), tiles_of(S), 2, out, c->stream));
    if (phi_host) {
        HIPCHK(hipMemcpyAsync(c->h_buf, out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        *phi_host = c->h_buf[0];
    }
    return BL_OK;
}

// ---------------------------------------------------------------------------- Hessian solve
namespace {
// One solve is a one-slot batch whose scratch lives in ws (checked by the caller).
bl_status solve_in(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, const double* g,
                   double* w, bl_recycle* rs, const bl_solve_opts* o, const WS& ws, bl_stats* out) {
    mark(c, 0);
    Batch B;
    TRY(B.init(c, 1, ws.slots(), ws.ctr(), c->h_hdr, c->poll_ev[0], c->poll_ev[1]));
    SlotBuffers buf{};
    buf.r = ws.vec(0);
    buf.p0 = ws.vec(1);
    buf.p1 = ws.vec(2);
    buf.q = ws.vec(3);
    buf.r2 = ws.vec(4);
    buf.q2 = ws.vec(5);
    buf.HC = ws.Ut();
    buf.M = ws.mhc();
    buf.mpart = ws.vec(1);   // vectors 1-4, free until the set-up
    buf.d1 = ws.d1();
    buf.d2 = ws.d2();
    buf.d2f = ws.d2f();
    buf.taps = ws.taps();
    buf.rec_res = ws.part_res();
    buf.rec_app = ws.part_app();
    buf.rec_upd = ws.part_upd();
    buf.rec_app2 = ws.part_app2();
    buf.fold = ws.part_fold(0);
    buf.st = ws.st();
    const SolveSpec sp{P, theta, xhat, g, w, rs, o};
    TRY(B.admit(0, sp, buf, c->h_buf));
    mark(c, 1);
    std::vector<int> done;
    TRY(B.run(INT_MAX, false, done));
    mark(c, 2);
    bl_stats st;
    B.stats(0, &st);
    if (out) {
        *out = st;
        out->ms[0] = elapsed(c, 0, 1);
        out->ms[1] = elapsed(c, 1, 2);
        out->ms[2] = 0.0;
        out->ms[3] = elapsed(c, 0, 2);
    }
    return (bl_status)st.status;
}

bl_status solve_args(bl_ctx* c, const bl_problem* P, const double* xhat, const double* g, double* w,
                     const bl_recycle* rs, const bl_solve_opts* o) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !g || !w) return c->err = "null argument", BL_E_ARG;
    TRY(check_solve_opts(c, o));
    const int s_max = rs ? rs->s_max : 0, v_cap = rs ? rs->v_cap : 0;
    if (s_max < 0 || s_max > S_MAX || v_cap < 0) return c->err = "s_max outside [0, 64] or v_cap < 0", BL_E_SHAPE;
    return BL_OK;
}

// Scratch of bl_hessian_solve_noalloc: one array per device that loads the library, held until
// the process ends.  In host code `scratch` names a host-side stand-in, never the device array:
// its device address comes from hipGetSymbolAddress, once per device, and only that address is
// handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = BL_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex scratch_mu;
void* scratch_ptr[NOALLOC_MAX_DEVICES] = {};

bl_status scratch_address(bl_ctx* c, void*& ptr) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return c->err = "device index above the scratch table", BL_E_ARG;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return c->err = "no device address for the scratch array", BL_E_HIP;
        scratch_ptr[dev] = p;
    }
    ptr = scratch_ptr[dev];
    return BL_OK;
}
}  // namespace

bl_status bl_hessian_solve(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, const double* g,
                           double* w, bl_recycle* rs, const bl_solve_opts* o, void* wsp, size_t ws_bytes,
                           bl_stats* out) {
    TRY(solve_args(c, P, xhat, g, w, rs, o));
    WS ws;
    TRY(check_ws(c, layout(P, rs ? rs->s_max : 0, rs ? rs->v_cap : 0), wsp, ws_bytes, ws));
    return solve_in(c, P, theta, xhat, g, w, rs, o, ws, out);
}

bl_status bl_hessian_solve_noalloc(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat,
                                   const double* g, double* w, bl_recycle* rs, const bl_solve_opts* o,
                                   bl_stats* out) {
    TRY(solve_args(c, P, xhat, g, w, rs, o));
    const Layout L = layout(P, rs ? rs->s_max : 0, 0, true);
    if (L.total > NOALLOC_SCRATCH_BYTES)
        return c->err = "problem needs " + std::to_string(L.total) + " scratch bytes, above the " +
                        std::to_string(NOALLOC_SCRATCH_BYTES) + " of the static array",
               BL_E_WORKSPACE;
    void* ptr = nullptr;
    TRY(scratch_address(c, ptr));
    WS ws;
    ws.L = L;
    ws.base = (char*)ptr;
    // direct launches only: capturing and instantiating graphs could allocate
    const int graphs = c->graphs;
    c->graphs = 0;
    const bl_status st = solve_in(c, P, theta, xhat, g, w, rs, o, ws, out);
    c->graphs = graphs;
    return st;
}

// ------------------------------------------------------------------------------ RMINRES
// One solve, launched step by step: the set-up, then an apply and an update launch per Lanczos
// step, with a record fold before a consumer whenever the records exceed REC_LIMIT values, and
// a poll of the stop flag every POLL steps.  The test of iterate j runs in the apply launch of
// step j + 2, so at most max_iter + 2 steps are launched.
bl_status bl_hessian_solve_rminres(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat,
                                   const double* g, double* w, bl_recycle* rs, const bl_solve_opts* o, void* wsp,
                                   size_t ws_bytes, bl_stats* out) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !g || !w) return c->err = "null argument", BL_E_ARG;
    TRY(check_solve_opts(c, o));
    if (P->prec != BL_PREC_FP64) return c->err = "RMINRES runs in FP64 only", BL_E_ARG;
    const int s = rs ? rs->s_cur : 0, s_max = rs ? rs->s_max : 0, v_cap = rs ? rs->v_cap : 0;
    if (s_max < 0 || s_max > S_MAX || v_cap < 0) return c->err = "s_max outside [0, 64] or v_cap < 0", BL_E_SHAPE;
    if (rs) {
        if (s < 0 || s > s_max) return c->err = "s_cur outside [0, s_max]", BL_E_SHAPE;
        if (s > 0 && (!rs->U || !rs->C || !rs->mu)) return c->err = "null recycle arrays", BL_E_ARG;
        if (o->store_basis && (!rs->V || v_cap < 1)) return c->err = "store_basis needs V", BL_E_ARG;
    }
    WS ws;
    TRY(check_ws(c, layout(P, s_max, v_cap), wsp, ws_bytes, ws));
    mark(c, 0);
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    TRY(filter_state(c, S, xhat, ws));
    const bool hg = o->stop == BL_STOP_HGERR && s > 0 && rs->Z;
    const bool store = o->store_basis && rs;
    const int n = P->h * P->w;
    MinresArgs a{};
    a.xhat = xhat;
    a.g = g;
    a.w = w;
    a.r = ws.vec(0);
    a.q = ws.vec(1);
    for (int k = 0; k < 3; ++k) a.u[k] = ws.vec(2 + k);
    for (int k = 0; k < 2; ++k) a.m[k] = ws.vec(5 + k);
    a.U = s ? rs->U : nullptr;
    a.C = s ? rs->C : nullptr;
    a.Z = hg ? rs->Z : nullptr;
    a.V = store ? rs->V : nullptr;
    a.st = ws.mst();
    a.rec_res = ws.part_res();
    a.rec_app = ws.part_app();
    a.rec_upd = ws.part_upd();
    a.fold = ws.part_fold(0);
    a.n = n;
    a.ntiles = ((P->w + QW - 1) / QW) * ((P->h + QTY - 1) / QTY);
    a.npix = (n + NT - 1) / NT;
    a.s = s;
    a.nz = hg ? s : 0;
    const MinresInit in{o->tol, o->hg_tol, o->max_iter, o->check_every, o->stop, s, a.nz, hg ? 1 : 0,
                        store ? 1 : 0, v_cap, s ? rs->mu : nullptr};
    HIPCHK(launch_m_residual(S, a, c->stream));
    const bool fold_res = (long)a.ntiles * (1 + s) > REC_LIMIT;
    if (fold_res) HIPCHK(launch_m_fold(a.rec_res, a.ntiles, 1 + s, a.fold, c->stream));
    HIPCHK(launch_m_init(a, in, fold_res, c->stream));
    mark(c, 1);
    const bool fold_app = (long)a.ntiles * (1 + s) > REC_LIMIT;
    int nvb = 1 + a.nz;   // the set-up's record: iterate 0 is always tested
    bool decided = false;
    const long kmax = (long)o->max_iter + 2;
    // Stop-flag polls: after every POLL steps the header goes to one of two pinned snapshots,
    // marked by an event; the host then waits for the previous snapshot only, so the device
    // runs the next chunk meanwhile.  Launches after the stop return after their reduction.
    int pending = -1, npoll = 0;
    for (long k = 1; k <= kmax && !decided; ++k) {
        const bool fold_upd = (long)a.npix * nvb > REC_LIMIT;
        if (fold_upd) HIPCHK(launch_m_fold(a.rec_upd, a.npix, nvb, a.fold, c->stream));
        HIPCHK(launch_m_apply(S, a, (int)k, nvb, fold_upd, c->stream));
        if (fold_app) HIPCHK(launch_m_fold(a.rec_app, a.ntiles, 1 + s, a.fold, c->stream));
        const int zr = (k >= 2 && a.nz > 0 && (k - 1) % o->check_every == 0) ? a.nz : 0;
        HIPCHK(launch_m_update(a, (int)k, zr, fold_app, c->stream));
        nvb = 1 + zr;
        if (k % POLL == 0 || k == kmax) {
            const int buf = npoll++ & 1;
            HIPCHK(hipMemcpyAsync(c->h_info + 4 * buf, a.st, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipEventRecord(c->poll_ev[buf], c->stream));
            if (pending >= 0) {
                HIPCHK(hipEventSynchronize(c->poll_ev[pending]));
                decided = c->h_info[4 * pending] != 0;
            }
            pending = buf;
        }
    }
    if (!decided && pending >= 0) {   // the snapshot taken after the last launched step
        HIPCHK(hipEventSynchronize(c->poll_ev[pending]));
        decided = c->h_info[4 * pending] != 0;
    }
    if (!decided) return c->err = "RMINRES ended without a stop decision", BL_E_HIP;
    if (s) HIPCHK(launch_m_finish(a, c->stream));
    mark(c, 2);
    static_assert(sizeof(MinresState) <= 8192 * sizeof(double), "state exceeds the staging buffer");
    HIPCHK(hipMemcpyAsync(c->h_buf, a.st, sizeof(MinresState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    MinresState hs;
    std::memcpy(&hs, c->h_buf, sizeof(MinresState));
    if (store) {
        rs->v_cur = std::min(hs.iters, v_cap);
        rs->v_lz = 0;   // Lanczos vectors: no CG coefficients for an inner refresh
    }
    if (out) {
        *out = bl_stats{};
        out->iters = hs.iters;
        out->status = hs.status;
        out->s_cur = s;
        out->res_norm = hs.res;
        out->res0_norm = hs.res0;
        out->g_norm = hs.gnorm;
        out->est = hs.est;
        out->ms[0] = elapsed(c, 0, 1);
        out->ms[1] = elapsed(c, 1, 2);
        out->ms[3] = elapsed(c, 0, 2);
    }
    return (bl_status)hs.status;
}

// ------------------------------------------------------------------------------ deflated CG
// One solve, launched step by step: the set-up, then an apply and an update launch per step,
// with a record fold before a consumer whenever the records exceed REC_LIMIT values, and a poll
// of the stop flag every POLL steps (double-buffered, as for RMINRES).  The test of iterate j
// runs in the apply launch of step j, so at most max_iter + 1 steps are launched.
bl_status bl_hessian_solve_deflated(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat,
                                    const double* g, double* w, bl_recycle* rs, const bl_solve_opts* o, void* wsp,
                                    size_t ws_bytes, bl_stats* out) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !g || !w) return c->err = "null argument", BL_E_ARG;
    TRY(check_solve_opts(c, o));
    if (P->prec != BL_PREC_FP64) return c->err = "deflated CG runs in FP64 only", BL_E_ARG;
    const int s = rs ? rs->s_cur : 0, s_max = rs ? rs->s_max : 0, v_cap = rs ? rs->v_cap : 0;
    if (s_max < 0 || s_max > S_MAX || v_cap < 0) return c->err = "s_max outside [0, 64] or v_cap < 0", BL_E_SHAPE;
    if (rs) {
        if (s < 0 || s > s_max) return c->err = "s_cur outside [0, s_max]", BL_E_SHAPE;
        if (s > 0 && (!rs->U || !rs->C || !rs->mu)) return c->err = "null recycle arrays", BL_E_ARG;
        if (o->store_basis && (!rs->V || v_cap < 1)) return c->err = "store_basis needs V", BL_E_ARG;
    }
    WS ws;
    TRY(check_ws(c, layout(P, s_max, v_cap), wsp, ws_bytes, ws));
    mark(c, 0);
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    TRY(filter_state(c, S, xhat, ws));
    const bool hg = o->stop == BL_STOP_HGERR && s > 0 && rs->Z;
    const bool store = o->store_basis && rs;
    const int n = P->h * P->w;
    const size_t T2 = (size_t)ws.L.t_max * ws.L.t_max;
    DeflArgs a{};
    a.xhat = xhat;
    a.g = g;
    a.w = w;
    a.r = ws.vec(0);
    a.p[0] = ws.vec(1);
    a.p[1] = ws.vec(2);
    a.q = ws.vec(3);
    a.U = s ? rs->U : nullptr;
    a.C = s ? rs->C : nullptr;
    a.Z = hg ? rs->Z : nullptr;
    a.mu = s ? rs->mu : nullptr;
    a.Einv = ws.small(0);
    a.V = store ? rs->V : nullptr;
    a.st = ws.st();
    a.rec_res = ws.part_res();
    a.rec_app = ws.part_app();
    a.rec_upd = ws.part_upd();
    a.fold = ws.part_fold(0);
    a.n = n;
    a.ntiles = ((P->w + QW - 1) / QW) * ((P->h + QTY - 1) / QTY);
    a.npix = (n + NT - 1) / NT;
    a.s = s;
    a.nz = hg ? s : 0;
    if (s) {   // E^{-1} = (U^T C)^{-1}: the deflation space's projected Hessian (E = U^T H U)
        int* info = ws.ctr();
        HIPCHK(launch_gram(n, s, s, rs->U, rs->C, ws.part(), ws.small(2 * T2), c->stream));
        HIPCHK(launch_d_einv(s, ws.small(2 * T2), ws.small(T2), ws.small(0), info, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_info, info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->h_info[0] != BL_OK) return c->err = "U^T C is not positive definite", BL_E_INDEFINITE;
    }
    const StateInit in{o->tol, o->hg_tol, o->max_iter, o->check_every, o->stop, s, store ? v_cap : 0,
                       store ? 1 : 0, hg ? 1 : 0};
    HIPCHK(launch_d_residual(S, a, c->stream));
    const bool fold_res = (long)a.ntiles * (1 + s) > REC_LIMIT;
    if (fold_res) HIPCHK(launch_m_fold(a.rec_res, a.ntiles, 1 + s, a.fold, c->stream));
    HIPCHK(launch_d_init(a, in, fold_res, c->stream));
    mark(c, 1);
    const bool fold_app = (long)a.ntiles > REC_LIMIT;
    const auto zw_of = [&](long j) { return (a.nz > 0 && j % o->check_every == 0) ? a.nz : 0; };
    bool decided = false;
    const long jmax = (long)o->max_iter;
    int pending = -1, npoll = 0;
    for (long j = 0; j <= jmax && !decided; ++j) {
        const int zw = zw_of(j);
        const bool fold_upd = (long)a.npix * (1 + s + zw) > REC_LIMIT;
        if (fold_upd) HIPCHK(launch_m_fold(a.rec_upd, a.npix, 1 + s + zw, a.fold, c->stream));
        HIPCHK(launch_d_apply(S, a, (int)j, zw, fold_upd, c->stream));
        if (j < jmax) {
            if (fold_app) HIPCHK(launch_m_fold(a.rec_app, a.ntiles, 1, a.fold, c->stream));
            HIPCHK(launch_d_update(a, (int)j, zw_of(j + 1), fold_app, c->stream));
        }
        if ((j + 1) % POLL == 0 || j == jmax) {
            const int buf = npoll++ & 1;
            HIPCHK(hipMemcpyAsync(c->h_hdr + (size_t)buf * HDR_BYTES, a.st, HDR_BYTES, hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipEventRecord(c->poll_ev[buf], c->stream));
            if (pending >= 0) {
                HIPCHK(hipEventSynchronize(c->poll_ev[pending]));
                decided = reinterpret_cast<const SolveState*>(c->h_hdr + (size_t)pending * HDR_BYTES)->done != 0;
            }
            pending = buf;
        }
    }
    if (!decided && pending >= 0) {
        HIPCHK(hipEventSynchronize(c->poll_ev[pending]));
        decided = reinterpret_cast<const SolveState*>(c->h_hdr + (size_t)pending * HDR_BYTES)->done != 0;
    }
    if (!decided) return c->err = "deflated CG ended without a stop decision", BL_E_HIP;
    mark(c, 2);
    HIPCHK(hipMemcpyAsync(c->h_state, a.st, sizeof(SolveState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const SolveState hs = *c->h_state;
    if (store) {
        rs->v_cur = std::min(hs.iters + (hs.status == BL_E_INDEFINITE ? 1 : 0), v_cap);
        rs->v_lz = 0;   // no CG coefficients of the Galerkin form: the inner refresh refuses this basis
    }
    if (out) {
        *out = bl_stats{};
        out->iters = hs.iters;
        out->status = hs.status;
        out->s_cur = s;
        out->res_norm = std::sqrt(std::max(hs.rho2[hs.iters & 1], 0.0));
        out->res0_norm = hs.res0;
        out->g_norm = hs.gnorm;
        out->est = hs.est;
        out->ms[0] = elapsed(c, 0, 1);
        out->ms[1] = elapsed(c, 1, 2);
        out->ms[3] = elapsed(c, 0, 2);
    }
    return (bl_status)hs.status;
}

// ------------------------------------------------------------------------------ tile heights
bl_status bl_tile_rows_set(const bl_problem* P, int rows) {
    bl_ctx tmp;
    if (check_problem(&tmp, P) != BL_OK) return BL_E_ARG;
    if (rows != 0 && !valid_rows(rows)) return BL_E_ARG;
    set_tile_rows(P, rows);
    return BL_OK;
}

int bl_tile_rows(const bl_problem* P) {
    bl_ctx tmp;
    if (check_problem(&tmp, P) != BL_OK) return 0;
    return tile_rows(P);
}

// Autotuner scratch inside the caller's workspace: the solve workspace (s recycle columns, no
// stored basis), then g, w, and the zero recycle columns U, C, Z with mu.
namespace {
struct TuneLayout {
    size_t solve, g, w, u, c, z, mu, total;
};
TuneLayout tune_layout(const bl_problem* P, int s) {
    TuneLayout T{};
    const size_t n = (size_t)P->h * P->w, sc = (size_t)std::max(s, 1);
    T.solve = bl_workspace_bytes(P, s, 0);
    T.g = al(T.solve);
    T.w = T.g + al(n * 8);
    T.u = T.w + al(n * 8);
    T.c = T.u + al(n * sc * 8);
    T.z = T.c + al(n * sc * 8);
    T.mu = T.z + al(n * sc * 8);
    T.total = T.mu + al(sc * 8);
    return T;
}

// Each height runs a short warm-up solve, then `iters` timed iterations of a solve whose
// recycle columns are zero (C^T q = 0, C e = 0: plain CG arithmetic, recycled memory traffic)
// with the stop test disabled (tol = 0).
bl_status autotune_time(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, int s, int iters,
                        char* mem, const TuneLayout& T, double us[3]) {
    const size_t n = (size_t)P->h * P->w, sc = (size_t)std::max(s, 1);
    const int heights[3] = {QTY, 2 * QTY, 4 * QTY};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto body = [&]() -> bl_status {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipMemsetAsync(mem + T.u, 0, T.mu + al(sc * 8) - T.u, c->stream));
        HIPCHK(hipMemcpyAsync(mem + T.g, xhat, n * 8, hipMemcpyDeviceToDevice, c->stream));
        bl_recycle rs{};
        rs.U = (double*)(mem + T.u);
        rs.C = (double*)(mem + T.c);
        rs.Z = (double*)(mem + T.z);
        rs.mu = (double*)(mem + T.mu);
        rs.s_max = s;
        rs.s_cur = s;
        bl_solve_opts o{};
        o.stop = BL_STOP_RESID;
        o.tol = 0.0;
        o.check_every = 1;
        o.rr_every = 50;
        // per tile height: a warm-up solve of a iterations, then timed solves of a and b: the
        // difference is the cost of b - a iterations, free of the per-solve set-up (the residual,
        // H C and C^T H C of a recycled solve); a and b are whole chunks of the batch engine
        const int a = CHUNK, b = CHUNK + CHUNK * std::max(1, iters / CHUNK);
        for (int k = 0; k < 3; ++k) {
            c->force_rows = heights[k];
            float ms[2] = {0.f, 0.f};
            int its[2] = {0, 0};
            for (int pass = 0; pass < 3; ++pass) {
                o.max_iter = pass == 2 ? b : a;
                HIPCHK(hipMemsetAsync(mem + T.w, 0, n * 8, c->stream));
                if (pass > 0) HIPCHK(hipEventRecord(e0, c->stream));
                bl_stats st{};
                const bl_status r = bl_hessian_solve(c, P, theta, xhat, (const double*)(mem + T.g),
                                                     (double*)(mem + T.w), s ? &rs : nullptr, &o, mem, T.solve, &st);
                if (r == BL_E_HIP || r == BL_E_ARG || r == BL_E_SHAPE || r == BL_E_WORKSPACE) return r;
                if (pass > 0) {
                    HIPCHK(hipEventRecord(e1, c->stream));
                    HIPCHK(hipEventSynchronize(e1));
                    HIPCHK(hipEventElapsedTime(&ms[pass - 1], e0, e1));
                    its[pass - 1] = st.iters;
                }
            }
            us[k] = its[1] > its[0] ? 1e3 * (ms[1] - ms[0]) / (its[1] - its[0])
                                    : 1e3 * ms[1] / std::max(its[1], 1);   // (a solve that stopped early)
        }
        return BL_OK;
    };
    const bl_status rc = body();
    c->force_rows = 0;
    (void)hipStreamSynchronize(c->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}
}  // namespace

size_t bl_autotune_workspace_bytes(const bl_problem* P, int s) {
    bl_ctx tmp;
    if (!P || check_problem(&tmp, P) != BL_OK || s < 0 || s > S_MAX) return 0;
    return tune_layout(P, s).total;
}

bl_status bl_autotune(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, int s, int iters,
                      const char* cache_path, void* wsp, size_t ws_bytes, int* best_rows, double* us_per_iter) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!best_rows) return c->err = "null best_rows", BL_E_ARG;
    if (s < 0 || s > S_MAX) return c->err = "s outside [0, 64]", BL_E_SHAPE;
    if (us_per_iter)
        for (int k = 0; k < 3; ++k) us_per_iter[k] = 0.0;
    if (cache_path) {
        int rows = 0;
        bool found = false;
        if (!tile_cache_lookup(cache_path, P, rows, found, c->err)) return BL_E_ARG;
        if (found) {   // a stored result: no timing, no device work
            set_tile_rows(P, rows);
            *best_rows = rows;
            return BL_OK;
        }
    }
    if (!theta || !xhat) return c->err = "null theta or xhat", BL_E_ARG;
    if (iters < 1 || iters > 100000) return c->err = "iters outside [1, 100000]", BL_E_ARG;
    const TuneLayout T = tune_layout(P, s);
    if (!wsp) return c->err = "null workspace", BL_E_WORKSPACE;
    if (ws_bytes < T.total) return c->err = "workspace smaller than bl_autotune_workspace_bytes()", BL_E_WORKSPACE;
    if ((uintptr_t)wsp % ALIGN) return c->err = "workspace must be 256-byte aligned", BL_E_WORKSPACE;
    double us[3] = {0.0, 0.0, 0.0};
    TRY(autotune_time(c, P, theta, xhat, s, iters, (char*)wsp, T, us));
    const int heights[3] = {QTY, 2 * QTY, 4 * QTY};
    int best = 0;
    for (int k = 1; k < 3; ++k)
        if (us[k] < us[best]) best = k;
    set_tile_rows(P, heights[best]);
    *best_rows = heights[best];
    if (us_per_iter)
        for (int k = 0; k < 3; ++k) us_per_iter[k] = us[k];
    if (cache_path && !tile_cache_store(cache_path, P, heights[best], us, c->err)) return BL_E_ARG;
    return BL_OK;
}

bl_status bl_tile_cache_load(const char* cache_path, int* entries) {
    if (!cache_path) return BL_E_ARG;
    int k = 0;
    std::string err;
    if (!tile_cache_load_all(cache_path, k, err)) return BL_E_ARG;
    if (entries) *entries = k;
    return BL_OK;
}

// ---------------------------------------------------------------------------- recycle storage
namespace {
struct RecLayout {
    size_t U, C, Z, mu, V, lz, total;
};
RecLayout rec_layout(const bl_problem* P, int s_max, int v_cap) {
    const size_t n = (size_t)P->h * P->w;
    RecLayout R{};
    R.U = 0;
    R.C = al(n * s_max * 8);
    R.Z = R.C + al(n * s_max * 8);
    R.mu = R.Z + al(n * s_max * 8);
    R.V = R.mu + al((size_t)s_max * 8);
    R.lz = R.V + al(n * v_cap * 8);
    R.total = std::max(R.lz + al((size_t)2 * v_cap * 8), ALIGN);   // never 0 for a valid shape (0: invalid)
    return R;
}
bool rec_shape_ok(const bl_problem* P, int s_max, int v_cap) {
    bl_ctx tmp;
    return P && check_problem(&tmp, P) == BL_OK && s_max >= 0 && s_max <= S_MAX && v_cap >= 0 && s_max + v_cap <= 256;
}
}  // namespace

size_t bl_recycle_bytes(const bl_problem* P, int s_max, int v_cap) {
    return rec_shape_ok(P, s_max, v_cap) ? rec_layout(P, s_max, v_cap).total : 0;
}

bl_status bl_recycle_init(const bl_problem* P, int s_max, int v_cap, void* base, size_t bytes, bl_recycle* rs) {
    if (!rs || !base) return BL_E_ARG;
    if (!rec_shape_ok(P, s_max, v_cap)) return BL_E_SHAPE;
    const RecLayout R = rec_layout(P, s_max, v_cap);
    if (bytes < R.total) return BL_E_WORKSPACE;
    if ((uintptr_t)base % ALIGN) return BL_E_WORKSPACE;
    char* b = (char*)base;
    rs->U = (double*)(b + R.U);
    rs->C = (double*)(b + R.C);
    rs->Z = (double*)(b + R.Z);
    rs->mu = (double*)(b + R.mu);
    rs->V = v_cap > 0 ? (double*)(b + R.V) : nullptr;
    rs->lz = v_cap > 0 ? (double*)(b + R.lz) : nullptr;
    rs->s_max = s_max;
    rs->s_cur = 0;
    rs->v_cap = v_cap;
    rs->v_cur = 0;
    rs->v_lz = 0;
    return BL_OK;
}

// ---------------------------------------------------------------------------- hypergradient
bl_status bl_hypergradient(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, const double* w,
                           double* grad, int project, void* wsp, size_t ws_bytes) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !w || !grad) return c->err = "null argument", BL_E_ARG;
    WS ws;
    TRY(check_ws(c, layout(P, 0, 0), wsp, ws_bytes, ws));
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    TRY(filter_state(c, S, xhat, ws));
    const int p = nparams(P);
    double* Gd = ws.vec(8);   // p doubles after the 8 work vectors
    HIPCHK(launch_jac(S, xhat, w, 1, ws.d1(), ws.d2(), ws.part(), Gd, project, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_buf, Gd, p * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(grad, c->h_buf, p * sizeof(double));
    for (int k = 0; k < p; ++k)
        if (!std::isfinite(grad[k])) return c->err = "non-finite hypergradient", BL_E_NONFINITE;
    return BL_OK;
}

// ---------------------------------------------------------------------------- recycle refresh
bl_status bl_recycle_update(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, bl_recycle* rs,
                            const bl_recycle_opts* o, void* wsp, size_t ws_bytes, bl_stats* out) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !rs || !o) return c->err = "null argument", BL_E_ARG;
    if (rs->s_max < 0 || rs->s_max > S_MAX || o->s < 0 || o->s > rs->s_max)
        return c->err = "s outside [0, s_max] or s_max > 64", BL_E_SHAPE;
    if (rs->s_cur < 0 || rs->s_cur > rs->s_max || rs->v_cur < 0 || rs->v_cur > rs->v_cap)
        return c->err = "s_cur / v_cur outside capacity", BL_E_SHAPE;
    if (!rs->U || !rs->C || !rs->Z || !rs->mu || (rs->v_cap > 0 && !rs->V))
        return c->err = "null recycle arrays", BL_E_ARG;
    if (!(o->rank_tol > 0.0 && o->rank_tol < 1.0)) return c->err = "rank_tol outside (0, 1)", BL_E_ARG;
    if (o->inner != 0 && o->inner != 1) return c->err = "inner must be 0 or 1", BL_E_ARG;
    const bool inner = o->inner == 1;
    if (inner) {
        if (o->select >= BL_SEL_HRITZ_S && o->select <= BL_SEL_HRITZ_M)
            return c->err = "the inner refresh has no (H W)^T (H W): harmonic Ritz selections are outer only", BL_E_ARG;
        if (rs->v_lz < 0 || rs->v_lz > rs->v_cur) return c->err = "v_lz outside [0, v_cur]", BL_E_SHAPE;
        if (rs->v_cur > 0 && (rs->v_lz == 0 || !rs->lz))
            return c->err = "inner refresh: no CG coefficients for the stored basis (store it with a CG solve)", BL_E_ARG;
    }
    if (o->select < BL_SEL_RGEN_L_R || o->select > BL_SEL_RGEN_M_M) return c->err = "unknown selection", BL_E_ARG;
    const bool rgen = o->select <= BL_SEL_RGEN_L_M || o->select >= BL_SEL_RGEN_S_R;
    // RGen: size 0 / 1 / 2 (largest / smallest / both ends), side 0 / 1 / 2 (right / left / sum)
    int gsize = 0, side = 0;
    if (o->select <= BL_SEL_RGEN_L_M) {
        side = o->select - BL_SEL_RGEN_L_R;
    } else if (o->select >= BL_SEL_RGEN_S_R) {
        const int q = o->select - BL_SEL_RGEN_S_R;
        gsize = 1 + q / 3;
        side = q % 3;
    }
    WS ws;
    TRY(check_ws(c, layout(P, rs->s_max, rs->v_cap), wsp, ws_bytes, ws));
    const int n = P->h * P->w, p = nparams(P);
    // inner: the stored residuals the CG coefficients describe (all of them, unless a residual
    // replacement of a mixed-precision solve cut the relation short)
    int v_use = inner ? rs->v_lz : rs->v_cur;
    int t0 = rs->s_cur + v_use;
    if (out) std::memset(out, 0, sizeof(*out));
    if (t0 == 0 || o->s == 0) {
        rs->s_cur = 0;
        return BL_OK;
    }
    mark(c, 0);
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    TRY(filter_state(c, S, xhat, ws));
    const int tm = ws.L.t_max;
    const size_t T2 = (size_t)tm * tm;
    double* Gram = ws.small(0);
    double* Xinv = ws.small(T2);
    double* Achol = ws.small(2 * T2);
    double* M = ws.small(3 * T2);
    double* Gj = ws.small(4 * T2);
    double* Xs = Gj + (size_t)p * tm;
    double* VHs = Xs + (size_t)tm * std::max(rs->s_max, 1);
    double* mu_tmp = VHs + (size_t)tm * std::max(rs->s_max, 1);
    double* gsc = mu_tmp + 256;
    double* X1c = gsc + gsvd_scratch_doubles(tm, p);   // inner: first-pass factor, X = X1 X2, Y = M0 X
    double* Xp = X1c + T2;
    double* Yp = Xp + T2;
    double* UtC = Xinv;                                  // inner: U^T C of the previous system (s0 x s0)
    int* ibuf = (int*)(Yp + T2);
    int* kept = ibuf;
    int* tk_dev = ibuf + tm;
    int* info = ibuf + tm + 4;
    // W0 = [U, V]
    double* W0 = ws.W0();
    double* W1 = ws.W1();
    if (rs->s_cur)
        HIPCHK(hipMemcpyAsync(W0, rs->U, (size_t)rs->s_cur * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (v_use)
        HIPCHK(hipMemcpyAsync(W0 + (size_t)rs->s_cur * n, rs->V, (size_t)v_use * n * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    // two passes of Cholesky QR with column drop: W = [U, V] X1 X2
    HIPCHK(launch_gram(n, t0, t0, W0, W0, ws.part(), Gram, c->stream));
    if (inner && v_use > 0) {
        // the previous solve's relation V^T H V = T holds to working precision only over the
        // semi-orthogonal leading part of its stored residuals (Simon's condition): keep that part
        HIPCHK(launch_semiorth_prefix(t0, rs->s_cur, Gram, 0x1p-26, tk_dev + 1, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_info, tk_dev + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->h_info[0] < v_use) {
            v_use = c->h_info[0];
            t0 = rs->s_cur + v_use;
            if (t0 == 0) {
                rs->s_cur = 0;
                return c->err = "inner refresh: no semi-orthogonal stored residual", BL_E_RANK;
            }
            HIPCHK(launch_gram(n, t0, t0, W0, W0, ws.part(), Gram, c->stream));
        }
    }
    HIPCHK(launch_chol_drop(t0, Gram, o->rank_tol, Achol, kept, tk_dev, Xinv, t0, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_info, tk_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int t1 = c->h_info[0];
    if (t1 == 0) {
        rs->s_cur = 0;
        return BL_E_RANK;
    }
    HIPCHK(launch_gemm_tall(n, t0, t1, W0, Xinv, t0, W1, c->stream));
    if (inner) HIPCHK(hipMemcpyAsync(X1c, Xinv, (size_t)t0 * t1 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(launch_gram(n, t1, t1, W1, W1, ws.part(), Gram, c->stream));
    HIPCHK(launch_chol_drop(t1, Gram, 1e-12, Achol, kept, tk_dev, Xinv, t1, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_info, tk_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int t = c->h_info[0];
    HIPCHK(launch_gemm_tall(n, t1, t, W1, Xinv, t1, W0, c->stream));   // W (orthonormal) in W0
    mark(c, 1);
    if (!inner) {
        // Y = H W (FP64), M = W^T Y
        // t columns give any tile height enough blocks: the tallest (measured fastest for this product)
        HIPCHK(launch_hvp(S, false, xhat, W0, W1, t, 4 * QTY, c->stream));
        HIPCHK(launch_gram(n, t, t, W0, W1, ws.part(), M, c->stream));
    } else {
        // M = W^T H_old W without products: W = [U, V] X with X = X1 X2, and [U, V]^T H_old [U, V]
        // = blockdiag(sym(U^T C), T) (U^T H_old V = C^T V = 0; T from the CG coefficients)
        const int s0 = rs->s_cur;
        HIPCHK(launch_small_gemm(t0, t1, t, false, X1c, t0, Xinv, t1, Xp, t0, c->stream));
        if (s0) HIPCHK(launch_gram(n, s0, s0, rs->U, rs->C, ws.part(), UtC, c->stream));
        HIPCHK(launch_inner_y(s0, v_use, t, UtC, rs->lz, Xp, Yp, c->stream));
        HIPCHK(launch_small_gemm(t, t0, t, true, Xp, t0, Yp, t0, M, t, c->stream));
    }
    if (rgen) HIPCHK(launch_jac(S, xhat, W0, t, ws.d1(), ws.d2(), ws.part(), Gj, 1, c->stream));
    mark(c, 2);
    if (rgen) {
        if (gsize != 0 && p < t) {
            rs->s_cur = 0;
            return c->err = "RGen sizes S and M need p >= t (J W of full column rank)", BL_E_ARG;
        }
        HIPCHK(launch_gsvd_select(t, p, o->s, gsize, M, Gj, gsc, Xs, VHs, mu_tmp, info, c->stream));
        if (side != 0) HIPCHK(launch_rgen_side(t, side, M, Xs, info, c->stream));
    } else {
        // Ritz values of W^T H W, or harmonic Ritz values from (H W)^T (H W) = Y^T Y
        const int kind = o->select >= BL_SEL_HRITZ_S ? 1 : 0;
        const int size = (o->select - (kind ? BL_SEL_HRITZ_S : BL_SEL_RITZ_S));
        if (kind) HIPCHK(launch_gram(n, t, t, W1, W1, ws.part(), Gram, c->stream));
        HIPCHK(launch_ritz_select(t, o->s, kind, size, M, Gram, gsc, Xs, VHs, mu_tmp, info, c->stream));
    }
    HIPCHK(hipMemcpyAsync(c->h_info, info, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int s_eff = c->h_info[0], rankG = c->h_info[1], gst = c->h_info[2];
    if (gst != BL_OK) {
        rs->s_cur = 0;
        c->err = rgen ? "projected Hessian W^T H W is not positive definite"
                      : "(H W)^T (H W) is not positive definite";
        return (bl_status)gst;
    }
    // U~ = W X~, C~ = Y X~ (inner: s products with the new Hessian), Z = W V_H~
    HIPCHK(launch_gemm_tall(n, t, s_eff, W0, Xs, t, ws.Ut(), c->stream));
    if (!inner) HIPCHK(launch_gemm_tall(n, t, s_eff, W1, Xs, t, ws.Ct(), c->stream));
    else HIPCHK(launch_hvp(S, false, xhat, ws.Ut(), ws.Ct(), s_eff, 4 * QTY, c->stream));
    HIPCHK(launch_gemm_tall(n, t, s_eff, W0, VHs, t, rs->Z, c->stream));
    HIPCHK(hipMemcpyAsync(rs->mu, mu_tmp, s_eff * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    // C~ = C R (two passes of Cholesky QR), U = U~ R^{-1}
    int sc = s_eff;
    double* srcU = ws.Ut();
    double* srcC = ws.Ct();
    for (int pass = 0; pass < 2; ++pass) {
        double* dstU = pass == 0 ? rs->U : ws.Ut();
        double* dstC = pass == 0 ? rs->C : ws.Ct();
        HIPCHK(launch_gram(n, sc, sc, srcC, srcC, ws.part(), Gram, c->stream));
        HIPCHK(launch_chol_drop(sc, Gram, 1e-13, Achol, kept, tk_dev, Xinv, sc, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_info, tk_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const int sk = c->h_info[0];
        HIPCHK(launch_gemm_tall(n, sc, sk, srcC, Xinv, sc, dstC, c->stream));
        HIPCHK(launch_gemm_tall(n, sc, sk, srcU, Xinv, sc, dstU, c->stream));
        sc = sk;
        srcU = dstU;
        srcC = dstC;
    }
    HIPCHK(hipMemcpyAsync(rs->U, ws.Ut(), (size_t)sc * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(rs->C, ws.Ct(), (size_t)sc * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    mark(c, 3);
    HIPCHK(hipStreamSynchronize(c->stream));
    rs->s_cur = sc;
    if (out) {
        out->t = t;
        out->s_cur = sc;
        out->iters = rankG;
        out->status = (t < t0 || sc < s_eff) ? BL_E_RANK : BL_OK;
        out->ms[0] = elapsed(c, 0, 1);
        out->ms[1] = elapsed(c, 1, 2);
        out->ms[2] = elapsed(c, 2, 3);
        out->ms[3] = elapsed(c, 0, 3);
    }
    return sc < s_eff ? BL_E_RANK : BL_OK;
}

// ---------------------------------------------------------------------------- lower-level solve
bl_status bl_lower_solve(bl_ctx* c, const bl_problem* P, const double* theta, const double* y, double* x,
                         double gtol, int max_iter, int m, void* wsp, size_t ws_bytes, bl_stats* out) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!y || !x) return c->err = "null vector", BL_E_ARG;
    if (m < 1 || m > LBFGS_MMAX || max_iter < 0 || !(gtol >= 0.0)) return c->err = "invalid L-BFGS options", BL_E_ARG;
    WS ws;
    TRY(check_ws(c, layout(P, 0, 0), wsp, ws_bytes, ws));
    Stencil S;
    TRY(make_stencil(c, P, theta, ws, S));
    const int n = P->h * P->w;
    const int vb = wide_blocks(n);   // records of the multi-dot pass (at most 1024)
    double* g = ws.vec(0);
    double* d = ws.vec(1);
    double* xt = ws.vec(2);
    double* gt = ws.vec(3);
    double* Sh = ws.lb();
    double* Yh = Sh + (size_t)(LBFGS_MMAX + 1) * n;
    double* md_rec = Yh + (size_t)(LBFGS_MMAX + 1) * n;   // multi-dot records: VL_MAX per block
    double* fout = md_rec + (size_t)VL_MAX * vb;           // host-bound scalars
    auto grad_at = [&](const double* xx, double* gg, double& f, double& gn2) -> bl_status {
        HIPCHK(launch_lower_grad(S, xx, y, gg, ws.part(), c->stream));
        HIPCHK(launch_finish_sum(ws.part(), tiles_of(S), 2, fout, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_buf, fout, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        f = c->h_buf[0];
        gn2 = c->h_buf[1];
        return BL_OK;
    };
    // dots a_i . b_i of a list of pairs, VL_MAX per pass, into host memory
    auto dots = [&](const std::vector<std::pair<const double*, const double*>>& pr, double* hout) -> bl_status {
        const int k = (int)pr.size();
        for (int c0 = 0; c0 < k; c0 += VL_MAX) {
            VecPairs vp{};
            vp.k = std::min(VL_MAX, k - c0);
            for (int i = 0; i < vp.k; ++i) {
                vp.a[i] = pr[c0 + i].first;
                vp.b[i] = pr[c0 + i].second;
            }
            HIPCHK(launch_multidot(n, vp, md_rec, c->stream));
            HIPCHK(launch_finish_sum(md_rec, vb, vp.k, fout + 2 + c0, c->stream));
        }
        HIPCHK(hipMemcpyAsync(c->h_buf, fout + 2, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        std::memcpy(hout, c->h_buf, k * sizeof(double));
        return BL_OK;
    };
    double f, gn2;
    TRY(grad_at(x, g, f, gn2));
    // History of kept pairs, oldest first (device buffers of m + 1 slots, so a new pair never
    // overwrites a kept one), with the small matrices of the compact representation
    // (Byrd, Nocedal, Schnabel 1994): SY[i][j] = s_i . y_j and YY[i][j] = y_i . y_j.
    constexpr int MM = LBFGS_MMAX + 1;
    std::vector<int> slot;
    std::vector<int> free_slots;
    for (int k = m; k >= 0; --k) free_slots.push_back(k);
    std::vector<double> SY(MM * MM, 0.0), YY(MM * MM, 0.0);
    std::vector<double> av(2 * MM), uv(MM), pv(MM), wv(MM), nd(5 * MM + 3);
    // the iterate and its gradient alternate between the caller's x (and g) and xt (and gt)
    double* xc = x;
    double* xn = xt;
    double* gc = g;
    double* gn = gt;
    int it = 0;
    double gnorm = std::sqrt(gn2);
    double gamma = 0.0;
    while (gnorm > gtol && it < max_iter) {
        if (!std::isfinite(f) || !std::isfinite(gnorm)) return c->err = "non-finite objective", BL_E_NONFINITE;
        // d = H_k g in the compact form: with a = S^T g, b = Y^T g (av, from the previous
        // iteration's dot pass), R the upper triangle of S^T Y and D its diagonal,
        // u = R^{-1} a, p = R^{-T} ((D + gamma Y^T Y) u - gamma b), d = gamma g + S p - gamma Y u.
        const int hsz = (int)slot.size();
        double gd;
        if (hsz == 0) {
            VecComb vc{};
            HIPCHK(launch_lincomb(n, 1.0 / gnorm, gc, vc, d, c->stream));
            gd = gnorm;
        } else {
            const double* A = av.data();
            const double* Bv = av.data() + hsz;
            for (int i = hsz - 1; i >= 0; --i) {
                double acc = A[i];
                for (int j = i + 1; j < hsz; ++j) acc -= SY[i * MM + j] * uv[j];
                uv[i] = acc / SY[i * MM + i];
            }
            for (int i = 0; i < hsz; ++i) {
                double acc = 0.0;
                for (int j = 0; j < hsz; ++j) acc += YY[i * MM + j] * uv[j];
                wv[i] = SY[i * MM + i] * uv[i] + gamma * acc - gamma * Bv[i];
            }
            for (int i = 0; i < hsz; ++i) {
                double acc = wv[i];
                for (int j = 0; j < i; ++j) acc -= SY[j * MM + i] * pv[j];
                pv[i] = acc / SY[i * MM + i];
            }
            VecComb vc{};
            vc.k = 2 * hsz;
            gd = gamma * gn2;
            for (int i = 0; i < hsz; ++i) {
                vc.c[i] = pv[i];
                vc.v[i] = Sh + (size_t)slot[i] * n;
                vc.c[hsz + i] = -gamma * uv[i];
                vc.v[hsz + i] = Yh + (size_t)slot[i] * n;
                gd += pv[i] * A[i] - gamma * uv[i] * Bv[i];
            }
            HIPCHK(launch_lincomb(n, gamma, gc, vc, d, c->stream));
        }
        // direction -d; slope = -(g . d)
        double slope = -gd;
        if (!(slope < 0.0)) {   // not a descent direction: steepest descent
            HIPCHK(hipMemcpyAsync(d, gc, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            slope = -gnorm * gnorm;
        }
        // backtracking Armijo on x - t d
        double tstep = 1.0, fn = 0.0, gn2n = 0.0;
        bool ok = false;
        for (int bt = 0; bt < 60; ++bt) {
            VecComb step{};
            step.k = 1;
            step.c[0] = -tstep;
            step.v[0] = d;
            HIPCHK(launch_lincomb(n, 1.0, xc, step, xn, c->stream));
            TRY(grad_at(xn, gn, fn, gn2n));
            if (fn <= f + 1e-4 * tstep * slope) {
                ok = true;
                break;
            }
            tstep *= 0.5;
        }
        if (!ok) break;
        // new pair s = x_new - x, y = g_new - g; one dot pass for its products with itself and
        // the kept pairs and for the next direction's S^T g_new, Y^T g_new (kept pairs and the
        // new one: whether the new pair is kept is decided from these dots)
        const int sl = free_slots.back();
        free_slots.pop_back();
        double* sv = Sh + (size_t)sl * n;
        double* yv = Yh + (size_t)sl * n;
        HIPCHK(launch_sub(n, xn, xc, sv, c->stream));
        HIPCHK(launch_sub(n, gn, gc, yv, c->stream));
        {
            std::vector<std::pair<const double*, const double*>> pr;
            pr.push_back({sv, yv});
            pr.push_back({sv, sv});
            pr.push_back({yv, yv});
            for (int j = 0; j < hsz; ++j) {
                const double* sj = Sh + (size_t)slot[j] * n;
                const double* yj = Yh + (size_t)slot[j] * n;
                pr.push_back({sv, yj});
                pr.push_back({sj, yv});
                pr.push_back({yv, yj});
            }
            for (int j = 0; j < hsz; ++j) pr.push_back({Sh + (size_t)slot[j] * n, gn});
            pr.push_back({sv, gn});
            for (int j = 0; j < hsz; ++j) pr.push_back({Yh + (size_t)slot[j] * n, gn});
            pr.push_back({yv, gn});
            TRY(dots(pr, nd.data()));
        }
        const double* sg = nd.data() + 3 + 3 * hsz;   // S^T g_new (kept pairs, then the new one)
        const double* yg = sg + hsz + 1;                // Y^T g_new
        std::swap(xc, xn);
        std::swap(gc, gn);
        const double sy = nd[0], ss = nd[1], yy = nd[2];
        int first = 0;   // first kept pair after this update (1 when the oldest is dropped)
        int hk = hsz;    // pairs kept after this update
        if (sy > 1e-12 * std::sqrt(ss) * std::sqrt(yy)) {
            const int q = hsz;   // position of the new pair
            for (int j = 0; j < hsz; ++j) {
                SY[q * MM + j] = nd[3 + 3 * j];       // s_new . y_j
                SY[j * MM + q] = nd[3 + 3 * j + 1];   // s_j . y_new
                YY[q * MM + j] = YY[j * MM + q] = nd[3 + 3 * j + 2];
            }
            SY[q * MM + q] = sy;
            YY[q * MM + q] = yy;
            slot.push_back(sl);
            gamma = sy / yy;
            hk = hsz + 1;
            if ((int)slot.size() > m) {   // drop the oldest pair: shift the matrices
                free_slots.push_back(slot.front());
                slot.erase(slot.begin());
                const int h2 = (int)slot.size();
                for (int i = 0; i < h2; ++i)
                    for (int j = 0; j < h2; ++j) {
                        SY[i * MM + j] = SY[(i + 1) * MM + j + 1];
                        YY[i * MM + j] = YY[(i + 1) * MM + j + 1];
                    }
                first = 1;
                hk = h2;
            }
        } else {
            free_slots.push_back(sl);
        }
        // a = S^T g and b = Y^T g over the pairs now kept (in their order)
        for (int i = 0; i < hk; ++i) {
            av[i] = sg[first + i];
            av[hk + i] = yg[first + i];
        }
        f = fn;
        gn2 = gn2n;
        gnorm = std::sqrt(gn2n);
        ++it;
    }
    if (xc != x) HIPCHK(hipMemcpyAsync(x, xc, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->iters = it;
        out->res_norm = gnorm;
        out->status = gnorm <= gtol ? BL_OK : BL_E_NOT_CONVERGED;
        out->est = f;
    }
    return gnorm <= gtol ? BL_OK : BL_E_NOT_CONVERGED;
}

}  // extern "C"
