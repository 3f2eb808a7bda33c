// Host side of the C ABI: argument validation, workspace carving and kernel orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "stencil.h"

using namespace bl;

struct bl_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    int timing = 0;
    SolveState* h_state = nullptr;   // pinned
    double* h_buf = nullptr;         // pinned staging (>= 4096 doubles)
    int* h_info = nullptr;           // pinned
    SolveState* h_hdr = nullptr;     // pinned: two slots for the scalar header of in-flight chunks
    hipEvent_t poll_ev[2] = {};
    hipEvent_t ev[6] = {};
    std::vector<hipEvent_t> kev;     // per-launch events (timing mode 2)
    double kt[4] = {0.0, 0.0, 0.0, 0.0};
};

namespace {

constexpr int LBFGS_MMAX = 20;
constexpr int POLL = 8;              // iterations launched between host polls of the stop flag
// Consumer kernels re-reduce the producer's per-block records in every block; above this many
// record values a one-block kernel first folds them into one record (keeps the re-reads linear).
constexpr long REC_LIMIT = 8192;
constexpr size_t ALIGN = 256;

size_t al(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

int nparams(const bl_problem* P) {
    return P->reg == BL_REG_TV ? 2 : P->n_filters * (1 + P->filter_size * P->filter_size);
}

bl_status check_problem(bl_ctx* c, const bl_problem* P) {
    if (!P) return c->err = "null problem", BL_E_ARG;
    if (P->h < 2 || P->w < 2) return c->err = "image must be at least 2 x 2", BL_E_SHAPE;
    if ((long long)P->h * P->w > (1LL << 30)) return c->err = "image too large", BL_E_SHAPE;
    if (P->blur_radius < 0 || P->blur_radius > MAX_R) return c->err = "blur radius outside [0, 8]", BL_E_ARG;
    if (!(P->blur_sigma > 0.0)) return c->err = "blur sigma must be positive", BL_E_ARG;
    if (P->reg != BL_REG_TV && P->reg != BL_REG_FILTERS) return c->err = "unknown regulariser", BL_E_ARG;
    if (P->prec != BL_PREC_FP64 && P->prec != BL_PREC_MIXED) return c->err = "unknown precision", BL_E_ARG;
    if (P->reg == BL_REG_FILTERS) {
        if (P->n_filters < 1 || P->n_filters > MAX_NF) return c->err = "n_filters outside [1, 8]", BL_E_ARG;
        if (P->filter_size < 1 || P->filter_size > MAX_FS || P->filter_size % 2 == 0)
            return c->err = "filter_size must be odd in [1, 7]", BL_E_ARG;
        if (P->penalty != BL_PEN_LOG && P->penalty != BL_PEN_QUAD) return c->err = "unknown penalty", BL_E_ARG;
        if (P->eps < 0.0) return c->err = "eps must be >= 0", BL_E_ARG;
    }
    return BL_OK;
}

// Workspace layout (all offsets in bytes from the workspace base).
struct Layout {
    size_t state, fold, part, vec, maps, taps, W0, W1, Ut, Ct, small, lb, total;
    size_t part_doubles;
    int n, p, s_max, v_cap, t_max, nf;
};

Layout layout(const bl_problem* P, int s_max, int v_cap) {
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
    L.fold = o;     o += al(4 * NV_RED * sizeof(double));
    L.part = o;     o += al(3 * pd * sizeof(double));   // records: residual / apply / update (and general)
    L.vec = o;      o += al(((size_t)8 * L.n + 2 * L.p) * sizeof(double));   // 8 vectors + a p-vector
    L.maps = o;     o += al((size_t)L.nf * L.n * (2 * sizeof(double) + sizeof(float)));
    L.taps = o;     o += al((size_t)(MAX_NF * MAX_FS * MAX_FS + MAX_NF + 16) * sizeof(double));
    L.W0 = o;       o += al((size_t)L.n * L.t_max * sizeof(double));
    L.W1 = o;       o += al((size_t)L.n * L.t_max * sizeof(double));
    L.Ut = o;       o += al((size_t)L.n * std::max(s_max, 1) * sizeof(double));
    L.Ct = o;       o += al((size_t)L.n * std::max(s_max, 1) * sizeof(double));
    const size_t T2 = (size_t)L.t_max * L.t_max;
    L.small = o;
    o += al((6 * T2 + (size_t)L.p * L.t_max + 2 * (size_t)L.t_max * std::max(s_max, 1) + 256 +
             gsvd_scratch_doubles(L.t_max, L.p)) * sizeof(double) + 4 * L.t_max * sizeof(int));
    L.lb = o;       o += al(((size_t)2 * (LBFGS_MMAX + 1) * L.n + (size_t)(LBFGS_MMAX + 6) * 1024 + 64) * sizeof(double));
    L.total = o;
    return L;
}

struct WS {
    Layout L;
    char* base;
    SolveState* st() const { return (SolveState*)(base + L.state); }
    double* part() const { return (double*)(base + L.part); }
    double* part_res() const { return part(); }
    double* part_app() const { return part() + L.part_doubles; }
    double* part_upd() const { return part() + 2 * L.part_doubles; }
    double* part_fold(int k) const { return (double*)(base + L.fold) + k * NV_RED; }
    double* vec(int k) const { return (double*)(base + L.vec) + (size_t)k * L.n; }
    double* d1() const { return (double*)(base + L.maps); }
    double* d2() const { return d1() + (size_t)L.nf * L.n; }
    float* d2f() const { return (float*)(d2() + (size_t)L.nf * L.n); }
    double* taps() const { return (double*)(base + L.taps); }
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

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
            return BL_E_HIP;                                                                 \
        }                                                                                    \
    } while (0)

// Stencil description at (theta); filters: taps and weights copied to the workspace.
bl_status make_stencil(bl_ctx* c, const bl_problem* P, const double* theta, const WS& ws, Stencil& S) {
    std::memset(&S, 0, sizeof(S));
    S.h = P->h;
    S.w = P->w;
    S.n = P->h * P->w;
    S.R = P->blur_radius;
    double g[2 * MAX_R + 1], sum = 0.0;
    for (int a = -S.R; a <= S.R; ++a) {
        g[a + S.R] = std::exp(-(double)a * a / (2.0 * P->blur_sigma * P->blur_sigma));
        sum += g[a + S.R];
    }
    for (int a = 0; a <= 2 * S.R; ++a) S.g[a] = g[a] / sum;
    S.reg = P->reg;
    S.tiles_x = (P->w + TW - 1) / TW;
    S.tiles_y = (P->h + TH - 1) / TH;
    if (!theta) return c->err = "null theta", BL_E_ARG;
    if (P->reg == BL_REG_TV) {
        S.lam = std::exp(theta[0]);
        S.gam2 = std::exp(2.0 * theta[1]);
        if (!std::isfinite(S.lam) || !std::isfinite(S.gam2) || S.gam2 <= 0.0)
            return c->err = "theta gives a non-finite or zero smoothing", BL_E_ARG;
    } else {
        S.nf = P->n_filters;
        S.fs = P->filter_size;
        S.eps = P->eps;
        S.penalty = P->penalty;
        const int f2 = S.fs * S.fs;
        double* h = c->h_buf;
        for (int j = 0; j < S.nf; ++j) {
            for (int k = 0; k < f2; ++k) h[j * f2 + k] = theta[j * (1 + f2) + 1 + k];
            h[S.nf * f2 + j] = std::exp(theta[j * (1 + f2)]);
            if (!std::isfinite(h[S.nf * f2 + j])) return c->err = "theta gives a non-finite weight", BL_E_ARG;
        }
        HIPCHK(hipMemcpyAsync(ws.taps(), h, (S.nf * f2 + S.nf) * sizeof(double), hipMemcpyHostToDevice, c->stream));
        // the staging buffer is reused by later calls: make the copy complete
        HIPCHK(hipStreamSynchronize(c->stream));
        S.taps = ws.taps();
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

#define TRY(expr)                        \
    do {                                 \
        bl_status s_ = (expr);           \
        if (s_ != BL_OK) return s_;      \
    } while (0)

extern "C" {

bl_status bl_create(bl_ctx** ctx, void* hip_stream) {
    if (!ctx) return BL_E_ARG;
    bl_ctx* c = new bl_ctx();
    c->stream = (hipStream_t)hip_stream;
    if (hipHostMalloc((void**)&c->h_state, sizeof(SolveState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_buf, 8192 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_info, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_hdr, 2 * sizeof(SolveState), hipHostMallocDefault) != hipSuccess) {
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
    HIPCHK(launch_hvp(S, P->prec == BL_PREC_MIXED, xhat, v, out, ncols, c->stream));
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
bl_status bl_hessian_solve(bl_ctx* c, const bl_problem* P, const double* theta, const double* xhat, const double* g,
                           double* w, bl_recycle* rs, const bl_solve_opts* o, void* wsp, size_t ws_bytes,
                           bl_stats* out) {
    if (!c) return BL_E_ARG;
    TRY(check_problem(c, P));
    if (!xhat || !g || !w || !o) return c->err = "null argument", BL_E_ARG;
    if (o->max_iter < 0 || o->check_every < 1 || o->rr_every < 0 || !(o->tol >= 0.0))
        return c->err = "invalid solve options", BL_E_ARG;
    if (o->stop != BL_STOP_RESID && o->stop != BL_STOP_HGERR) return c->err = "unknown stop rule", BL_E_ARG;
    const int s = rs ? rs->s_cur : 0;
    const int s_max = rs ? rs->s_max : 0, v_cap = rs ? rs->v_cap : 0;
    if (rs) {
        if (s < 0 || s > s_max || s_max > S_MAX) return c->err = "s_cur outside [0, s_max] or s_max > 64", BL_E_SHAPE;
        if (s > 0 && (!rs->U || !rs->C || !rs->mu)) return c->err = "null recycle arrays", BL_E_ARG;
        if (o->store_basis && (!rs->V || v_cap < 1)) return c->err = "store_basis needs V", BL_E_ARG;
    }
    const bool hg = o->stop == BL_STOP_HGERR && s > 0 && rs->Z;
    WS ws;
    TRY(check_ws(c, layout(P, s_max, v_cap), wsp, ws_bytes, ws));
    const int n = P->h * P->w;
    Stencil S;
    mark(c, 0);
    TRY(make_stencil(c, P, theta, ws, S));
    TRY(filter_state(c, S, xhat, ws));
    // device scalars
    SolveState* hs = c->h_state;
    std::memset(hs, 0, sizeof(SolveState));
    hs->tol = o->tol;
    hs->hg_tol = o->hg_tol;
    hs->max_iter = o->max_iter;
    hs->check_every = o->check_every;
    hs->stop = o->stop;
    hs->s = s;
    hs->v_cap = (o->store_basis && rs) ? v_cap : 0;
    hs->store_basis = (o->store_basis && rs) ? 1 : 0;
    hs->hgerr_on = hg ? 1 : 0;
    SolveState* st = ws.st();
    HIPCHK(hipMemcpyAsync(st, hs, sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
    if (s > 0) HIPCHK(hipMemcpyAsync(st->mu, rs->mu, s * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    const double* U = s ? rs->U : nullptr;
    const double* C = s ? rs->C : nullptr;
    const double* Z = hg ? rs->Z : nullptr;
    double* V = (o->store_basis && rs) ? rs->V : nullptr;
    double* r = ws.vec(0);
    double* pb[2] = {ws.vec(1), ws.vec(2)};
    double* q = ws.vec(3);
    const bool fp32 = P->prec == BL_PREC_MIXED;
    const int tiles = tiles_of(S), nb1 = red_blocks(n);
    double* prs = ws.part_res();
    double* pap = ws.part_app();
    double* pup = ws.part_upd();
    // Records handed from kernel to kernel: (pointer, number of blocks), folded when large.
    auto fold = [&](double* part, int nb, int nv, int slot, const double*& out, int& out_nb) -> bl_status {
        if ((long)nb * nv > REC_LIMIT) {
            HIPCHK(launch_finish_sum(part, nb, nv, ws.part_fold(slot), c->stream));
            out = ws.part_fold(slot);
            out_nb = 1;
        } else {
            out = part;
            out_nb = nb;
        }
        return BL_OK;
    };
    const int nz = hg ? s : 0;
    const double* rec;
    int rec_nb;
    // r = g - H w0 (FP64) with record [g.g, C^T r];  w += U c0;  r -= C c0
    HIPCHK(launch_residual(S, xhat, w, g, r, C, s, prs, c->stream));
    TRY(fold(prs, tiles, 1 + s, 0, rec, rec_nb));
    HIPCHK(launch_cg_init(n, w, r, U, C, Z, st, rec, rec_nb, pup, c->stream));
    mark(c, 1);
    const int rr_every = fp32 ? o->rr_every : 0;
    const bool ktime = c->timing == 2;
    std::vector<int> launched;   // iteration index of each timed launch triple
    // Iteration j = apply(j) [stop test on r_j, p, q = H p] + update(j) [alpha, w, r].  The
    // last index j = max_iter launches apply only: it tests r_max_iter.
    int j = 0;
    auto launch_iter = [&]() -> bl_status {
        if (ktime) {
            const size_t need = 3 * (launched.size() + 1);
            while (c->kev.size() < need) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                c->kev.push_back(e);
            }
            HIPCHK(hipEventRecord(c->kev[3 * launched.size()], c->stream));
        }
        const double* ru;
        int ru_nb;
        TRY(fold(pup, nb1, 1 + nz, 1, ru, ru_nb));
        HIPCHK(launch_cg_apply(S, fp32, j, xhat, r, pb[j & 1], pb[(j + 1) & 1], q, C, V, st, ru, ru_nb, pap,
                               c->stream));
        if (ktime) HIPCHK(hipEventRecord(c->kev[3 * launched.size() + 1], c->stream));
        if (j < o->max_iter) {
            const double* ra;
            int ra_nb;
            TRY(fold(pap, tiles, 1 + s, 2, ra, ra_nb));
            HIPCHK(launch_cg_update(n, j, w, r, pb[(j + 1) & 1], q, C, Z, st, ra, ra_nb, pup, c->stream));
        }
        if (ktime) {
            HIPCHK(hipEventRecord(c->kev[3 * launched.size() + 2], c->stream));
            launched.push_back(j);
        }
        ++j;
        return BL_OK;
    };
    const size_t hdr = offsetof(SolveState, e);
    if (!rr_every) {
        // Chunks of POLL iterations; the next chunk is enqueued before the host waits for the
        // stop flag of the previous one, so the device never idles on a poll.  Iterations
        // launched after the stop exit at once (the kernels test the device flag).
        auto enqueue = [&](int chunk) -> bl_status {
            for (int k = 0; k < POLL && j <= o->max_iter; ++k) TRY(launch_iter());
            HIPCHK(hipMemcpyAsync(&c->h_hdr[chunk & 1], st, hdr, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipEventRecord(c->poll_ev[chunk & 1], c->stream));
            return BL_OK;
        };
        int chunk = 0;
        TRY(enqueue(0));
        for (;;) {
            const bool more = j <= o->max_iter;
            if (more) TRY(enqueue(chunk + 1));
            HIPCHK(hipEventSynchronize(c->poll_ev[chunk & 1]));
            if (c->h_hdr[chunk & 1].done || !more) break;
            ++chunk;
        }
    } else {
        for (;;) {
            const int chunk = std::min(POLL, rr_every - (j % rr_every));
            for (int k = 0; k < chunk && j <= o->max_iter; ++k) TRY(launch_iter());
            HIPCHK(hipMemcpyAsync(hs, st, hdr, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            const bool converged = hs->done && hs->status == BL_OK;
            if (hs->done && !converged) break;
            if (!converged && j % rr_every != 0 && j <= o->max_iter) continue;
            if (!converged && j > o->max_iter) break;
            // residual replacement in FP64: r = g - H w, z = C^T r, r -= C z; the apply step
            // of the current index re-tests (and goes on if the true residual misses the test)
            if (converged) j = hs->iters;
            HIPCHK(launch_residual(S, xhat, w, g, r, C, s, prs, c->stream));
            TRY(fold(prs, tiles, 1 + s, 0, rec, rec_nb));
            HIPCHK(launch_cg_replace(n, r, C, Z, st, rec, rec_nb, pup, c->stream));
            TRY(launch_iter());
            HIPCHK(hipMemcpyAsync(hs, st, hdr, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            if (hs->done || j > o->max_iter) break;
        }
    }
    mark(c, 2);
    if (s > 0) HIPCHK(launch_cg_finish(n, w, U, st, c->stream));
    mark(c, 3);
    HIPCHK(hipMemcpyAsync(hs, st, sizeof(SolveState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    int status = hs->done ? hs->status : BL_E_NOT_CONVERGED;
    if (ktime) {   // durations of launches whose iteration actually ran
        for (size_t u = 0; u < launched.size(); ++u) {
            if (launched[u] >= hs->iters + (status == BL_E_INDEFINITE ? 1 : 0)) break;
            float a = 0.f, b = 0.f;
            HIPCHK(hipEventElapsedTime(&a, c->kev[3 * u], c->kev[3 * u + 1]));
            HIPCHK(hipEventElapsedTime(&b, c->kev[3 * u + 1], c->kev[3 * u + 2]));
            c->kt[0] += a;
            c->kt[1] += 1.0;
            c->kt[2] += b;
            c->kt[3] += 1.0;
        }
    }
    if (rs && o->store_basis) {
        int nv = hs->iters + (status == BL_E_INDEFINITE ? 1 : 0);
        rs->v_cur = std::min(nv, v_cap);
    }
    if (out) {
        out->iters = hs->iters;
        out->status = status;
        out->t = 0;
        out->s_cur = s;
        out->res_norm = std::sqrt(std::max(hs->rho2[hs->iters & 1], 0.0));
        out->res0_norm = hs->res0;
        out->g_norm = hs->gnorm;
        out->est = hs->est;
        out->ms[0] = elapsed(c, 0, 1);
        out->ms[1] = elapsed(c, 1, 2);
        out->ms[2] = elapsed(c, 2, 3);
        out->ms[3] = elapsed(c, 0, 3);
    }
    return (bl_status)status;
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
    WS ws;
    TRY(check_ws(c, layout(P, rs->s_max, rs->v_cap), wsp, ws_bytes, ws));
    const int n = P->h * P->w, p = nparams(P);
    const int t0 = rs->s_cur + rs->v_cur;
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
    int* ibuf = (int*)(gsc + gsvd_scratch_doubles(tm, p));
    int* kept = ibuf;
    int* tk_dev = ibuf + tm;
    int* info = ibuf + tm + 4;
    // W0 = [U, V]
    double* W0 = ws.W0();
    double* W1 = ws.W1();
    if (rs->s_cur)
        HIPCHK(hipMemcpyAsync(W0, rs->U, (size_t)rs->s_cur * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (rs->v_cur)
        HIPCHK(hipMemcpyAsync(W0 + (size_t)rs->s_cur * n, rs->V, (size_t)rs->v_cur * n * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    // two passes of Cholesky QR with column drop: W = [U, V] X1 X2
    HIPCHK(launch_gram(n, t0, t0, W0, W0, ws.part(), Gram, c->stream));
    HIPCHK(launch_chol_drop(t0, Gram, o->rank_tol, Achol, kept, tk_dev, Xinv, t0, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_info, tk_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int t1 = c->h_info[0];
    if (t1 == 0) {
        rs->s_cur = 0;
        return BL_E_RANK;
    }
    HIPCHK(launch_gemm_tall(n, t0, t1, W0, Xinv, t0, W1, c->stream));
    HIPCHK(launch_gram(n, t1, t1, W1, W1, ws.part(), Gram, c->stream));
    HIPCHK(launch_chol_drop(t1, Gram, 1e-12, Achol, kept, tk_dev, Xinv, t1, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_info, tk_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int t = c->h_info[0];
    HIPCHK(launch_gemm_tall(n, t1, t, W1, Xinv, t1, W0, c->stream));   // W (orthonormal) in W0
    mark(c, 1);
    // Y = H W (FP64), M = W^T Y, G = J W
    HIPCHK(launch_hvp(S, false, xhat, W0, W1, t, c->stream));
    HIPCHK(launch_gram(n, t, t, W0, W1, ws.part(), M, c->stream));
    HIPCHK(launch_jac(S, xhat, W0, t, ws.d1(), ws.d2(), ws.part(), Gj, 1, c->stream));
    mark(c, 2);
    HIPCHK(launch_gsvd_select(t, p, o->s, M, Gj, gsc, Xs, VHs, mu_tmp, info, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_info, info, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int s_eff = c->h_info[0], rankG = c->h_info[1], gst = c->h_info[2];
    if (gst != BL_OK) {
        rs->s_cur = 0;
        c->err = "projected Hessian W^T H W is not positive definite";
        return (bl_status)gst;
    }
    // U~ = W X~, C~ = Y X~, Z = W V_H~
    HIPCHK(launch_gemm_tall(n, t, s_eff, W0, Xs, t, ws.Ut(), c->stream));
    HIPCHK(launch_gemm_tall(n, t, s_eff, W1, Xs, t, ws.Ct(), c->stream));
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
    const int vb = vec_blocks(n);
    double* g = ws.vec(0);
    double* d = ws.vec(1);
    double* xt = ws.vec(2);
    double* gt = ws.vec(3);
    double* qv = ws.vec(4);
    double* Sh = ws.lb();
    double* Yh = Sh + (size_t)(LBFGS_MMAX + 1) * n;
    double* dq_rec = Yh + (size_t)(LBFGS_MMAX + 1) * n;   // records of s_k . q, one per slot
    double* dr_rec = dq_rec + (size_t)(LBFGS_MMAX + 1) * vb;
    double* d3_rec = dr_rec + vb;                           // [s.y, s.s, y.y] records
    double* sl_rec = d3_rec + 3 * (size_t)vb;               // g . d records
    double* fout = sl_rec + vb;                             // host-bound scalars
    auto grad_at = [&](const double* xx, double* gg, double& f, double& gn2) -> bl_status {
        HIPCHK(launch_lower_grad(S, xx, y, gg, ws.part(), c->stream));
        HIPCHK(launch_finish_sum(ws.part(), tiles_of(S), 2, fout, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_buf, fout, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        f = c->h_buf[0];
        gn2 = c->h_buf[1];
        return BL_OK;
    };
    double f, gn2;
    TRY(grad_at(x, g, f, gn2));
    std::vector<double> rho;
    std::vector<int> slot;   // history slots in use, oldest first
    std::vector<int> free_slots;
    for (int k = m; k >= 0; --k) free_slots.push_back(k);   // m + 1 buffers: a new pair never overwrites a kept one
    int it = 0;
    double gnorm = std::sqrt(gn2);
    double gamma = 0.0;
    while (gnorm > gtol && it < max_iter) {
        if (!std::isfinite(f) || !std::isfinite(gnorm)) return c->err = "non-finite objective", BL_E_NONFINITE;
        // two-loop recursion with the coefficients kept on the device: q = g, d = H_k q
        HIPCHK(hipMemcpyAsync(qv, g, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        const int hsz = (int)slot.size();
        for (int k = hsz - 1; k >= 0; --k) {
            const double* sk = Sh + (size_t)slot[k] * n;
            const double* yk = Yh + (size_t)slot[k] * n;
            double* rec = dq_rec + (size_t)slot[k] * vb;
            HIPCHK(launch_dots_part(n, 1, sk, qv, rec, c->stream));
            HIPCHK(launch_axpy_red(n, 1.0, qv, yk, rec, -rho[k], nullptr, 0.0, c->stream));
        }
        const double scale0 = hsz ? gamma : 1.0 / gnorm;
        HIPCHK(launch_axpy_red(n, 0.0, d, qv, nullptr, scale0, nullptr, 0.0, c->stream));
        for (int k = 0; k < hsz; ++k) {
            const double* sk = Sh + (size_t)slot[k] * n;
            const double* yk = Yh + (size_t)slot[k] * n;
            HIPCHK(launch_dots_part(n, 1, yk, d, dr_rec, c->stream));
            HIPCHK(launch_axpy_red(n, 1.0, d, sk, dq_rec + (size_t)slot[k] * vb, rho[k], dr_rec, -rho[k], c->stream));
        }
        // direction -d; slope = -(g . d)
        HIPCHK(launch_dots_part(n, 1, g, d, sl_rec, c->stream));
        HIPCHK(launch_finish_sum(sl_rec, vb, 1, fout + 2, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_buf, fout + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double slope = -c->h_buf[0];
        if (!(slope < 0.0)) {   // not a descent direction: steepest descent
            HIPCHK(hipMemcpyAsync(d, g, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            slope = -gnorm * gnorm;
        }
        // backtracking Armijo on x - t d
        double tstep = 1.0, fn = 0.0, gn2n = 0.0;
        bool ok = false;
        for (int bt = 0; bt < 60; ++bt) {
            HIPCHK(hipMemcpyAsync(xt, x, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(launch_axpy_red(n, 1.0, xt, d, nullptr, -tstep, nullptr, 0.0, c->stream));
            TRY(grad_at(xt, gt, fn, gn2n));
            if (fn <= f + 1e-4 * tstep * slope) {
                ok = true;
                break;
            }
            tstep *= 0.5;
        }
        if (!ok) break;
        // new pair s = xt - x, y = gt - g
        const int sl = free_slots.back();
        free_slots.pop_back();
        double* sv = Sh + (size_t)sl * n;
        double* yv = Yh + (size_t)sl * n;
        HIPCHK(launch_sub(n, xt, x, sv, c->stream));
        HIPCHK(launch_sub(n, gt, g, yv, c->stream));
        HIPCHK(launch_dots_part(n, 3, sv, yv, d3_rec, c->stream));
        HIPCHK(launch_finish_sum(d3_rec, vb, 3, fout + 3, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_buf, fout + 3, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(x, xt, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(g, gt, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const double sy = c->h_buf[0], ss = c->h_buf[1], yy = c->h_buf[2];
        if (sy > 1e-12 * std::sqrt(ss) * std::sqrt(yy)) {
            slot.push_back(sl);
            rho.push_back(1.0 / sy);
            gamma = sy / yy;
            if ((int)slot.size() > m) {
                free_slots.push_back(slot.front());
                slot.erase(slot.begin());
                rho.erase(rho.begin());
            }
        } else {
            free_slots.push_back(sl);
        }
        f = fn;
        gnorm = std::sqrt(gn2n);
        ++it;
    }
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
