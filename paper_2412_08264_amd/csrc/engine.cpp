// Batched recycled CG (host side): slot admission, block maps, chunked pipelined stepping,
// mixed-precision residual replacement and retirement; the C-ABI engine and the batched
// solve built on it.  Recycled CG as in Section 2.2.2 (Galerkin counterpart of RMINRES),
// stop tests of Section 4.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "host.h"
#include "tile.h"

using namespace bl;

namespace blh {

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

bl_status check_solve_opts(bl_ctx* c, const bl_solve_opts* o) {
    if (!o) return c->err = "null solve options", BL_E_ARG;
    if (o->max_iter < 0 || o->check_every < 1 || o->rr_every < 0 || !(o->tol >= 0.0))
        return c->err = "invalid solve options", BL_E_ARG;
    if (o->stop != BL_STOP_RESID && o->stop != BL_STOP_HGERR) return c->err = "unknown stop rule", BL_E_ARG;
    return BL_OK;
}

void class_stencil(const bl_problem* P, Stencil& S) {
    std::memset(&S, 0, sizeof(S));
    S.R = P->blur_radius;
    double g[2 * MAX_R + 1], sum = 0.0;
    for (int a = -S.R; a <= S.R; ++a) {
        g[a + S.R] = std::exp(-(double)a * a / (2.0 * P->blur_sigma * P->blur_sigma));
        sum += g[a + S.R];
    }
    for (int a = 0; a <= 2 * S.R; ++a) S.g[a] = g[a] / sum;
    S.reg = P->reg;
    if (P->reg == BL_REG_FILTERS) {
        S.nf = P->n_filters;
        S.fs = P->filter_size;
        S.eps = P->eps;
        S.penalty = P->penalty;
    }
}

bl_status theta_values(bl_ctx* c, const bl_problem* P, const double* theta, double& lam, double& gam2,
                       double* taps_host) {
    if (!theta) return c->err = "null theta", BL_E_ARG;
    lam = gam2 = 0.0;
    if (P->reg == BL_REG_TV) {
        lam = std::exp(theta[0]);
        gam2 = std::exp(2.0 * theta[1]);
        if (!std::isfinite(lam) || !std::isfinite(gam2) || gam2 <= 0.0)
            return c->err = "theta gives a non-finite or zero smoothing", BL_E_ARG;
        return BL_OK;
    }
    const int nf = P->n_filters, f2 = P->filter_size * P->filter_size;
    for (int j = 0; j < nf; ++j) {
        for (int k = 0; k < f2; ++k) taps_host[j * f2 + k] = theta[j * (1 + f2) + 1 + k];
        taps_host[nf * f2 + j] = std::exp(theta[j * (1 + f2)]);
        if (!std::isfinite(taps_host[nf * f2 + j])) return c->err = "theta gives a non-finite weight", BL_E_ARG;
    }
    float* tf = reinterpret_cast<float*>(taps_host + TAPS_MAX);
    for (int k = 0; k < nf * f2 + nf; ++k) tf[k] = (float)taps_host[k];
    return BL_OK;
}

bool same_class(const bl_problem* a, const bl_problem* b) {
    if (a->blur_radius != b->blur_radius || a->blur_sigma != b->blur_sigma || a->reg != b->reg || a->prec != b->prec)
        return false;
    if (a->reg == BL_REG_FILTERS)
        return a->n_filters == b->n_filters && a->filter_size == b->filter_size && a->eps == b->eps &&
               a->penalty == b->penalty;
    return true;
}

static int ntiles_of(int h, int w, int rows) { return ((w + QW - 1) / QW) * ((h + rows - 1) / rows); }
static int npix_of(long n) { return (int)((n + NT - 1) / NT); }

// ------------------------------------------------------------------------------ tile heights
// Rows per tile of the recycled-CG Hessian-vector kernels: a process-wide table keyed by the
// operator class and the size class floor(log2 n), filled by the autotuner (or by the caller
// from a stored table); without an entry the tallest tile that still gives the image at least
// one block per compute unit, else the shortest.  A solve keeps the height it was admitted
// with; solves of different heights run in different launches.
namespace {
using TileKey = std::tuple<int, int, int, int, int, int>;   // reg, radius, filters, size, prec, log2 n
std::mutex tile_mu;
std::map<TileKey, int> tile_table;
constexpr int FILL_BLOCKS = 256;

int log2_floor(long n) {
    int k = 0;
    while (n > 1) {
        n >>= 1;
        ++k;
    }
    return k;
}
TileKey tile_key(const bl_problem* P) {
    const bool f = P->reg == BL_REG_FILTERS;
    return TileKey(P->reg, P->blur_radius, f ? P->n_filters : 0, f ? P->filter_size : 0, P->prec,
                   log2_floor((long)P->h * P->w));
}
}  // namespace

bool valid_rows(int rows) { return rows == QTY || rows == 2 * QTY || rows == 4 * QTY; }

int default_rows(const bl_problem* P) {
    for (int rows = 4 * QTY; rows > QTY; rows /= 2)
        if (ntiles_of(P->h, P->w, rows) >= FILL_BLOCKS) return rows;
    return QTY;
}

int tile_rows(const bl_problem* P) {
    std::lock_guard<std::mutex> lk(tile_mu);
    const auto it = tile_table.find(tile_key(P));
    return it == tile_table.end() ? default_rows(P) : it->second;
}

void set_tile_rows(const bl_problem* P, int rows) {
    std::lock_guard<std::mutex> lk(tile_mu);
    if (rows == 0) tile_table.erase(tile_key(P));
    else tile_table[tile_key(P)] = rows;
}

// Tile cache file: one line per entry, "reg radius n_filters filter_size prec log2n rows us8 us16
// us32" (the key of the table, the chosen height and the timings that chose it); '#' starts a
// comment line.  The whole file is parsed before it is used or rewritten, so a malformed file is
// reported instead of being overwritten.
namespace {
struct CacheLine {
    int rows;
    double us[3];
};
bool read_tile_cache(const char* path, std::map<TileKey, CacheLine>& out, bool& exists, std::string& err) {
    out.clear();
    FILE* f = std::fopen(path, "r");
    exists = f != nullptr;
    if (!f) return true;
    char line[512];
    int lineno = 0;
    bool ok = true;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        const char* q = line;
        while (*q == ' ' || *q == '\t') ++q;
        if (*q == '#' || *q == '\n' || *q == '\0') continue;
        int k[7];
        double us[3];
        if (std::sscanf(q, "%d %d %d %d %d %d %d %lf %lf %lf", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6], &us[0],
                        &us[1], &us[2]) != 10 ||
            !valid_rows(k[6])) {
            err = std::string("malformed tile cache line ") + std::to_string(lineno) + " in " + path;
            ok = false;
            break;
        }
        out[TileKey(k[0], k[1], k[2], k[3], k[4], k[5])] = CacheLine{k[6], {us[0], us[1], us[2]}};
    }
    std::fclose(f);
    return ok;
}
}  // namespace

bool tile_cache_lookup(const char* path, const bl_problem* P, int& rows, bool& found, std::string& err) {
    std::map<TileKey, CacheLine> m;
    bool exists = false;
    found = false;
    if (!read_tile_cache(path, m, exists, err)) return false;
    const auto it = m.find(tile_key(P));
    if (it != m.end()) {
        found = true;
        rows = it->second.rows;
    }
    return true;
}

bool tile_cache_load_all(const char* path, int& entries, std::string& err) {
    std::map<TileKey, CacheLine> m;
    bool exists = false;
    entries = 0;
    if (!read_tile_cache(path, m, exists, err)) return false;
    if (!exists) {
        err = std::string("cannot read ") + path;
        return false;
    }
    std::lock_guard<std::mutex> lk(tile_mu);
    for (const auto& kv : m) tile_table[kv.first] = kv.second.rows;
    entries = (int)m.size();
    return true;
}

bool tile_cache_store(const char* path, const bl_problem* P, int rows, const double us[3], std::string& err) {
    std::map<TileKey, CacheLine> m;
    bool exists = false;
    if (!read_tile_cache(path, m, exists, err)) return false;
    m[tile_key(P)] = CacheLine{rows, {us[0], us[1], us[2]}};
    // written next to the target and renamed over it: readers see the old or the new file whole
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) {
        err = std::string("cannot write ") + tmp;
        return false;
    }
    std::fprintf(f, "# bilevel tile cache: reg radius n_filters filter_size prec log2n rows us8 us16 us32\n");
    for (const auto& kv : m) {
        const TileKey& k = kv.first;
        std::fprintf(f, "%d %d %d %d %d %d %d %.3f %.3f %.3f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                     std::get<3>(k), std::get<4>(k), std::get<5>(k), kv.second.rows, kv.second.us[0], kv.second.us[1],
                     kv.second.us[2]);
    }
    const bool wrote = std::fclose(f) == 0;
    if (!wrote || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        err = std::string("cannot replace ") + path;
        return false;
    }
    return true;
}

// Records are sized for the shortest tiles (the most tiles), whatever height a solve uses.
size_t slot_bytes(const bl_problem* P, int s) {
    const size_t n = (size_t)P->h * P->w;
    const size_t nf = P->reg == BL_REG_FILTERS ? P->n_filters : 0;
    const size_t nt = ntiles_of(P->h, P->w, QTY), np = npix_of((long)n);
    return 6 * al(n * 8) + al(n * s * 8) + al((size_t)s * s * 8) + 2 * al(nf * n * 8) + al(nf * n * 4) +
           al(TAPS_BYTES) +
           al(nt * (1 + s) * 8) + 2 * al(nt * (4 + 2 * s) * 8) + al(np * (1 + s) * 8) +
           al((size_t)3 * FOLD_BLOCKS * NV_RED * 8);
}

SlotBuffers carve_slot(char* base, const bl_problem* P, int s) {
    const size_t n = (size_t)P->h * P->w;
    const size_t nf = P->reg == BL_REG_FILTERS ? P->n_filters : 0;
    const size_t nt = ntiles_of(P->h, P->w, QTY), np = npix_of((long)n);
    SlotBuffers B{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base + o;
        o += al(bytes);
        return p;
    };
    B.r = (double*)take(n * 8);
    B.p0 = (double*)take(n * 8);
    B.p1 = (double*)take(n * 8);
    B.q = (double*)take(n * 8);
    B.r2 = (double*)take(n * 8);
    B.q2 = (double*)take(n * 8);
    B.HC = (double*)take(n * s * 8);
    B.M = (double*)take((size_t)s * s * 8);
    B.mpart = B.p0;   // p0, p1, q, r2: consecutive, free until the set-up
    B.d1 = nf ? (double*)take(nf * n * 8) : nullptr;
    B.d2 = nf ? (double*)take(nf * n * 8) : nullptr;
    B.d2f = nf ? (float*)take(nf * n * 4) : nullptr;
    B.taps = (double*)take(TAPS_BYTES);
    B.rec_res = (double*)take(nt * (1 + s) * 8);
    B.rec_app = (double*)take(nt * (4 + 2 * s) * 8);
    B.rec_upd = (double*)take(np * (1 + s) * 8);
    B.rec_app2 = (double*)take(nt * (4 + 2 * s) * 8);
    B.fold = (double*)take((size_t)3 * FOLD_BLOCKS * NV_RED * 8);
    B.st = nullptr;
    return B;
}

// ------------------------------------------------------------------------------------- Batch
Batch::~Batch() {
    if ((graph_cache.empty() && retired.empty()) || !c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : graph_cache) (void)hipGraphExecDestroy(kv.second);
    for (hipGraphExec_t ex : retired) (void)hipGraphExecDestroy(ex);
}

bl_status Batch::init(bl_ctx* ctx, int capacity, Slot* slots, int* ctr_dev, char* hdr_pinned,
                      hipEvent_t ev0, hipEvent_t ev1) {
    c = ctx;
    groups.clear();
    cap = capacity;
    d_slots = slots;
    d_ctr = ctr_dev;
    HIPCHK(hipMemsetAsync(d_ctr, 0, sizeof(int), c->stream));
    h_hdr = hdr_pinned;
    poll_ev[0] = ev0;
    poll_ev[1] = ev1;
    S.assign(cap, Host());
    step = 0;
    chunk_id = 0;
    dirty = true;
    return BL_OK;
}

int Batch::running() const {
    int k = 0;
    for (const Host& h : S) k += h.running ? 1 : 0;
    return k;
}

// Tile-grid maps give every slot a multiple of 8 blocks (the XCD-aware tile order of a slot
// starts on XCD 0); padding blocks return at once.
static BatchMap make_map(const std::vector<Batch::Host>& S, const std::vector<int>& idx, bool tiles) {
    BatchMap M{};
    M.ns = (int)idx.size();
    int off = 0;
    for (int k = 0; k < M.ns; ++k) {
        const Slot& d = S[idx[k]].d;
        M.slot[k] = idx[k];
        M.off[k] = off;
        off += tiles ? (d.ntiles + 7) / 8 * 8 : d.npix;
    }
    M.off[M.ns] = off;
    return M;
}

// Outdated graphs wait in `retired` until run() has drained the stream.
void Batch::drop_graphs() {
    for (auto& kv : graph_cache) retired.push_back(kv.second);
    graph_cache.clear();
    seen.clear();
}

bl_status Batch::rebuild() {
    ++gen;
    drop_graphs();
    run_list.clear();
    for (int i = 0; i < cap; ++i)
        if (S[i].running) run_list.push_back(i);
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        std::vector<int> mine;
        for (int i : run_list)
            if (S[i].group == gi) mine.push_back(i);
        groups[gi].tmap = make_map(S, mine, true);
    }
    std::vector<int> two;
    for (int i : run_list)
        if (!S[i].d.fused) two.push_back(i);
    pmap = make_map(S, two, false);
    fold_app = BatchMap{};
    fold_upd = BatchMap{};
    fold_fused = BatchMap{};
    for (int i : run_list) {
        if (S[i].d.fused) {
            if (S[i].d.fold_app || S[i].d.fold_upd) fold_fused.slot[fold_fused.ns++] = i;
            continue;
        }
        if (S[i].d.fold_app) fold_app.slot[fold_app.ns++] = i;
        if (S[i].d.fold_upd) fold_upd.slot[fold_upd.ns++] = i;
    }
    dirty = false;
    return BL_OK;
}

bl_status Batch::admit(int idx, const SolveSpec& sp, const SlotBuffers& B, double* taps_stage) {
    const bl_problem* P = sp.P;
    const bl_solve_opts* o = sp.o;
    bl_recycle* rs = sp.rs;
    if (idx < 0 || idx >= cap || S[idx].used) return c->err = "slot index in use or out of range", BL_E_ARG;
    TRY(check_problem(c, P));
    if (!sp.xhat || !sp.g || !sp.w) return c->err = "null argument", BL_E_ARG;
    TRY(check_solve_opts(c, o));
    const int s = rs ? rs->s_cur : 0;
    const int s_max = rs ? rs->s_max : 0, v_cap = rs ? rs->v_cap : 0;
    if (rs) {
        if (s < 0 || s > s_max || s_max > S_MAX) return c->err = "s_cur outside [0, s_max] or s_max > 64", BL_E_SHAPE;
        if (s > 0 && (!rs->U || !rs->C || !rs->mu)) return c->err = "null recycle arrays", BL_E_ARG;
        if (o->store_basis && (!rs->V || v_cap < 1)) return c->err = "store_basis needs V", BL_E_ARG;
    }
    const bool hg = o->stop == BL_STOP_HGERR && s > 0 && rs->Z;
    const bool store = o->store_basis && rs;
    const int rows = c->force_rows ? c->force_rows : tile_rows(P);
    int gid = -1;
    for (int gi = 0; gi < (int)groups.size() && gid < 0; ++gi)
        if (groups[gi].users > 0 && same_class(&groups[gi].cls, P) && groups[gi].rows == rows &&
            groups[gi].rec == (s > 0))
            gid = gi;
    for (int gi = 0; gi < (int)groups.size() && gid < 0; ++gi)
        if (groups[gi].users == 0) gid = gi;   // reuse an idle entry
    if (gid < 0) {
        if ((int)groups.size() >= MAX_GROUPS)
            return c->err = "more than 16 (operator class, tile height, recycling) groups in one batch", BL_E_ARG;
        groups.emplace_back();
        gid = (int)groups.size() - 1;
    }
    Group& grp = groups[gid];
    if (grp.users == 0) {
        grp.cls = *P;
        class_stencil(P, grp.base);
        grp.fp32 = P->prec == BL_PREC_MIXED;
        grp.rows = rows;
        grp.rec = s > 0;
    }
    const Stencil& base = grp.base;
    double lam, gam2;
    TRY(theta_values(c, P, sp.theta, lam, gam2, taps_stage));
    const int n = P->h * P->w;
    Slot v{};
    v.h = P->h;
    v.width = P->w;
    v.n = n;
    v.tiles_x = (P->w + QW - 1) / QW;
    v.ntiles = ntiles_of(P->h, P->w, rows);
    v.rows = rows;
    v.npix = npix_of(n);
    v.j0 = step;
    v.s = s;
    v.nz = hg ? s : 0;
    v.fused = grp.fp32 ? 0 : 1;
    v.fold_res = (long)v.ntiles * (1 + s) > REC_LIMIT;
    v.fold_app = v.fused ? fused_fold(v.ntiles, rows, s, v.nz) : v.fold_res;
    v.fold_upd = (long)v.npix * (1 + v.nz) > REC_LIMIT;
    v.lam = lam;
    v.gam2 = gam2;
    v.xhat = sp.xhat;
    v.g = sp.g;
    v.w = sp.w;
    v.r = B.r;
    v.p[0] = B.p0;
    v.p[1] = B.p1;
    v.q = B.q;
    v.r2 = B.r2;
    v.q2 = B.q2;
    v.HC = (v.fused && s) ? B.HC : nullptr;
    v.M = (v.fused && s) ? B.M : nullptr;
    v.U = s ? rs->U : nullptr;
    v.C = s ? rs->C : nullptr;
    v.Z = hg ? rs->Z : nullptr;
    v.V = store ? rs->V : nullptr;
    v.lz = store ? rs->lz : nullptr;
    v.st = B.st;
    v.rec_res = B.rec_res;
    v.rec_app = B.rec_app;
    v.rec_upd = B.rec_upd;
    v.rec_app2 = B.rec_app2;
    v.fold = B.fold;
    if (P->reg == BL_REG_FILTERS) {
        const int nf = P->n_filters, f2 = P->filter_size * P->filter_size;
        HIPCHK(hipMemcpyAsync(B.taps, taps_stage, TAPS_MAX * sizeof(double) + (size_t)(nf * f2 + nf) * sizeof(float),
                              hipMemcpyHostToDevice, c->stream));
        v.taps = B.taps;
        v.tapsf = reinterpret_cast<const float*>(B.taps + TAPS_MAX);
        v.lamj = B.taps + nf * f2;
        v.d2 = B.d2;
        v.d2f = B.d2f;
        Stencil Sx = base;
        Sx.h = P->h;
        Sx.w = P->w;
        Sx.n = n;
        Sx.tiles_x = v.tiles_x;
        Sx.tiles_y = (P->h + TH - 1) / TH;
        Sx.taps = v.taps;
        Sx.tapsf = v.tapsf;
        Sx.lamj = v.lamj;
        Sx.d2 = v.d2;
        Sx.d2f = v.d2f;
        HIPCHK(launch_filter_state(Sx, sp.xhat, B.d1, B.d2, B.d2f, c->stream));
    }
    if (v.fused && s) {   // H C and C^T H C for the fused steps: s FP64 products at (xhat, theta)
        Stencil Sx = base;
        Sx.h = P->h;
        Sx.w = P->w;
        Sx.n = n;
        Sx.tiles_x = v.tiles_x;
        Sx.tiles_y = (P->h + TH - 1) / TH;
        Sx.lam = lam;
        Sx.gam2 = gam2;
        Sx.taps = v.taps;
        Sx.tapsf = v.tapsf;
        Sx.lamj = v.lamj;
        Sx.d2 = v.d2;
        Sx.d2f = v.d2f;
        HIPCHK(launch_hvp(Sx, false, sp.xhat, rs->C, B.HC, s, 4 * QTY, c->stream));
        HIPCHK(launch_gram_n(n, s, s, rs->C, B.HC, mhc_chunks(n, s), B.mpart, B.M, c->stream));
    }
    StateInit init{o->tol, o->hg_tol, o->max_iter, o->check_every, o->stop, s, store ? v_cap : 0, store ? 1 : 0,
                   hg ? 1 : 0};
    HIPCHK(launch_b_admit(d_slots, idx, v, init, s ? rs->mu : nullptr, c->stream));
    Host& h = S[idx];
    h = Host();
    h.used = true;
    h.running = true;
    h.group = gid;
    grp.users += 1;
    h.d = v;
    h.max_iter = o->max_iter;
    h.rr_every = grp.fp32 ? o->rr_every : 0;
    h.store_basis = store;
    h.v_cap = v_cap;
    h.rs = rs;
    h.valid_from = chunk_id;
    h.rr_js.assign(1, 0);   // the first test is on the FP64 residual of the set-up
    // set-up: r = g - H w0 (FP64), c0 = C^T r, w += U c0, r -= C c0
    const std::vector<int> one{idx};
    HIPCHK(launch_b_residual(base, rows, s > 0, d_slots, make_map(S, one, true), 0, c->stream));
    if (v.fold_res) {
        BatchMap f{};
        f.ns = 1;
        f.slot[0] = idx;
        HIPCHK(launch_b_fold(d_slots, f, 0, StepRef{d_ctr, 0}, c->stream));
    }
    HIPCHK(launch_b_init(d_slots, make_map(S, one, false), c->stream));
    dirty = true;
    return BL_OK;
}

// Residual replacement in FP64 for the listed slots: r = g - H w, z = C^T r, r -= C z, launched
// on stream ls at position k of the current chunk (k = 0 between chunks).
bl_status Batch::replace_residual(const std::vector<int>& idx, int periodic, int k, hipStream_t ls) {
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        std::vector<int> mine;
        for (int i : idx)
            if (S[i].group == gi) mine.push_back(i);
        if (!mine.empty())
            HIPCHK(launch_b_residual(groups[gi].base, groups[gi].rows, groups[gi].rec, d_slots, make_map(S, mine, true),
                                     periodic, ls));
    }
    BatchMap f{};
    for (int i : idx)
        if (S[i].d.fold_res) f.slot[f.ns++] = i;
    HIPCHK(launch_b_fold(d_slots, f, 0, StepRef{d_ctr, k}, ls));
    HIPCHK(launch_b_replace(d_slots, make_map(S, idx, false), periodic, StepRef{d_ctr, k}, ls));
    return BL_OK;
}

bl_status Batch::finish(int idx) {
    if (S[idx].d.s > 0) HIPCHK(launch_b_finish(d_slots, make_map(S, std::vector<int>{idx}, false), c->stream));
    return BL_OK;
}

// The launches of one chunk of nsteps iterations on stream ls: scheduled replacements, record
// folds, one launch per group (the fused step of an FP64 group, the apply of a mixed one) and
// one update launch over the mixed-precision slots per iteration, then the header gather
// (which advances the step counter) and its copy to pinned buffer buf.  With time_all (timing
// mode 2) HIP events bracket the group launches and the update of every iteration; without
// graphs, those of every KT_SAMPLE-th step.  No host-side state changes here, so the same
// sequence can be captured.
bl_status Batch::launch_chunk(int nsteps, int buf, const std::vector<std::vector<int>>& rr, hipStream_t ls,
                              bool time_all) {
    bool any_rec = false;
    for (const Group& grp : groups) any_rec |= grp.rec && !grp.fused() && grp.tmap.ns > 0;
    for (int k = 0; k < nsteps; ++k) {
        const StepRef sr{d_ctr, k};
        const bool ktime = c->timing == 2 && (time_all || (!c->graphs && (step + k) % KT_SAMPLE == 0));
        if (!rr[k].empty()) TRY(replace_residual(rr[k], 1, k, ls));
        if (fold_upd.ns) HIPCHK(launch_b_fold(d_slots, fold_upd, 2, sr, ls));
        if (fold_fused.ns) HIPCHK(launch_b_fold(d_slots, fold_fused, 3, sr, ls));
        int ev = 0;
        if (ktime) {
            ev = 3 * (int)timed.size();
            while ((int)c->kev.size() < ev + 3) {
                hipEvent_t e;
                HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
                c->kev.push_back(e);
            }
            HIPCHK(hipEventRecord(c->kev[ev], ls));
        }
        for (const Group& grp : groups) {
            if (!grp.tmap.ns) continue;
            if (grp.fused()) {
                // a group of one solve passes its descriptor by value (a fused slot's descriptor
                // does not change between admission and retirement, so a captured graph stays valid)
                const Slot* one = grp.tmap.ns == 1 ? &S[grp.tmap.slot[0]].d : nullptr;
                HIPCHK(launch_f_step(grp.base, grp.rows, grp.rec, d_slots, grp.tmap, sr, one, ls));
            }
            else HIPCHK(launch_b_apply(grp.base, grp.rows, grp.rec, grp.fp32, d_slots, grp.tmap, sr, ls));
        }
        if (ktime) HIPCHK(hipEventRecord(c->kev[ev + 1], ls));
        if (fold_app.ns) HIPCHK(launch_b_fold(d_slots, fold_app, 1, sr, ls));
        HIPCHK(launch_b_update(d_slots, pmap, sr, any_rec, ls));
        if (ktime) {
            HIPCHK(hipEventRecord(c->kev[ev + 2], ls));
            Timed t;
            t.ev = ev;
            for (int i : run_list) t.sj.push_back(make_int2(i, step + k - S[i].d.j0));
            timed.push_back(std::move(t));
        }
    }
    BatchMap all{};
    all.ns = (int)run_list.size();
    for (int k = 0; k < all.ns; ++k) all.slot[k] = run_list[k];
    // the header kernel writes the snapshot straight into pinned host memory (the poll event
    // after it orders those writes before the host's read): no copy launch per chunk
    HIPCHK(launch_b_headers(d_slots, all, reinterpret_cast<int*>(h_hdr + (size_t)buf * cap * HDR_BYTES), d_ctr,
                            nsteps, ls));
    return BL_OK;
}

// Capture a chunk on the context's private stream (nothing runs) into an executable graph.  On
// failure the stage and HIP error are left in the context's error string.
bl_status Batch::capture(int nsteps, int buf, const std::vector<std::vector<int>>& rr, hipGraphExec_t& ex) {
    ex = nullptr;
    auto fail = [&](const char* stage, hipError_t e) {
        c->err = std::string("graph capture (") + stage + "): " + hipGetErrorString(e);
        (void)hipGetLastError();
        return BL_E_HIP;
    };
    if (!c->cap_stream) {
        const hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            c->cap_stream = nullptr;
            return fail("stream", e);
        }
    }
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return fail("begin", e);
    const bl_status st = launch_chunk(nsteps, buf, rr, c->cap_stream, false);
    const std::string launch_err = st == BL_OK ? std::string() : c->err;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != BL_OK) {
        if (g) (void)hipGraphDestroy(g);
        c->err = "graph capture (launch): " + launch_err;
        (void)hipGetLastError();
        return BL_E_HIP;
    }
    if (e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail("end", e);
    }
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ex = nullptr;
        return fail("instantiate", e);
    }
    return BL_OK;
}

bl_status Batch::enqueue_chunk(int max_steps, int& steps_done, long& id, std::vector<int>& slots) {
    if (dirty) TRY(rebuild());
    slots = run_list;
    id = chunk_id++;
    const int buf = (int)(id & 1);
    // a lone solve takes long chunks (fewer polls and graph launches); in a batch a stopped slot
    // idles until the chunk ends and retires a chunk later, so its chunks are shorter
    const int nsteps = std::min(run_list.size() > 1 ? CHUNK_MANY : CHUNK, max_steps - steps_done);
    // scheduled replacements (mixed precision): before the test of every rr_every-th iteration
    std::vector<std::vector<int>> rr(nsteps);
    for (int k = 0; k < nsteps; ++k)
        for (int i : run_list) {
            Host& h = S[i];
            const int j = step + k - h.d.j0;
            if (h.rr_every > 0 && j > 0 && j <= h.max_iter && j % h.rr_every == 0) {
                rr[k].push_back(i);
                h.rr_js.push_back(j);
            }
        }
    // timing mode 2 with graphs: every KT_SAMPLE-th chunk runs directly, with events on each step
    const bool sampled = c->timing == 2 && c->graphs && id % KT_SAMPLE == 0;
    bool launched = false;
    if (c->graphs && !graphs_off && !sampled) {
        GraphKey key(gen, nsteps, buf, rr);
        auto it = graph_cache.find(key);
        if (it == graph_cache.end()) {
            if (seen.count(key)) {
                hipGraphExec_t ex = nullptr;
                if (capture(nsteps, buf, rr, ex) == BL_OK) {
                    it = graph_cache.emplace(key, ex).first;
                    ++c->graph_captures;
                } else {
                    graphs_off = true;
                }
            } else {
                seen.insert(key);
            }
        }
        if (it != graph_cache.end()) {
            HIPCHK(hipGraphLaunch(it->second, c->stream));
            ++c->graph_replays;
            launched = true;
        }
    }
    if (!launched) TRY(launch_chunk(nsteps, buf, rr, c->stream, sampled));
    step += nsteps;
    steps_done += nsteps;
    HIPCHK(hipEventRecord(poll_ev[buf], c->stream));
    return BL_OK;
}

// Read a chunk's header snapshot.  A stopped slot completes, except that in mixed precision a
// converged slot whose last test did not follow a residual replacement is re-tested: its
// residual is replaced in FP64 and it resumes at the iteration that stopped.
bl_status Batch::process_chunk(long id, const std::vector<int>& slots, std::vector<int>& done) {
    const int buf = (int)(id & 1);
    HIPCHK(hipEventSynchronize(poll_ev[buf]));
    const char* src = h_hdr + (size_t)buf * cap * HDR_BYTES;
    std::vector<int> retest;
    for (int i : slots) {
        Host& h = S[i];
        if (!h.running || id < h.valid_from) continue;
        std::memcpy(&h.hdr, src + (size_t)i * HDR_BYTES, HDR_BYTES);
        if (!h.hdr.done) continue;
        const int jd = h.hdr.iters;
        const bool replaced = std::find(h.rr_js.begin(), h.rr_js.end(), jd) != h.rr_js.end();
        if (groups[h.group].fp32 && h.hdr.status == BL_OK && !replaced) {
            retest.push_back(i);
        } else {
            TRY(finish(i));
            h.running = false;
            h.complete = true;
            dirty = true;
            done.push_back(i);
        }
    }
    if (!retest.empty()) {
        for (int i : retest) {
            Host& h = S[i];
            h.d.j0 = step - h.hdr.iters;
            HIPCHK(launch_b_set_j0(d_slots, i, h.d.j0, c->stream));
            h.rr_js.assign(1, h.hdr.iters);
            h.valid_from = chunk_id;
        }
        TRY(replace_residual(retest, 0, 0, c->stream));
    }
    return BL_OK;
}

// Kernel durations of the steps in which some slot ran a full iteration.
void Batch::account_times() {
    for (const Timed& t : timed) {
        bool real = false;
        for (const int2& p : t.sj) {
            const Host& h = S[p.x];
            const int bound = h.hdr.done ? h.hdr.iters + (h.hdr.status == BL_E_INDEFINITE ? 1 : 0) : h.hdr.iters + 1;
            if (p.y < bound) real = true;
        }
        if (!real) continue;
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, c->kev[t.ev], c->kev[t.ev + 1]) != hipSuccess) continue;
        if (hipEventElapsedTime(&b, c->kev[t.ev + 1], c->kev[t.ev + 2]) != hipSuccess) continue;
        c->kt[0] += a;
        c->kt[1] += 1.0;
        c->kt[2] += b;
        c->kt[3] += 1.0;
    }
    timed.clear();
}

bl_status Batch::run(int max_steps, bool until_any, std::vector<int>& done) {
    std::deque<std::pair<long, std::vector<int>>> inflight;
    int steps_done = 0;
    bool stop = false;
    auto can_enqueue = [&]() -> bool {
        if (stop || steps_done >= max_steps) return false;
        if (dirty) (void)rebuild();
        return !run_list.empty();
    };
    auto enqueue = [&]() -> bl_status {
        long id;
        std::vector<int> slots;
        TRY(enqueue_chunk(max_steps, steps_done, id, slots));
        inflight.emplace_back(id, std::move(slots));
        return BL_OK;
    };
    if (can_enqueue()) TRY(enqueue());
    while (!inflight.empty()) {
        if (can_enqueue()) TRY(enqueue());
        const auto ch = std::move(inflight.front());
        inflight.pop_front();
        TRY(process_chunk(ch.first, ch.second, done));
        if (until_any && !done.empty()) stop = true;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    for (hipGraphExec_t ex : retired) (void)hipGraphExecDestroy(ex);
    retired.clear();
    if (c->timing == 2) account_times();
    return BL_OK;
}

void Batch::stats(int idx, bl_stats* out) const {
    const Host& h = S[idx];
    std::memset(out, 0, sizeof(*out));
    out->iters = h.hdr.iters;
    out->status = h.hdr.done ? h.hdr.status : BL_E_NOT_CONVERGED;
    out->s_cur = h.d.s;
    out->res_norm = std::sqrt(std::max(h.hdr.rho2[h.hdr.iters & 1], 0.0));
    out->res0_norm = h.hdr.res0;
    out->g_norm = h.hdr.gnorm;
    out->est = h.hdr.est;
    if (h.rs && h.store_basis) {
        const int nv = h.hdr.iters + (out->status == BL_E_INDEFINITE && !h.d.fused ? 1 : 0);
        h.rs->v_cur = std::min(nv, h.v_cap);
        // the CG coefficients describe the stored residuals up to the first residual replacement
        // after the set-up (mixed precision): the relation of the later ones to them is broken
        int vl = h.rs->lz ? std::min(h.rs->v_cur, h.hdr.iters) : 0;
        for (int j : h.rr_js)
            if (j > 0 && j < vl) vl = j;
        h.rs->v_lz = vl;
    }
}

void Batch::release(int idx) {
    if (S[idx].group >= 0) groups[S[idx].group].users -= 1;
    S[idx] = Host();
    dirty = true;
}

}  // namespace blh

using namespace blh;

// ------------------------------------------------------------------------------------ engine
struct bl_engine {
    bl_ctx* c = nullptr;
    int cap = 0;
    Batch B;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::map<size_t, size_t> free_blocks;   // offset -> size
    std::vector<std::pair<size_t, size_t>> alloc;   // per slot (offset, size)
    SolveState* states = nullptr;
    double* h_taps = nullptr;   // pinned [cap][2 * TAPS_MAX]: taps staging (doubles, then floats)
    char* h_hdr = nullptr;      // pinned [2][cap][HDR_BYTES]
    hipEvent_t ev[2] = {};

    bool take(size_t bytes, size_t& off) {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_blocks.erase(it);
            if (rest) free_blocks[off + bytes] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free_blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_blocks.erase(nx);
        }
        if (it != free_blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_blocks.erase(it);
            }
        }
    }
};

namespace {

struct EngineLayout {
    size_t slots, ctr, states, arena, total;
};

EngineLayout engine_layout(int cap, size_t arena_bytes) {
    EngineLayout L{};
    size_t o = 0;
    L.slots = o;   o += al((size_t)cap * sizeof(Slot));
    L.ctr = o;     o += al(sizeof(int));
    L.states = o;  o += al((size_t)cap * sizeof(SolveState));
    L.arena = o;   o += al(arena_bytes);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

size_t bl_engine_slot_bytes(const bl_problem* P, int s) {
    if (!P || s < 0 || s > S_MAX) return 0;
    return slot_bytes(P, s);
}

size_t bl_engine_workspace_bytes(int cap, size_t arena_bytes) {
    if (cap < 1 || cap > B_MAX) return 0;
    return engine_layout(cap, arena_bytes).total;
}

bl_status bl_engine_create(bl_ctx* c, int cap, void* ws, size_t ws_bytes, bl_engine** out) {
    if (!c) return BL_E_ARG;
    if (!out) return c->err = "null engine handle", BL_E_ARG;
    *out = nullptr;
    if (cap < 1 || cap > B_MAX) return c->err = "engine capacity outside [1, 64]", BL_E_ARG;
    if (!ws || (uintptr_t)ws % ALIGN) return c->err = "workspace missing or not 256-byte aligned", BL_E_WORKSPACE;
    const EngineLayout L0 = engine_layout(cap, 0);
    if (ws_bytes < L0.total) return c->err = "workspace smaller than bl_engine_workspace_bytes(cap, 0)", BL_E_WORKSPACE;
    const size_t arena_bytes = (ws_bytes - L0.arena) / ALIGN * ALIGN;
    bl_engine* e = new bl_engine();
    e->c = c;
    e->cap = cap;
    char* base = (char*)ws;
    e->arena = base + L0.arena;
    e->arena_bytes = arena_bytes;
    if (arena_bytes) e->free_blocks[0] = arena_bytes;
    e->alloc.assign(cap, {0, 0});
    e->states = (SolveState*)(base + L0.states);
    if (hipHostMalloc((void**)&e->h_taps, (size_t)cap * 2 * TAPS_MAX * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&e->h_hdr, (size_t)2 * cap * HDR_BYTES, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev[1], hipEventDisableTiming) != hipSuccess) {
        c->err = "pinned host memory or event creation failed";
        if (e->h_taps) hipHostFree(e->h_taps);
        if (e->h_hdr) hipHostFree(e->h_hdr);
        for (auto& ev : e->ev)
            if (ev) hipEventDestroy(ev);
        delete e;
        return BL_E_HIP;
    }
    if (e->B.init(c, cap, (Slot*)(base + L0.slots), (int*)(base + L0.ctr), e->h_hdr, e->ev[0],
                  e->ev[1]) != BL_OK) {
        hipHostFree(e->h_taps);
        hipHostFree(e->h_hdr);
        for (auto& ev : e->ev) hipEventDestroy(ev);
        delete e;
        return BL_E_HIP;
    }
    *out = e;
    return BL_OK;
}

bl_status bl_engine_destroy(bl_engine* e) {
    if (!e) return BL_E_ARG;
    hipStreamSynchronize(e->c->stream);
    hipHostFree(e->h_taps);
    hipHostFree(e->h_hdr);
    for (auto& ev : e->ev) hipEventDestroy(ev);
    delete e;
    return BL_OK;
}

bl_status bl_engine_admit(bl_engine* e, const bl_problem* P, const double* theta, const double* xhat,
                          const double* g, double* w, bl_recycle* rs, const bl_solve_opts* opts, int* slot) {
    if (!e) return BL_E_ARG;
    bl_ctx* c = e->c;
    if (!slot) return c->err = "null slot output", BL_E_ARG;
    *slot = -1;
    TRY(check_problem(c, P));
    const int s = rs ? rs->s_cur : 0;
    if (s < 0 || s > S_MAX) return c->err = "s_cur outside [0, 64]", BL_E_SHAPE;
    int idx = -1;
    for (int i = 0; i < e->cap; ++i)
        if (!e->B.S[i].used) {
            idx = i;
            break;
        }
    if (idx < 0) return c->err = "engine full: no free slot", BL_E_WORKSPACE;
    const size_t bytes = slot_bytes(P, s);
    size_t off = 0;
    if (!e->take(bytes, off)) return c->err = "engine full: arena has no block of the slot's size", BL_E_WORKSPACE;
    SlotBuffers buf = carve_slot(e->arena + off, P, s);
    buf.st = e->states + idx;
    const SolveSpec sp{P, theta, xhat, g, w, rs, opts};
    const bl_status st = e->B.admit(idx, sp, buf, e->h_taps + (size_t)idx * 2 * TAPS_MAX);
    if (st != BL_OK) {
        e->give(off, bytes);
        return st;
    }
    e->alloc[idx] = {off, bytes};
    *slot = idx;
    return BL_OK;
}

bl_status bl_engine_step(bl_engine* e, int max_iters, int return_on_done, int* done, int* n_done) {
    if (!e) return BL_E_ARG;
    bl_ctx* c = e->c;
    if (max_iters < 1 || !n_done || !done) return c->err = "invalid step arguments", BL_E_ARG;
    std::vector<int> fin;
    TRY(e->B.run(max_iters, return_on_done != 0, fin));
    *n_done = (int)fin.size();
    for (size_t k = 0; k < fin.size(); ++k) done[k] = fin[k];
    return BL_OK;
}

bl_status bl_engine_retire(bl_engine* e, int slot, bl_stats* out) {
    if (!e) return BL_E_ARG;
    bl_ctx* c = e->c;
    if (slot < 0 || slot >= e->cap || !e->B.S[slot].complete) return c->err = "slot is not complete", BL_E_ARG;
    bl_stats tmp;
    e->B.stats(slot, &tmp);
    if (out) *out = tmp;
    e->give(e->alloc[slot].first, e->alloc[slot].second);
    e->alloc[slot] = {0, 0};
    e->B.release(slot);
    return (bl_status)tmp.status;
}

bl_status bl_engine_query(const bl_engine* e, int* running, int* free_slots, size_t* free_bytes,
                          size_t* largest_free) {
    if (!e) return BL_E_ARG;
    int used = 0;
    for (const auto& h : e->B.S) used += h.used ? 1 : 0;
    size_t fb = 0, lf = 0;
    for (const auto& kv : e->free_blocks) {
        fb += kv.second;
        lf = std::max(lf, kv.second);
    }
    if (running) *running = e->B.running();
    if (free_slots) *free_slots = e->cap - used;
    if (free_bytes) *free_bytes = fb;
    if (largest_free) *largest_free = lf;
    return BL_OK;
}

size_t bl_batched_workspace_bytes(int nprob, const bl_problem* P, const int* s) {
    if (nprob < 1 || !P) return 0;
    size_t arena = 0;
    for (int k = 0; k < nprob; ++k) {
        const int sk = s ? s[k] : 0;
        if (sk < 0 || sk > S_MAX) return 0;
        arena += slot_bytes(&P[k], sk);
    }
    return engine_layout(std::min(nprob, B_MAX), arena).total;
}

bl_status bl_hessian_solve_batched(bl_ctx* c, int nprob, const bl_problem* P, const double* const* theta,
                                   const double* const* xhat, const double* const* g, double* const* w,
                                   bl_recycle* rs, const bl_solve_opts* opts, void* ws, size_t ws_bytes,
                                   bl_stats* out) {
    if (!c) return BL_E_ARG;
    if (nprob < 1 || !P || !theta || !xhat || !g || !w || !out) return c->err = "null or empty batch", BL_E_ARG;
    for (int k = 0; k < nprob; ++k) TRY(check_problem(c, &P[k]));
    bl_engine* e = nullptr;
    TRY(bl_engine_create(c, std::min(nprob, B_MAX), ws, ws_bytes, &e));
    struct Guard {
        bl_engine* e;
        ~Guard() { bl_engine_destroy(e); }
    } guard{e};
    std::vector<int> slot_of(std::min(nprob, B_MAX), -1);
    bl_status first_bad = BL_OK;
    int next = 0, left = nprob;
    std::vector<int> done(e->cap);
    while (left > 0) {
        // admit in order while slots and arena space last
        while (next < nprob) {
            int sl;
            const bl_status st =
                bl_engine_admit(e, &P[next], theta[next], xhat[next], g[next], w[next], rs ? &rs[next] : nullptr, opts, &sl);
            if (st == BL_E_WORKSPACE) break;
            if (st != BL_OK) return st;
            slot_of[sl] = next++;
        }
        if (e->B.running() == 0) return c->err = "batched workspace too small for the next problem", BL_E_WORKSPACE;
        int nd = 0;
        TRY(bl_engine_step(e, INT_MAX, next < nprob ? 1 : 0, done.data(), &nd));
        for (int k = 0; k < nd; ++k) {
            const int sl = done[k], pk = slot_of[sl];
            const bl_status st = bl_engine_retire(e, sl, &out[pk]);
            if (st != BL_OK && first_bad == BL_OK) first_bad = st;
            --left;
        }
    }
    return first_bad;
}

}  // extern "C"
