// Host-side definitions shared by the C-ABI translation units: the context, argument
// checks, and the batch of recycled-CG solves that every Hessian solve runs through.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"

struct bl_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    int timing = 0;
    int graphs = 1;                      // replay repeated chunks of iterations from captured graphs
    hipStream_t cap_stream = nullptr;    // private stream graphs are captured on (created on first use)
    long graph_captures = 0, graph_replays = 0;
    int force_rows = 0;                  // autotuner: tile height of the solves it times (0: table)
    bl::SolveState* h_state = nullptr;   // pinned
    double* h_buf = nullptr;             // pinned staging (8192 doubles)
    int* h_info = nullptr;               // pinned
    char* h_hdr = nullptr;               // pinned: two header snapshots of a one-slot batch
    hipEvent_t poll_ev[2] = {};
    hipEvent_t ev[6] = {};
    std::vector<hipEvent_t> kev;         // per-launch events (timing mode 2)
    double kt[4] = {0.0, 0.0, 0.0, 0.0};
};

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
            return BL_E_HIP;                                                                 \
        }                                                                                    \
    } while (0)

#define TRY(expr)                        \
    do {                                 \
        bl_status s_ = (expr);           \
        if (s_ != BL_OK) return s_;      \
    } while (0)

namespace blh {

constexpr int POLL = 8;              // iterations launched between host polls of the stop flags
constexpr int CHUNK = 16;            // batch engine: iterations per chunk of a lone solve (one graph, one poll)
constexpr int CHUNK_MANY = 8;        // ... and of a batch, whose slots stop at different steps
constexpr int KT_SAMPLE = 8;         // timing mode 2: kernel events on every KT_SAMPLE-th step
// Consumer kernels re-reduce the producer's per-block records in every block; above this many
// record values a fold kernel (FOLD_BLOCKS blocks per solve) first reduces them to FOLD_BLOCKS
// records, so the consumers' re-reads stay bounded whatever the image size.
constexpr long REC_LIMIT = 8192;
// The fused FP64 step reduces the previous launch's records in every block, G threads per
// value (G the largest power of two with 2 G nv <= 256) with U loads in flight each (32 on
// recycled 8-row tiles, else 8): records are folded first (one more launch) only when that
// reduction would take more than two dependent rounds of loads.
inline bool fused_fold(int ntiles, int rows, int s, int nz) {
    const int nv = 4 + s + nz;
    int G = 1;
    while (G * 2 * nv <= 256) G *= 2;
    const int U = (s > 0 && rows == 8) ? 32 : 8;
    return ntiles > 2 * U * G;
}
constexpr size_t ALIGN = 256;
constexpr int TAPS_MAX = bl::MAX_NF * bl::MAX_FS * bl::MAX_FS + bl::MAX_NF;
// Device and pinned staging layout of a problem's taps: TAPS_MAX doubles, then TAPS_MAX floats.
constexpr size_t TAPS_BYTES = (size_t)TAPS_MAX * (sizeof(double) + sizeof(float));

inline size_t al(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

int nparams(const bl_problem* P);
bl_status check_problem(bl_ctx* c, const bl_problem* P);
bl_status check_solve_opts(bl_ctx* c, const bl_solve_opts* o);
// Operator-class part of the stencil (blur taps, regulariser, filter shape, penalty).
void class_stencil(const bl_problem* P, bl::Stencil& S);
// theta-dependent scalars: TV weight and smoothing; filters: taps then weights e^{w_j}
// into taps_host (nf*f*f + nf doubles, followed at TAPS_MAX doubles by their FP32 copies).
bl_status theta_values(bl_ctx* c, const bl_problem* P, const double* theta, double& lam, double& gam2,
                       double* taps_host);
// Problems that can share a batched launch: everything but the image size.
bool same_class(const bl_problem* a, const bl_problem* b);
// Tile height (rows) of the recycled-CG Hessian-vector kernels for P: the table entry of P's
// class and size class, else the block-count default.
bool valid_rows(int rows);
int default_rows(const bl_problem* P);
int tile_rows(const bl_problem* P);
void set_tile_rows(const bl_problem* P, int rows);
// Tile cache file (persisted autotuner results): the stored height of P's class and size class
// (found = false without an entry or file), and an entry stored or replaced.  False with err set
// when the file is malformed or cannot be written.
bool tile_cache_lookup(const char* path, const bl_problem* P, int& rows, bool& found, std::string& err);
bool tile_cache_store(const char* path, const bl_problem* P, int rows, const double us[3], std::string& err);
// Every entry of a cache file into the table (false with err: missing or malformed file, and
// then nothing is loaded).
bool tile_cache_load_all(const char* path, int& entries, std::string& err);

// Device scratch of one solve.
struct SlotBuffers {
    double *r, *p0, *p1, *q;
    double *r2, *q2, *HC;     // fused FP64 steps: second r and q buffers, H C (n x s)
    double *M, *mpart;        // C^T H C (s x s) and the partial sums that form it
    double *d1, *d2;
    float* d2f;
    double* taps;
    double *rec_res, *rec_app, *rec_upd, *rec_app2, *fold;
    bl::SolveState* st;
};
// Bytes of SlotBuffers (without st) for an h x w problem of this class with s recycle columns,
// and the carving of a region of that size.
size_t slot_bytes(const bl_problem* P, int s);
SlotBuffers carve_slot(char* base, const bl_problem* P, int s);

struct SolveSpec {
    const bl_problem* P;
    const double* theta;
    const double* xhat;
    const double* g;
    double* w;
    bl_recycle* rs;
    const bl_solve_opts* o;
};

// Recycled CG over up to `cap` concurrent solves in up to MAX_GROUPS groups (operator class,
// tile height, with or without a recycle space).  Each iteration is one launch per group with
// running solves (FP64: the fused step) and, for the mixed-precision groups, one update launch
// over their solves; the host enqueues chunks of CHUNK (one solve) or CHUNK_MANY iterations and reads the solves' stop
// flags one chunk behind, so the device never waits for the host.  A solve's arithmetic and
// decisions do not depend on the others.
constexpr int MAX_GROUPS = 16;

class Batch {
public:
    bl_ctx* c = nullptr;
    int cap = 0;
    bl::Slot* d_slots = nullptr;   // device [cap]
    int* d_ctr = nullptr;          // device step counter (equals `step` at chunk boundaries)
    char* h_hdr = nullptr;         // pinned [2][cap * HDR_BYTES], written by the header kernel
    hipEvent_t poll_ev[2] = {};

    struct Group {                 // operator class, tile height, recycling: stencil template, precision
                                   // (FP64 groups run the fused one-launch step, FP32-stencil ones the
                                   // apply + update pair with residual replacement)
        bl_problem cls{};
        bl::Stencil base{};
        bool fp32 = false;
        int rows = 0;
        bool rec = false;          // solves with a recycle space (projection code) or plain CG
        bool fused() const { return !fp32; }
        int users = 0;             // slots in use
        bl::BatchMap tmap{};       // tile map of its running slots
    };
    std::vector<Group> groups;

    struct Host {
        bool used = false, running = false, complete = false;
        int group = -1;
        bl::Slot d{};
        int max_iter = 0, rr_every = 0;
        bool store_basis = false;
        int v_cap = 0;
        bl_recycle* rs = nullptr;
        long valid_from = 0;       // first chunk whose header snapshot reflects the current run
        std::vector<int> rr_js;    // iterations whose test follows a residual replacement
        bl::SolveState hdr{};      // last valid header snapshot
    };
    std::vector<Host> S;
    int step = 0;                  // next global step index
    long chunk_id = 0;

    Batch() = default;
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;
    ~Batch();
    bl_status init(bl_ctx* ctx, int capacity, bl::Slot* slots, int* ctr_dev, char* hdr_pinned,
                   hipEvent_t ev0, hipEvent_t ev1);
    // Validate and start solve `sp` in free slot idx with device scratch B; taps_stage is
    // pinned host memory of TAPS_MAX doubles that stays untouched until the slot retires.
    bl_status admit(int idx, const SolveSpec& sp, const SlotBuffers& B, double* taps_stage);
    // Advance running slots by at most max_steps iterations, returning early once a slot
    // completes (until_any) or none is running.  Completed slots are appended to `done`;
    // their iterate is final when this returns.
    bl_status run(int max_steps, bool until_any, std::vector<int>& done);
    int running() const;
    void stats(int idx, bl_stats* out) const;
    void release(int idx);

private:
    bool dirty = true;
    bl::BatchMap pmap{}, fold_app{}, fold_upd{}, fold_fused{};   // pmap / fold_*: two-launch slots only
    std::vector<int> run_list;
    struct Timed {
        int ev;                    // first of 3 events
        std::vector<int2> sj;      // (slot, iteration) pairs of the step
    };
    std::vector<Timed> timed;
    // Captured chunks, keyed by the slot-set generation, the chunk length, the header buffer and
    // the scheduled replacements of each position; a chunk is captured the second time its key
    // occurs and replayed after that.  Graphs of an outdated generation are destroyed once the
    // stream has drained.
    using GraphKey = std::tuple<long, int, int, std::vector<std::vector<int>>>;
    std::map<GraphKey, hipGraphExec_t> graph_cache;
    std::set<GraphKey> seen;
    std::vector<hipGraphExec_t> retired;
    long gen = 0;
    bool graphs_off = false;       // a capture failed: launch directly from then on
    bl_status rebuild();
    bl_status replace_residual(const std::vector<int>& idx, int periodic, int k, hipStream_t ls);
    bl_status finish(int idx);
    bl_status launch_chunk(int nsteps, int buf, const std::vector<std::vector<int>>& rr, hipStream_t ls,
                           bool time_all);
    bl_status capture(int nsteps, int buf, const std::vector<std::vector<int>>& rr, hipGraphExec_t& ex);
    void drop_graphs();
    bl_status enqueue_chunk(int max_steps, int& steps_done, long& id, std::vector<int>& slots);
    bl_status process_chunk(long id, const std::vector<int>& slots, std::vector<int>& done);
    void account_times();
};

}  // namespace blh
