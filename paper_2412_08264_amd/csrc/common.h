// Internal definitions shared by the HIP translation units of libbilevel_hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bilevel.h"

namespace bl {

constexpr int TW = 32;          // stencil tile width  (pixels)
constexpr int TH = 8;           // stencil tile height (pixels): one pixel per thread
constexpr int NT = 256;         // threads per stencil / reduction block (4 wavefronts)
constexpr int NWAVE = NT / 64;
constexpr int S_MAX = 64;       // largest recycle dimension
constexpr int MAX_R = 8;        // largest blur radius
constexpr int MAX_NF = 8;       // largest number of filters
constexpr int MAX_FS = 7;       // largest filter size
constexpr int RED_BLOCKS = 512; // blocks of 1-D reduction kernels
constexpr int NV_RED = 4 + 2 * S_MAX;   // widest per-block partial record
constexpr int FOLD_BLOCKS = 128;        // blocks (and folded records) per slot of a record fold

// Stencil description passed by value to kernels.
struct Stencil {
    int h, w, n;
    int R;                      // blur radius
    double g[2 * MAX_R + 1];    // 1-D normalised Gaussian; the 2-D kernel is g g^T
    int reg;                    // BL_REG_TV / BL_REG_FILTERS
    double lam;                 // TV: e^{theta0}
    double gam2;                // TV: e^{2 theta1}
    int nf, fs;                 // filters
    double eps;
    int penalty;
    const double* taps;         // device: nf * fs * fs filter taps (row-major per filter), then nf weights
    const float* tapsf;         // device: the same nf * fs * fs + nf values in FP32
    const double* lamj;         // device: nf weights e^{w_j} (= taps + nf * fs * fs)
    const double* d2;           // device: nf maps phi''(K_j xhat), FP64
    const float* d2f;           // device: nf maps phi''(K_j xhat), FP32 (mixed precision)
    int tiles_x, tiles_y;
};

// Scalars of one Krylov solve, resident in device memory.  Every block of a kernel
// recomputes the scalars it needs from the previous kernel's partial records (same
// data, same order: identical values in every block); block 0 stores them here.
// Values rewritten during a kernel that other blocks of the same kernel read are
// double-buffered by iteration parity (rho2).
struct SolveState {
    double rho2[2];     // rho_j = r_j . r_j, slot j & 1
    double alpha, gnorm, tol, hg_tol, res0, est, pad0[3];
    int iters, done, status, max_iter, check_every, stop, s, v_cap, v_cur, store_basis, hgerr_on;
    int rr_j;             // iteration whose test follows the last residual replacement (-1: none)
    int stop_at;          // 1 + the step index of the launch that stopped the solve (0: running)
    double e[S_MAX];      // C^T q of the current iteration
    double zr[S_MAX];     // Z^T r
    double zacc[S_MAX];   // coefficient of U accumulated over the iterations
    double mu[S_MAX];     // selected generalized singular values
    double c0[S_MAX];     // C^T r0 / scratch
};

// One independent Krylov solve inside a batched launch (device memory).  Blocks of a
// tile-grid launch map to (slot, local tile) and blocks of a pixel-grid launch to (slot,
// local block) through per-launch maps; each slot reduces only its own records, in the
// same order as when it runs alone, so its results do not depend on the batch.
struct Slot {
    int h, width, n, tiles_x, ntiles, npix;   // image, tiles, pixel blocks (ceil(n / NT))
    int j0;                               // global step index at which the slot started
    int s, nz;                            // recycle columns; error-estimate columns (0: off)
    int fold_app, fold_upd, fold_res;     // records folded by k_fold before use
    int rows;                             // tile height of the Hessian-vector launches
    double lam, gam2;                     // TV weight e^{theta0}, smoothing e^{2 theta1}
    const double* taps;                   // filters: taps (then weights), FP32 copy, weights, phi'' maps
    const float* tapsf;
    const double* lamj;
    const double* d2;
    const float* d2f;
    const double* xhat;
    const double* g;
    double* w;
    double* r;
    double* p[2];
    double* q;
    double* r2;                           // fused FP64 steps: r_j, q_j alternate between r / r2, q / q2
    double* q2;
    const double* HC;                     // fused FP64 steps with a recycle space: H C (n x s)
    const double* M;                      // and C^T H C (s x s, column-major)
    int fused;                            // one launch per iteration (FP64 solves)
    const double* U;
    const double* C;
    const double* Z;
    double* V;
    double* lz;                           // CG coefficients of the stored residuals: alpha_j at 2j, rho_j at 2j+1
    SolveState* st;
    double* rec_res;                      // records: residual (tiles), apply (tiles), update (pixel blocks)
    double* rec_app;
    double* rec_upd;
    double* rec_app2;                     // fused steps: records of odd iterations (a launch reads the
                                          // records of the previous one while writing its own)
    double* fold;                         // folded records: 3 kinds x FOLD_BLOCKS records of NV_RED values
};

// Block-to-slot map of one batched launch, passed by value: slot k of the launch is
// slots[slot[k]] and owns blocks off[k] .. off[k+1]-1.  In tile-grid launches every off[k]
// is a multiple of 8, so a slot's local tile index modulo 8 is the XCD its block runs on.
constexpr int B_MAX = 64;       // slots per batched launch
struct BatchMap {
    int ns;
    int slot[B_MAX];
    int off[B_MAX + 1];
};

// Slot and local block of block b (binary search over the offsets; uniform per block).
__device__ __forceinline__ int2 map_block(const BatchMap& M, int b) {
    int lo = 0, hi = M.ns;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b >= M.off[mid]) lo = mid;
        else hi = mid;
    }
    return make_int2(M.slot[lo], b - M.off[lo]);
}

// Global step index of a launch: a device counter, advanced by the header kernel at the end of
// each chunk of iterations, plus the launch's position in its chunk.  A chunk's launches then
// take the same arguments every time, so a captured chunk can be replayed as a graph.
struct StepRef {
    const int* ctr;
    int k;
};
__device__ __forceinline__ int step_of(const StepRef& sr) { return sr.ctr[0] + sr.k; }

// Per-solve settings written into a fresh SolveState at admission.
struct StateInit {
    double tol, hg_tol;
    int max_iter, check_every, stop, s, v_cap, store_basis, hgerr_on;
};

constexpr int HDR_BYTES = (int)offsetof(SolveState, e);   // scalar header polled by the host

// ------------------------------------------------------------------------------------ reductions

// A double moved across lanes by a DPP control (two 32-bit moves; every lane of a row takes
// part, so the row and bank masks are full).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of G consecutive lanes (G a power of two, 1..64); every lane of a
// group ends with the same value.  Lanes pair within quads (DPP quad permutations), then
// mirror within half rows and rows of 16 (each partner already holds the other half's sum),
// then across rows with LDS permutes.  Additions are commutative, so partners compute
// identical sums; the pattern is fixed, so the result is deterministic.
__device__ __forceinline__ double group_sum(double v, int G) {
    if (G >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    if (G >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    if (G >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
    if (G >= 16) v += dpp_f64<0x140>(v);  // row_mirror
    if (G >= 32) v += __shfl_xor(v, 16, 64);
    if (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum(v, 64); }

// DPP move whose lanes outside the rows of ROWS keep zero.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64_rows(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums over aligned groups of 32 or 64 lanes without LDS permutes: the row sums of group_sum,
// then DPP row broadcasts (row_bcast:15 adds row 0 into row 1 and row 2 into row 3; for 64,
// row_bcast:31 then adds rows 0-1 into rows 2-3), so the last lane of each group holds its sum
// (lanes 31 and 63; the other lanes hold partial sums).  A fixed pattern: deterministic.
__device__ __forceinline__ double group_sum_last(double v, int G) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    v += dpp_f64_rows<0x142, 0xA>(v);                // row_bcast:15 into rows 1 and 3
    if (G >= 64) v += dpp_f64_rows<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// The wave's sum as a uniform value (lane 63 of group_sum_last, read into scalar registers).
__device__ __forceinline__ double wave_total(double v) {
    v = group_sum_last(v, 64);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum `val` over the block; result valid in every thread.  `red` has NWAVE doubles.
__device__ __forceinline__ double block_sum(double val, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    val = wave_sum(val);
    __syncthreads();
    if (lane == 0) red[wave] = val;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NWAVE; ++k) s += red[k];
    return s;
}

// Global-memory views of generic pointers: accesses through them compile to global (not flat)
// memory instructions, which do not count against the LDS wait counter (a flat load in flight
// would hold up every later LDS wait) and take a uniform base address in scalar registers.
template <typename T>
using gbl_t = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gbl_t<T> gbl(T* p) {
    return (gbl_t<T>)p;
}

// Block partial record of nv values (nv <= NV_RED): value k of this thread is val(k).
// Each wavefront reduces with shuffles, one barrier, then threads k < nv add the NWAVE
// wave sums in fixed order and write part[blockIdx.x * nv + k].
// block_partials_in takes the NWAVE x NV_RED doubles of LDS for the wave sums from the caller
// (a tile kernel passes its tile region, free once the product is in registers).
template <typename Val>
__device__ __forceinline__ void block_partials_in(double* wred, double* part, int nv, Val val, int rec_index = -1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k0 = 0; k0 < nv; k0 += 8) {
        // the values of a group of 8 (typically loads of 8 columns) are all in flight
        // before the first shuffle reduction waits on them
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (k0 + u < nv) ? val(k0 + u) : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (k0 + u >= nv) break;   // uniform: no reduction of the padding values
            const double sum = wave_total(v[u]);
            if (lane == 0) wred[wave * NV_RED + k0 + u] = sum;
        }
    }
    __syncthreads();
    const size_t rec = rec_index < 0 ? (size_t)blockIdx.x : (size_t)rec_index;
    for (int k = threadIdx.x; k < nv; k += NT) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NWAVE; ++w) s += wred[w * NV_RED + k];
        gbl(part)[rec * nv + k] = s;
    }
}
template <typename Val>
__device__ __forceinline__ void block_partials(double* part, int nv, Val val, int rec_index = -1) {
    __shared__ double wred[NWAVE * NV_RED];
    block_partials_in(wred, part, nv, val, rec_index);
}

// out[k] = sum over blocks of part[b*nv + k], k < nv (nv <= NT), into LDS `out` (all threads).
// G threads share value k (G the largest power of two with G * nv <= NT): thread (k, j) sums
// blocks j, j+G, ..., all of its first U loads issued before the first addition (one memory
// round trip for up to U * G records: the records come from other compute units' caches, so
// each dependent round costs a full miss; U = 32 covers the 256 tiles of a 256 x 256 image
// with a 20-column recycle record, at the price of 64 registers), then the G partial sums are
// combined by a group sum (within a wave; across the waves of a group in wave order).  The
// order depends only on (U, nblocks, nv), so every block that reduces the same records with
// the same U obtains bit-identical values.
template <int U = 8>
__device__ __forceinline__ void reduce_partials(const double* part, int nblocks, int nv, double* out) {
    __shared__ double wsum[NWAVE];
    int G = 1;
    while (G * 2 * nv <= NT) G *= 2;
    const int k = threadIdx.x / G, j = threadIdx.x & (G - 1);
    const gbl_t<const double> gp = gbl(part);
    double acc = 0.0;
    if (k < nv) {
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = j + u * G;
            a[u] = b < nblocks ? gp[(size_t)b * nv + k] : 0.0;
        }
        // beyond U * G records (unfolded large record arrays): further rounds of 8 loads
        for (int b = j + U * G; b < nblocks; b += 8 * G) {
            double c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = b + u * G < nblocks ? gp[(size_t)(b + u * G) * nv + k] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += c[u];
        }
#pragma unroll
        for (int w2 = U / 2; w2 > 0; w2 >>= 1)
#pragma unroll
            for (int u = 0; u < w2; ++u) a[u] += a[u + w2];
        acc = a[0];
    }
    // groups of 32 or more lanes: the sum in the group's last lane (no LDS permutes)
    const int Gw = G < 64 ? G : 64;
    acc = Gw >= 32 ? group_sum_last(acc, Gw) : group_sum(acc, Gw);
    if (G <= 64) {
        if (j == (Gw >= 32 ? G - 1 : 0) && k < nv) out[k] = acc;
    } else {
        if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = acc;
        __syncthreads();
        if ((int)threadIdx.x < nv) {
            const int wpg = G / 64;
            double s = 0.0;
            for (int q = 0; q < wpg; ++q) s += wsum[threadIdx.x * wpg + q];
            out[threadIdx.x] = s;
        }
    }
    __syncthreads();
}

// Width of the residual record that the test of iteration j reads: r.r, and Z^T r (nz values)
// only when that test evaluates the error estimate (every check_every-th iteration), so the
// columns of Z are read on tested iterations only.
// Loads of the solve state go through global-address-space pointers: before a kernel's first
// store they are uniform and unclobbered, so they become scalar loads that no vector load waits
// behind (a flat load waits for every vector load issued before it).
__device__ __forceinline__ int zr_width(int check_every, int nz, int j) {
    return (nz > 0 && j % check_every == 0) ? nz : 0;
}
__device__ __forceinline__ int zr_width(const SolveState* st, int nz, int j) {
    return zr_width(gbl(st)->check_every, nz, j);
}

// Stop decision after j completed iterations from the reduced residual record (r.r and,
// when the record holds it, Z^T r).  Order of tests: non-finite; exact zero residual; only
// every check_every iterations: the hypergradient-error estimate ||mu . Z^T r|| <= hg_tol
// (when enabled) or ||r|| <= tol ||g||; then the iteration limit.
struct Decision {
    bool done;
    int status;
    double est;
};

// A value every lane of the wave holds (loaded from one address), moved to a scalar register,
// so that keeping it across a long stretch of code costs no vector registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A solve stopped by an earlier launch: its blocks have nothing to do and leave before their
// record reduction.  stop_at is written once, by block 0 of the stopping launch (step S writes
// S + 1), so the blocks of that launch read 0 or S + 1 and carry on to the decision they share,
// and every later launch reads the same value in every wave: the test is uniform per block
// without a barrier.  The mark is loaded first and tested later (stop_mark, then
// stopped_before), so that no wave waits for it before issuing its other loads.
__device__ __forceinline__ int stop_mark(const SolveState* st) { return *gbl(&st->stop_at); }
__device__ __forceinline__ bool stopped_before(int mark, int step) {
    const int a = uni(mark);
    return a != 0 && a <= step;
}

// The settings the test reads, loaded once: a kernel can issue these loads before its record
// reduction, so the decision does not wait on them afterwards.
struct TestSettings {
    double tol, hg_tol, gnorm;
    int check_every, stop, hgerr_on, s, max_iter;
};
__device__ __forceinline__ TestSettings test_settings(const SolveState* st) {
    const gbl_t<const SolveState> g = gbl(st);
    return TestSettings{uni(g->tol),  uni(g->hg_tol),   uni(g->gnorm), uni(g->check_every),
                        uni(g->stop), uni(g->hgerr_on), uni(g->s),     uni(g->max_iter)};
}

// Lane k of the wave holds mu[k] (k < s <= 64, s the solve state's count): one load per lane, issued with the kernel's
// other early loads, instead of s dependent loads inside the test.
__device__ __forceinline__ double mu_of_lane(const SolveState* st, int s) {
    const int k = (int)(threadIdx.x & 63);
    return k < s ? gbl(st->mu)[k] : 0.0;
}

__device__ __forceinline__ double lane_value(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ Decision decide(const TestSettings& ts, int j, double rho, const double* zr, bool have_zr,
                                           double mu_lane) {
    Decision d{false, BL_OK, NAN};
    if (ts.hgerr_on && have_zr) {
        double acc = 0.0;
        for (int k = 0; k < ts.s; ++k) {
            const double t = lane_value(mu_lane, k) * zr[k];
            acc += t * t;
        }
        d.est = sqrt(acc);
    }
    if (!(rho == rho) || fabs(rho) == INFINITY) {
        d.done = true;
        d.status = BL_E_NONFINITE;
        return d;
    }
    bool met;
    if (rho == 0.0) met = true;
    else if (j % ts.check_every) met = false;
    else if (ts.stop == BL_STOP_HGERR && ts.hgerr_on) met = d.est <= ts.hg_tol;
    else met = sqrt(rho) <= ts.tol * ts.gnorm;
    if (met) {
        d.done = true;
    } else if (j >= ts.max_iter) {
        d.done = true;
        d.status = BL_E_NOT_CONVERGED;
    }
    return d;
}

// sum_k M[k*n + i] * c[k], k < s, with the loads of 8 columns issued together.
__device__ __forceinline__ double combo(const double* __restrict__ M, size_t n, int i, const double* c, int s) {
    double acc = 0.0;
    for (int k0 = 0; k0 < s; k0 += 8) {
        double m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = (k0 + u < s) ? M[(size_t)(k0 + u) * n + i] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + u < s) acc += m[u] * c[k0 + u];
    }
    return acc;
}

// Map a block index to a tile index so that each XCD (blocks are dealt round-robin over
// 8 XCDs) works on a contiguous band of tiles and neighbouring halos share one L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    if (nblocks % 8 != 0) return bid;
    return (bid & 7) * (nblocks >> 3) + (bid >> 3);
}

}  // namespace bl
