// Internal definitions shared by the HIP translation units of libbilevel_hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bilevel.h"

namespace bl {

constexpr int TW = 32;          // stencil tile width  (pixels)
constexpr int TH = 16;          // stencil tile height (pixels)
constexpr int NT = 256;         // threads per stencil / reduction block (4 wavefronts)
constexpr int NWAVE = NT / 64;
constexpr int S_MAX = 64;       // largest recycle dimension
constexpr int MAX_R = 8;        // largest blur radius
constexpr int MAX_NF = 8;       // largest number of filters
constexpr int MAX_FS = 7;       // largest filter size
constexpr int RED_BLOCKS = 512; // blocks of 1-D reduction kernels
constexpr int NV_RED = 2 + 2 * S_MAX;   // widest per-block partial record

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
    const double* taps;         // device: nf * fs * fs filter taps (row-major per filter)
    const double* lamj;         // device: nf weights e^{w_j}
    const double* d2;           // device: nf maps phi''(K_j xhat), FP64
    const float* d2f;           // device: nf maps phi''(K_j xhat), FP32 (mixed precision)
    int tiles_x, tiles_y;
};

// Scalars of one Krylov solve, resident in device memory.
struct SolveState {
    double rho, sigma, alpha, beta, gnorm, tol, hg_tol, res0, est, rho_true;
    int iters, done, status, max_iter, check_every, stop, s, v_cap, v_cur, store_basis, hgerr_on, pad;
    double e[S_MAX];      // C^T q of the current iteration
    double zr[S_MAX];     // Z^T r
    double zacc[S_MAX];   // coefficient of U accumulated over the iterations
    double mu[S_MAX];     // selected generalized singular values
    double c0[S_MAX];     // C^T r0 / scratch
};

// ------------------------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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

// After every block has written its partial record, exactly one block (the last to
// arrive) returns true; its threads then see all records.  Release/acquire at device
// scope makes the records visible across XCDs.  The counter is reset for reuse.
__device__ __forceinline__ bool last_block(unsigned* counter, unsigned nblocks) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == nblocks - 1) ? 1 : 0;
        if (s_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

// In the last block: out[k] = sum over blocks b (fixed order) of part[b*nv + k], k < nv.
// Deterministic: thread t sums blocks t, t+NT, ... in order, then a fixed tree.
__device__ __forceinline__ void reduce_partials(const double* part, int nblocks, int nv, double* out, double* red) {
    for (int k = 0; k < nv; ++k) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += NT) acc += __builtin_nontemporal_load(&part[(size_t)b * nv + k]);
        double s = block_sum(acc, red);
        if (threadIdx.x == 0) out[k] = s;
    }
    __syncthreads();
}

// Map a block index to a tile index so that each XCD (blocks are dealt round-robin over
// 8 XCDs) works on a contiguous band of tiles and neighbouring halos share one L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    if (nblocks % 8 != 0) return bid;
    return (bid & 7) * (nblocks >> 3) + (bid >> 3);
}

}  // namespace bl
