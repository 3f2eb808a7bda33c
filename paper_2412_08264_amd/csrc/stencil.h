// Device cores of the matrix-free Hessian-vector products on LDS tiles.
//
// A block owns a TH x TW tile of the image.  The input vector is staged in LDS on the
// tile plus a halo E = max(2R, 2F, 1) (R blur radius, F filter half-size), and
//   H v = 2 A(A v) + lambda D^T(B D v)                             (smoothed TV)
//   H v = 2 A(A v) + eps v + sum_j lambda_j K_j^T(phi''_j . K_j v)   (filters)
// is evaluated on the tile:
//   * A(A v): separable blur applied twice (rows, columns, rows, columns); after the
//     first blur values outside the image are zeroed, because A pads with zeros;
//   * TV term: per-pixel 2x2 blocks B = (psi^2 I - u u^T)/psi^3 of u = (D xhat)_i with
//     psi = sqrt(|u|^2 + gamma^2), recomputed from xhat on the fly, a flux grid on the
//     tile plus one row/column, then D^T of the flux;
//   * filter term: K_j v on the tile plus F, times the precomputed phi''_j map, then
//     K_j^T back to the tile.
// T is the arithmetic type (double, or float in mixed precision); inputs and outputs
// in global memory are float64.
#pragma once

#include "common.h"

namespace bl {

struct TileLayout {
    int E, F, RW, RH;       // halo, filter half-size, region-0 width and height
    int o_v, o_h1, o_t1, o_x, o_fx, o_fy, o_t, o_out, o_taps, total;  // offsets (elements of T)
};

__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }

__host__ __device__ inline TileLayout tile_layout(int R, int reg, int fs) {
    TileLayout L;
    L.F = (reg == BL_REG_FILTERS) ? fs / 2 : 0;
    L.E = imax(imax(2 * R, 2 * L.F), 1);
    L.RW = TW + 2 * L.E;
    L.RH = TH + 2 * L.E;
    int o = 0;
    L.o_v = o;   o += L.RH * L.RW;
    L.o_h1 = o;  o += L.RH * (TW + 2 * R);
    L.o_t1 = o;  o += (TH + 2 * R) * (TW + 2 * R);
    L.o_x = o;   o += (TH + 2) * (TW + 2);
    L.o_fx = o;  o += (TH + 1) * (TW + 1);
    L.o_fy = o;  o += (TH + 1) * (TW + 1);
    L.o_t = o;   o += (TH + 2 * L.F) * (TW + 2 * L.F);
    L.o_out = o; o += TH * TW;
    L.o_taps = o; o += MAX_NF * MAX_FS * MAX_FS + MAX_NF;
    L.total = o;
    return L;
}

// Loop over a rows x cols region with a 2-D thread layout (32 columns x NT/32 rows): no
// integer division per element and unit-stride LDS access along rows.
#define TILE_LOOP(rows, cols, rr, cc)                                 \
    for (int rr = (int)(threadIdx.x >> 5); rr < (rows); rr += NT / 32) \
        for (int cc = (int)(threadIdx.x & 31); cc < (cols); cc += 32)

template <typename T>
__host__ inline size_t tile_lds_bytes(int R, int reg, int fs) {
    return (size_t)tile_layout(R, reg, fs).total * sizeof(T);
}

// Stage `fetch(global index)` on [r0-E, r0+TH+E) x [c0-E, c0+TW+E); zero outside the image.
// The loads of all of a thread's elements are issued before any is stored, so the staging
// costs one memory round trip (a block per CU has no other waves to hide latency with).
constexpr int STAGE_MAX = ((TH + 4 * MAX_R) * (TW + 4 * MAX_R) + NT - 1) / NT;
template <typename T, typename Fetch>
__device__ __forceinline__ void stage_region(T* buf, const Stencil& S, const TileLayout& L, int r0, int c0,
                                             Fetch fetch) {
    const int rows = L.RH, cols = L.RW, tot = rows * cols;
    double v[STAGE_MAX];
#pragma unroll
    for (int u = 0; u < STAGE_MAX; ++u) {
        const int idx = threadIdx.x + u * NT;
        v[u] = 0.0;
        if (idx < tot) {
            const int rr = idx / cols, cc = idx - rr * cols;
            const int gi = r0 - L.E + rr, gj = c0 - L.E + cc;
            if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) v[u] = fetch(gi * S.w + gj);
        }
    }
#pragma unroll
    for (int u = 0; u < STAGE_MAX; ++u) {
        const int idx = threadIdx.x + u * NT;
        if (idx < tot) buf[idx] = (T)v[u];
    }
}

// Stage xhat on [r0-1, r0+TH+1) x [c0-1, c0+TW+1) (TV flux) with one batch of loads.
constexpr int XSTAGE_MAX = ((TH + 2) * (TW + 2) + NT - 1) / NT;
template <typename T>
__device__ __forceinline__ void stage_xhat(T* xs, const Stencil& S, const double* __restrict__ xhat, int r0, int c0) {
    const int XW = TW + 2, tot = (TH + 2) * XW;
    double v[XSTAGE_MAX];
#pragma unroll
    for (int u = 0; u < XSTAGE_MAX; ++u) {
        const int idx = threadIdx.x + u * NT;
        v[u] = 0.0;
        if (idx < tot) {
            const int rr = idx / XW, cc = idx - rr * XW;
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) v[u] = xhat[gi * S.w + gj];
        }
    }
#pragma unroll
    for (int u = 0; u < XSTAGE_MAX; ++u) {
        const int idx = threadIdx.x + u * NT;
        if (idx < tot) xs[idx] = (T)v[u];
    }
}

}  // namespace bl
