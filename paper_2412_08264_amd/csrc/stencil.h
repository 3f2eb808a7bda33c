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

// Evaluate H v on the owned TH x TW tile from the staged region; result in lds[o_out].
// xs_staged: the TV kernels staged xhat already (stage_xhat before the barrier).
// RB is the blur radius as a compile-time constant (the tap loops unroll fully and their LDS
// loads issue together); LDS views are __restrict__ so passes pipeline across outputs.
template <typename T, int RB>
__device__ void hvp_tile(T* lds, const Stencil& S, const TileLayout& L, const double* __restrict__ xhat,
                         int r0, int c0, bool xs_staged = false) {
    constexpr int R = RB;
    const int E = L.E, RW = L.RW, RH = L.RH;
    const T* __restrict__ v = lds + L.o_v;
    T* __restrict__ h1 = lds + L.o_h1;
    T* __restrict__ t1 = lds + L.o_t1;
    T* __restrict__ out = lds + L.o_out;
    T g[2 * RB + 1];
#pragma unroll
    for (int a = 0; a <= 2 * RB; ++a) g[a] = (T)S.g[a];

    // ---- A(A v), separable
    const int W1 = TW + 2 * R;
    TILE_LOOP(RH, W1, rr, cc) {                                       // rows of region 0
        const int idx = rr * W1 + cc;
        const T* src = v + rr * RW + cc + (E - R) - R;
        T acc = T(0);
        _Pragma("unroll") for (int b = 0; b <= 2 * R; ++b) acc += g[b] * src[b];
        h1[idx] = acc;
    }
    __syncthreads();
    const int H1 = TH + 2 * R;
    TILE_LOOP(H1, W1, rr, cc) {                                       // columns -> A v
        const int idx = rr * W1 + cc;
        const T* src = h1 + (rr + E - R - R) * W1 + cc;
        T acc = T(0);
        _Pragma("unroll") for (int a = 0; a <= 2 * R; ++a) acc += g[a] * src[a * W1];
        const int gi = r0 - R + rr, gj = c0 - R + cc;
        t1[idx] = (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) ? acc : T(0);
    }
    __syncthreads();
    T* __restrict__ h2 = h1;                                          // reuse: (TH+2R) x TW
    TILE_LOOP(H1, TW, rr, cc) {
        const int idx = rr * TW + cc;
        const T* src = t1 + rr * W1 + cc;
        T acc = T(0);
        _Pragma("unroll") for (int b = 0; b <= 2 * R; ++b) acc += g[b] * src[b];
        h2[idx] = acc;
    }
    __syncthreads();
    TILE_LOOP(TH, TW, rr, cc) {
        const int idx = rr * TW + cc;
        const T* src = h2 + rr * TW + cc;
        T acc = T(0);
        _Pragma("unroll") for (int a = 0; a <= 2 * R; ++a) acc += g[a] * src[a * TW];
        out[idx] = T(2) * acc;
    }

    if (S.reg == BL_REG_TV) {
        // ---- lambda D^T (B D v)
        T* xs = lds + L.o_x;               // xhat on [r0-1, r0+TH+1) x [c0-1, c0+TW+1)
        T* fx = lds + L.o_fx;              // flux on [r0-1, r0+TH) x [c0-1, c0+TW)
        T* fy = lds + L.o_fy;
        const int XW = TW + 2;
        if (!xs_staged) {
            stage_xhat<T>(xs, S, xhat, r0, c0);
            __syncthreads();
        }
        const T gam2 = (T)S.gam2;
        const int FW = TW + 1;
        TILE_LOOP((TH + 1), FW, rr, cc) {
            const int idx = rr * FW + cc;
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            T fxv = T(0), fyv = T(0);
            if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) {
                const T xc = xs[rr * XW + cc];
                const T a = (gj < S.w - 1) ? xs[rr * XW + cc + 1] - xc : T(0);
                const T b = (gi < S.h - 1) ? xs[(rr + 1) * XW + cc] - xc : T(0);
                const T* vc = v + (rr - 1 + E) * RW + (cc - 1 + E);
                const T da = (gj < S.w - 1) ? vc[1] - vc[0] : T(0);
                const T db = (gi < S.h - 1) ? vc[RW] - vc[0] : T(0);
                const T psi2 = a * a + b * b + gam2;
                const T psi = sqrt(psi2);
                const T ip3 = T(1) / (psi2 * psi);
                fxv = ((b * b + gam2) * da - a * b * db) * ip3;
                fyv = ((a * a + gam2) * db - a * b * da) * ip3;
            }
            fx[idx] = fxv;
            fy[idx] = fyv;
        }
        __syncthreads();
        const T lam = (T)S.lam;
        TILE_LOOP(TH, TW, rr, cc) {
            const int idx = rr * TW + cc;
            const int f = (rr + 1) * FW + (cc + 1);
            const T dt = -fx[f] + fx[f - 1] - fy[f] + fy[f - FW];
            out[idx] += lam * dt;
        }
        __syncthreads();
    } else {
        // ---- eps v + sum_j lambda_j K_j^T (phi''_j . K_j v)
        const int F = L.F, fs = S.fs, TWF = TW + 2 * F, THF = TH + 2 * F;
        T* tb = lds + L.o_t;
        T* taps = lds + L.o_taps;
        const int ntap = S.nf * fs * fs;
        for (int k = threadIdx.x; k < ntap + S.nf; k += NT)
            taps[k] = (k < ntap) ? (T)S.taps[k] : (T)S.lamj[k - ntap];
        const T eps = (T)S.eps;
        TILE_LOOP(TH, TW, rr, cc) {
            const int idx = rr * TW + cc;
            out[idx] += eps * v[(rr + E) * RW + (cc + E)];
        }
        __syncthreads();
        for (int j = 0; j < S.nf; ++j) {
            const T* kj = taps + j * fs * fs;
            TILE_LOOP(THF, TWF, rr, cc) {
                const int idx = rr * TWF + cc;
                const int gi = r0 - F + rr, gj = c0 - F + cc;
                T val = T(0);
                if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) {
                    const T* src = v + (rr + E - F - F) * RW + (cc + E - F - F);
                    T acc = T(0);
                    for (int a = 0; a < fs; ++a)
                        for (int b = 0; b < fs; ++b) acc += kj[a * fs + b] * src[a * RW + b];
                    const size_t gidx = (size_t)j * S.n + (size_t)gi * S.w + gj;
                    const T d2 = (sizeof(T) == 4) ? (T)S.d2f[gidx] : (T)S.d2[gidx];
                    val = d2 * acc;
                }
                tb[idx] = val;
            }
            __syncthreads();
            const T lj = taps[ntap + j];
            TILE_LOOP(TH, TW, rr, cc) {
                const int idx = rr * TW + cc;
                // K^T t at (rr, cc): sum_{a,b} k[a][b] t(rr - (a - F), cc - (b - F))
                const T* src = tb + (rr + F + F) * TWF + (cc + F + F);
                T acc = T(0);
                for (int a = 0; a < fs; ++a)
                    for (int b = 0; b < fs; ++b) acc += kj[a * fs + b] * src[-a * TWF - b];
                out[idx] += lj * acc;
            }
            __syncthreads();
        }
    }
}

}  // namespace bl
