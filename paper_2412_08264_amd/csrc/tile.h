// Hessian-vector product on 32 x (8 Q) pixel tiles (256 threads, Q = 1, 2 or 4 pixels per thread).
//
// The Hessian of the lower-level objective (Section 2.1; TV and filter regularisers of
// Section 5):  H v = 2 A^T A v + lambda D^T (B(x) D v)            (smoothed TV)
//              H v = 2 A^T A v + eps v + sum_j lambda_j K_j^T (phi''_j . K_j v)   (filters)
// with A the normalised (2R+1)^2 Gaussian correlation (zero outside the image, A^T = A).
//
// A block stages v on its tile plus a halo of E = max(2R, 2F, 1) pixels into LDS once and
// evaluates every term from there.  Thread (tx, ty) owns column tx and rows Q ty .. Q ty + Q - 1
// of the tile; the result of those Q pixels is returned in registers.  The TV term's 2 x 2
// flux blocks, which depend on x_hat only, are formed in registers by each thread for the
// flux points around its own pixels (x_hat read from global memory, no LDS), and A v takes the
// LDS space of the staged v once that is no longer read, so a TV tile holds two regions.
// Taller tiles share
// more halo and register windows per staged value; shorter ones give small images more
// blocks (the rows per tile of each operator class and image size come from a timing
// autotuner, with a block-count rule as the default).  Passes along
// columns work on strips of consecutive rows held in registers, so every LDS value loaded
// serves several outputs; the filter correlation loads each input window once and applies
// all filters to it; filter taps are uniform (scalar) loads.
#pragma once

#include <type_traits>

#include "common.h"

namespace bl {

constexpr int QW = 32;                  // tile columns
constexpr int QTY = NT / QW;            // thread rows of a block (8); a tile has QTY * Q rows

enum TileClass { TC_TV = 0, TC_F7 = 1, TC_FG = 2 };   // TV; filters 7x7; filters of another size

__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int R, int CLS, int Q>
struct QGeo {
    static constexpr int QH = QTY * Q;                       // tile rows
    static constexpr int F = CLS == TC_TV ? 0 : 3;           // largest filter half-size
    static constexpr int E = cmax(cmax(2 * R, 2 * F), 1);    // halo of the staged region
    static constexpr int RW = QW + 2 * E, RH = QH + 2 * E;   // staged region
    static constexpr int W1 = QW + 2 * R, H1 = QH + 2 * R;   // where A v is needed
    static constexpr int HR = QH + 4 * R;                    // rows of the first horizontal pass
    static constexpr int N_V = RH * RW;
    static constexpr int N_H = cmax(HR * W1, H1 * QW);
    static constexpr int N_T1 = H1 * W1;
    static constexpr int TWF = QW + 2 * F, THF = QH + 2 * F; // where K_j v is needed
};

template <typename T, int R, int CLS, int Q>
struct QLayout {
    using G = QGeo<R, CLS, Q>;
    static constexpr int NFG = CLS == TC_TV ? 1 : (sizeof(T) == 8 ? 4 : 8);   // filters per LDS pass
    static constexpr int o_v = 0;
    static constexpr int o_h = o_v + G::N_V;
    // TV: A v replaces the staged v (read by the first pass only; N_T1 <= N_V); the filter
    // terms read v again after the blur
    static constexpr int o_t1 = CLS == TC_TV ? o_v : o_h + G::N_H;
    static constexpr int o_tb = o_h;   // filters: the blur scratch is reused once A^T A v is in registers
    static constexpr int total = CLS == TC_TV ? o_h + G::N_H : cmax(o_tb + NFG * G::THF * G::TWF, o_t1 + G::N_T1);
    static_assert(G::N_T1 <= G::N_V, "A v must fit in the staged region");
    // the kernels reuse the region for their per-wave record sums (NWAVE x NV_RED doubles) once
    // the product is in registers
    static constexpr size_t bytes = cmax(total * (int)sizeof(T), NWAVE * NV_RED * (int)sizeof(double));
};

__host__ __device__ inline int tile_class(int reg, int fs) {
    return reg == BL_REG_TV ? TC_TV : (fs == 7 ? TC_F7 : TC_FG);
}

// Stage fetch(global index) on the region [r0-E, r0+QH+E) x [c0-E, c0+QW+E), zero outside
// the image; all of a thread's loads are issued before the first store.
template <typename T, int R, int CLS, int Q, typename Fetch>
__device__ __forceinline__ void q_stage(T* buf, int h, int w, int r0, int c0, Fetch fetch) {
    using G = QGeo<R, CLS, Q>;
    constexpr int NST = (G::N_V + NT - 1) / NT;
    double val[NST];
#pragma unroll
    for (int u = 0; u < NST; ++u) {
        const int idx = threadIdx.x + u * NT;
        val[u] = 0.0;
        if (idx < G::N_V) {
            const int rr = idx / G::RW, cc = idx - rr * G::RW;
            const int gi = r0 - G::E + rr, gj = c0 - G::E + cc;
            if (gi >= 0 && gi < h && gj >= 0 && gj < w) val[u] = fetch(gi * w + gj);
        }
    }
#pragma unroll
    for (int u = 0; u < NST; ++u) {
        const int idx = threadIdx.x + u * NT;
        if (idx < G::N_V) buf[idx] = (T)val[u];
    }
}

// 1 / sqrt(x) for x > 0: the hardware estimate refined by Newton's iteration for x^(-1/2),
// y <- y + y (1 - x y^2) / 2, which doubles the correct bits per step (two steps in FP64 from
// the estimate's roughly 22 bits, one in FP32).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
}

// TV: x_hat around the thread's pixels (rows i0 .. i0 + Q - 1 of column j), zero outside the
// image.  Loaded once per launch; the flux blocks below depend on nothing else.
template <int Q>
struct TvX {
    double c[Q + 2];   // column j, rows i0 - 1 .. i0 + Q
    double r[Q + 1];   // column j + 1, rows i0 - 1 .. i0 + Q - 1
    double l[Q + 1];   // column j - 1, rows i0 .. i0 + Q
};
template <int Q>
__device__ __forceinline__ TvX<Q> tv_xload(int h, int w, const double* __restrict__ xhat, int r0, int c0) {
    const int tx = threadIdx.x & (QW - 1), ty = threadIdx.x / QW;
    const int i0 = r0 + Q * ty, j = c0 + tx;
    const gbl_t<const double> gx = gbl(xhat);
    auto at = [&](int i, int jj) { return (i >= 0 && i < h && jj >= 0 && jj < w) ? gx[i * w + jj] : 0.0; };
    TvX<Q> X;
#pragma unroll
    for (int m = 0; m < Q + 2; ++m) X.c[m] = at(i0 - 1 + m, j);
#pragma unroll
    for (int m = 0; m < Q + 1; ++m) X.r[m] = at(i0 - 1 + m, j + 1);
#pragma unroll
    for (int m = 0; m < Q + 1; ++m) X.l[m] = at(i0 + m, j - 1);
    return X;
}

// The smoothed-TV Hessian (Section 5, eq. of the smoothed TV regulariser) is D^T B(x) D with, at
// flux point (i, j), a = x(i, j+1) - x(i, j), b = x(i+1, j) - x(i, j) (zero on the last column
// / row, where the forward difference is not taken) and psi^2 = a^2 + b^2 + gamma^2, the block
//   psi^-3 [[b^2 + gamma^2, -a b], [-a b, a^2 + gamma^2]]
// acting on the differences (dx, dy) of v.  The coefficient of a difference that is not taken is
// set to zero (then so is -a b), and a point outside the image has no flux.
template <typename T>
__device__ __forceinline__ void tv_block(double xc, double xr, double xd, bool in, bool last_col, bool last_row,
                                         T gam2, T& c11, T& c12, T& c22) {
    const T a = last_col ? T(0) : (T)xr - (T)xc;
    const T b = last_row ? T(0) : (T)xd - (T)xc;
    const T psi2 = a * a + b * b + gam2;
    const T y = rsqrt_nr(psi2);
    const T s3 = y * y * y;
    c11 = (in && !last_col) ? (b * b + gam2) * s3 : T(0);
    c12 = in ? -(a * b) * s3 : T(0);
    c22 = (in && !last_row) ? (a * a + gam2) * s3 : T(0);
}

// x_hat around the thread's pixels for a TV tile (nothing is loaded for the filter classes).
template <int CLS, int Q>
__device__ __forceinline__ TvX<Q> tv_x(int h, int w, const double* __restrict__ xhat, int r0, int c0) {
    TvX<Q> X{};
    if constexpr (CLS == TC_TV) X = tv_xload<Q>(h, w, xhat, r0, c0);
    return X;
}

// Filter taps and weights of filter j in precision T: k_j (fs*fs) then lambda_j at nf*fs*fs + j.
// Read through global pointers: uniform tap loads become scalar loads, and the phi'' loads
// global ones, so that neither waits behind LDS traffic (as flat loads would).
template <typename T>
__device__ __forceinline__ gbl_t<const T> taps_of(const Stencil& S);
template <>
__device__ __forceinline__ gbl_t<const double> taps_of<double>(const Stencil& S) { return gbl(S.taps); }
template <>
__device__ __forceinline__ gbl_t<const float> taps_of<float>(const Stencil& S) { return gbl(S.tapsf); }

template <typename T>
__device__ __forceinline__ T d2_at(const Stencil& S, size_t gidx);
template <>
__device__ __forceinline__ double d2_at<double>(const Stencil& S, size_t gidx) { return gbl(S.d2)[gidx]; }
template <>
__device__ __forceinline__ float d2_at<float>(const Stencil& S, size_t gidx) { return gbl(S.d2f)[gidx]; }

// Horizontal pass of the separable blur: dst[r][c] = sum_b g[b] src[r][c + b] for r < NR,
// c < NC (src rows hold NC + 2R values).  A thread computes SEG consecutive outputs of one row
// from a register window of SEG + 2R inputs, so each LDS value it loads serves up to 2R + 1
// outputs; SEG is the segment length with the fewest loads per thread over the block's rounds.
__host__ __device__ constexpr int hseg_cost(int nr, int nc, int r, int seg) {
    return ((nr * ((nc + seg - 1) / seg) + NT - 1) / NT) * (seg + 2 * r);
}
__host__ __device__ constexpr int hseg(int nr, int nc, int r) {
    int best = 1;
    for (int seg = 2; seg <= 8; ++seg)
        if (hseg_cost(nr, nc, r, seg) < hseg_cost(nr, nc, r, best)) best = seg;
    return best;
}
template <typename T, int R, int NR, int NC, int SLD, int DLD>
__device__ __forceinline__ void hpass(const T* src, T* __restrict__ dst, const T* g) {
    constexpr int SEG = hseg(NR, NC, R);
    constexpr int SPR = (NC + SEG - 1) / SEG;   // segments per row
    for (int item = threadIdx.x; item < NR * SPR; item += NT) {
        const int r = item / SPR, c0 = (item - r * SPR) * SEG;
        const T* sr = src + r * SLD + c0;
        T win[SEG + 2 * R];
#pragma unroll
        for (int u = 0; u < SEG + 2 * R; ++u) win[u] = (c0 + u < NC + 2 * R) ? sr[u] : T(0);
#pragma unroll
        for (int k = 0; k < SEG; ++k) {
            T acc = T(0);
#pragma unroll
            for (int b = 0; b <= 2 * R; ++b) acc += g[b] * win[k + b];
            if (c0 + k < NC) dst[r * DLD + c0 + k] = acc;
        }
    }
}

// H v at the thread's Q pixels (rows r0 + Q ty + k, column c0 + tx) from the staged region
// (and, for TV, x_hat around them, X), into out[].  Ends with a barrier after its last LDS read.
template <typename T, int R, int CLS, int Q>
__device__ __forceinline__ void q_hvp(T* lds, const Stencil& S, int r0, int c0, T out[Q], const TvX<Q>& X) {
    using G = QGeo<R, CLS, Q>;
    using L = QLayout<T, R, CLS, Q>;
    constexpr int QR = Q;
    // (TV: t1 and v share their space: no restrict on either)
    const T* v = lds + L::o_v;
    T* __restrict__ hb = lds + L::o_h;
    T* t1 = lds + L::o_t1;
    const int tx = threadIdx.x & (QW - 1), ty = threadIdx.x / QW;
    const int h = S.h, w = S.w;
    T g[2 * R + 1];
#pragma unroll
    for (int a = 0; a <= 2 * R; ++a) g[a] = (T)S.g[a];

    // TV: the divergence D^T B D v at the own pixels, from the staged v (x_hat is not needed
    // after this).  Each flux block is formed where it is used.
    T div[QR];
    if constexpr (CLS == TC_TV) {
        const int i0 = r0 + QR * ty, j = c0 + tx;
        const T g2 = (T)S.gam2;
        const T* vc = v + (QR * ty + G::E) * G::RW + (tx + G::E);   // the thread's first pixel
        T b11, b12, b22;
        // y flux at (i0 - 1, j)
        tv_block<T>(X.c[0], X.r[0], X.c[1], i0 >= 1 && i0 - 1 < h && j < w, j == w - 1, i0 - 1 == h - 1, g2, b11,
                    b12, b22);
        T fy_up = b12 * (vc[1 - G::RW] - vc[-G::RW]) + b22 * (vc[0] - vc[-G::RW]);
#pragma unroll
        for (int k = 0; k < QR; ++k) {
            const int i = i0 + k;
            const T* p = vc + k * G::RW;
            const T da = p[1] - p[0], db = p[G::RW] - p[0];
            tv_block<T>(X.c[k + 1], X.r[k + 1], X.c[k + 2], i < h && j < w, j == w - 1, i == h - 1, g2, b11, b12,
                        b22);
            const T fx = b11 * da + b12 * db;
            const T fy = b12 * da + b22 * db;
            tv_block<T>(X.l[k], X.c[k + 1], X.l[k + 1], i < h && j >= 1 && j - 1 < w, j - 1 == w - 1, i == h - 1, g2,
                        b11, b12, b22);
            const T fx_left = b11 * (p[0] - p[-1]) + b12 * (p[G::RW - 1] - p[-1]);
            div[k] = -fx + fx_left - fy + fy_up;
            fy_up = fy;
        }
    }
    // ---- pass 1: rows of the region, hb = horizontal blur of v on HR x W1
    hpass<T, R, G::HR, G::W1, G::RW, G::W1>(v + (G::E - 2 * R) * G::RW + (G::E - 2 * R), hb, g);
    __syncthreads();
    // ---- pass 2: t1 = A v on H1 x W1 (columns, strips of 4 rows), zero outside the image
    {
        constexpr int NS = (G::H1 + 3) / 4;
        for (int q = threadIdx.x; q < NS * G::W1; q += NT) {
            const int sidx = q / G::W1, c = q - sidx * G::W1, rb = 4 * sidx;
            T col[4 + 2 * R];
#pragma unroll
            for (int u = 0; u < 4 + 2 * R; ++u) col[u] = (rb + u < G::HR) ? hb[(rb + u) * G::W1 + c] : T(0);
            const int gj = c0 - R + c;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int r = rb + k;
                if (r < G::H1) {
                    T acc = T(0);
#pragma unroll
                    for (int a = 0; a <= 2 * R; ++a) acc += g[a] * col[k + a];
                    const int gi = r0 - R + r;
                    t1[r * G::W1 + c] = (gi >= 0 && gi < h && gj >= 0 && gj < w) ? acc : T(0);
                }
            }
        }
    }
    __syncthreads();
    // ---- pass 3: hb = horizontal blur of t1 on H1 x QW
    hpass<T, R, G::H1, QW, G::W1, QW>(t1, hb, g);
    __syncthreads();
    // ---- pass 4: own strip, out = 2 A(A v)
    {
        T col[QR + 2 * R];
#pragma unroll
        for (int u = 0; u < QR + 2 * R; ++u) col[u] = hb[(QR * ty + u) * QW + tx];
#pragma unroll
        for (int k = 0; k < QR; ++k) {
            T acc = T(0);
#pragma unroll
            for (int a = 0; a <= 2 * R; ++a) acc += g[a] * col[k + a];
            out[k] = T(2) * acc;
        }
    }
    if constexpr (CLS == TC_TV) {
        const T lam = (T)S.lam;
#pragma unroll
        for (int k = 0; k < QR; ++k) out[k] += lam * div[k];
        __syncthreads();
    } else {
        const T eps = (T)S.eps;
#pragma unroll
        for (int k = 0; k < QR; ++k) out[k] += eps * v[(QR * ty + k + G::E) * G::RW + tx + G::E];
        const int nf = S.nf;
        const gbl_t<const T> __restrict__ tp = taps_of<T>(S);
        constexpr int NFG = L::NFG;
        T* __restrict__ tb = lds + L::o_tb;
        if constexpr (CLS == TC_F7) {
            constexpr int FS = 7, F = 3, F2 = 49;
            for (int j0 = 0; j0 < nf; j0 += NFG) {
                __syncthreads();   // the previous readers of the tb space are done
                // t_j = lambda_j phi''_j (K_j v) on THF x TWF, strips of 2 rows; the phi'' values of
                // the next strip are loaded while the current one is computed
                constexpr int NS = (G::THF + 1) / 2;
                auto load_d2 = [&](int q, T (&dst)[NFG][2]) {
                    const int sidx = q / G::TWF, cc = q - sidx * G::TWF, rb = 2 * sidx;
                    const int gj = c0 - F + cc;
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int gi = r0 - F + rb + k;
                        const bool in = q < NS * G::TWF && rb + k < G::THF && gi >= 0 && gi < h && gj >= 0 && gj < w;
#pragma unroll
                        for (int jj = 0; jj < NFG; ++jj)
                            dst[jj][k] = (in && j0 + jj < nf)
                                             ? d2_at<T>(S, (size_t)(j0 + jj) * S.n + (size_t)gi * w + gj)
                                             : T(0);
                    }
                };
                T d2n[NFG][2];
                load_d2(threadIdx.x, d2n);
                for (int q = threadIdx.x; q < NS * G::TWF; q += NT) {
                    const int sidx = q / G::TWF, cc = q - sidx * G::TWF, rb = 2 * sidx;
                    T d2v[NFG][2];
#pragma unroll
                    for (int jj = 0; jj < NFG; ++jj) {
                        d2v[jj][0] = d2n[jj][0];
                        d2v[jj][1] = d2n[jj][1];
                    }
                    load_d2(q + NT, d2n);
                    T win[2 + FS - 1][FS];
#pragma unroll
                    for (int u = 0; u < 2 + FS - 1; ++u)
#pragma unroll
                        for (int b = 0; b < FS; ++b) {
                            const int rr = rb + u + G::E - 2 * F;
                            win[u][b] = rr < G::RH ? v[rr * G::RW + cc + b + G::E - 2 * F] : T(0);
                        }
#pragma unroll
                    for (int jj = 0; jj < NFG; ++jj) {
                        if (j0 + jj >= nf) break;
                        const gbl_t<const T> kj = tp + (j0 + jj) * F2;
                        T acc0 = T(0), acc1 = T(0);
#pragma unroll
                        for (int a = 0; a < FS; ++a)
#pragma unroll
                            for (int b = 0; b < FS; ++b) {
                                const T kv = kj[a * FS + b];
                                acc0 += kv * win[a][b];
                                acc1 += kv * win[a + 1][b];
                            }
                        const T lj = tp[nf * F2 + j0 + jj];
                        T* tj = tb + jj * G::THF * G::TWF;
                        tj[rb * G::TWF + cc] = lj * d2v[jj][0] * acc0;
                        if (rb + 1 < G::THF) tj[(rb + 1) * G::TWF + cc] = lj * d2v[jj][1] * acc1;
                    }
                }
                __syncthreads();
                // K_j^T t_j at the own strip: sum_{a,b} k[a][b] t(i - (a - F), j - (b - F))
#pragma unroll 1
                for (int jj = 0; jj < NFG; ++jj) {
                    if (j0 + jj >= nf) break;
                    const gbl_t<const T> kj = tp + (j0 + jj) * F2;
                    const T* tj = tb + jj * G::THF * G::TWF;
                    T win[QR + FS - 1][FS];
#pragma unroll
                    for (int u = 0; u < QR + FS - 1; ++u)
#pragma unroll
                        for (int b = 0; b < FS; ++b) win[u][b] = tj[(QR * ty + u) * G::TWF + tx + b];
#pragma unroll
                    for (int k = 0; k < QR; ++k) {
                        T acc = T(0);
#pragma unroll
                        for (int a = 0; a < FS; ++a)
#pragma unroll
                            for (int b = 0; b < FS; ++b) acc += kj[a * FS + b] * win[k + 2 * F - a][2 * F - b];
                        out[k] += acc;
                    }
                }
            }
        } else {
            // any odd size fs <= 7: the same passes with run-time loops (no register windows)
            const int fs = S.fs, F = fs / 2, f2 = fs * fs;
            for (int j0 = 0; j0 < nf; j0 += NFG) {
                __syncthreads();
                for (int idx = threadIdx.x; idx < G::THF * G::TWF; idx += NT) {
                    const int rr = idx / G::TWF, cc = idx - rr * G::TWF;
                    // tb covers [r0 - 3, ..) x [c0 - 3, ..); positions within F of the tile are used
                    const int gi = r0 - G::F + rr, gj = c0 - G::F + cc;
                    const bool in = gi >= 0 && gi < h && gj >= 0 && gj < w;
                    for (int jj = 0; jj < NFG && j0 + jj < nf; ++jj) {
                        T val = T(0);
                        if (in) {
                            const gbl_t<const T> kj = tp + (j0 + jj) * f2;
                            const T* src = v + (rr + G::E - G::F - F) * G::RW + (cc + G::E - G::F - F);
                            T acc = T(0);
                            for (int a = 0; a < fs; ++a)
                                for (int b = 0; b < fs; ++b) acc += kj[a * fs + b] * src[a * G::RW + b];
                            val = tp[nf * f2 + j0 + jj] * d2_at<T>(S, (size_t)(j0 + jj) * S.n + (size_t)gi * w + gj) * acc;
                        }
                        tb[jj * G::THF * G::TWF + idx] = val;
                    }
                }
                __syncthreads();
                for (int jj = 0; jj < NFG && j0 + jj < nf; ++jj) {
                    const gbl_t<const T> kj = tp + (j0 + jj) * f2;
                    const T* tj = tb + jj * G::THF * G::TWF;
                    for (int k = 0; k < QR; ++k) {
                        const int rr = QR * ty + k + G::F, cc = tx + G::F;   // own pixel in tb coordinates
                        T acc = T(0);
                        for (int a = 0; a < fs; ++a)
                            for (int b = 0; b < fs; ++b) acc += kj[a * fs + b] * tj[(rr + F - a) * G::TWF + cc + F - b];
                        out[k] += acc;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Run fn(integral_constant<R>, integral_constant<class>) for the run-time radius and class.
template <typename Fn>
inline void q_dispatch(int R, int cls, Fn&& fn) {
    auto by_cls = [&](auto rc) {
        switch (cls) {
            case TC_TV: fn(rc, std::integral_constant<int, TC_TV>{}); break;
            case TC_F7: fn(rc, std::integral_constant<int, TC_F7>{}); break;
            default: fn(rc, std::integral_constant<int, TC_FG>{}); break;
        }
    };
    switch (R) {
        case 0: by_cls(std::integral_constant<int, 0>{}); break;
        case 1: by_cls(std::integral_constant<int, 1>{}); break;
        case 2: by_cls(std::integral_constant<int, 2>{}); break;
        case 3: by_cls(std::integral_constant<int, 3>{}); break;
        case 4: by_cls(std::integral_constant<int, 4>{}); break;
        case 5: by_cls(std::integral_constant<int, 5>{}); break;
        case 6: by_cls(std::integral_constant<int, 6>{}); break;
        case 7: by_cls(std::integral_constant<int, 7>{}); break;
        default: by_cls(std::integral_constant<int, 8>{}); break;
    }
}

}  // namespace bl
