// Hessian-vector product on 32 x (8 Q) pixel tiles (256 threads, Q = 1, 2 or 4 pixels per thread).
//
// The Hessian of the lower-level objective (Section 2.1; TV and filter regularisers of
// Section 5):  H v = 2 A^T A v + lambda D^T (B(x) D v)            (smoothed TV)
//              H v = 2 A^T A v + eps v + sum_j lambda_j K_j^T (phi''_j . K_j v)   (filters)
// with A the normalised (2R+1)^2 Gaussian correlation (zero outside the image, A^T = A).
//
// A block stages v on its tile plus a halo of E = max(2R, 2F, 1) pixels into LDS once and
// evaluates every term from there.  Thread (tx, ty) owns column tx and rows Q ty .. Q ty + Q - 1
// of the tile; the result of those Q pixels is returned in registers.  Taller tiles share
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
    static constexpr int N_X = (QH + 2) * (QW + 2);          // TV: xhat with a 1-pixel halo
    static constexpr int N_FL = (QH + 1) * (QW + 1);         // TV: flux grid
};

template <typename T, int R, int CLS, int Q>
struct QLayout {
    using G = QGeo<R, CLS, Q>;
    static constexpr int NFG = CLS == TC_TV ? 1 : (sizeof(T) == 8 ? 4 : 8);   // filters per LDS pass
    static constexpr int o_v = 0;
    static constexpr int o_h = o_v + G::N_V;
    static constexpr int o_t1 = o_h + G::N_H;
    static constexpr int o_x = o_t1 + G::N_T1;
    static constexpr int o_fx = o_x + G::N_X;
    static constexpr int o_fy = o_fx + G::N_FL;
    static constexpr int o_tb = o_h;   // filters: the blur scratch is reused once A^T A v is in registers
    static constexpr int total = CLS == TC_TV ? o_fy + G::N_FL : cmax(o_tb + NFG * G::THF * G::TWF, o_t1 + G::N_T1);
    static constexpr size_t bytes = (size_t)total * sizeof(T);
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

// TV: stage xhat on [r0-1, r0+QH+1) x [c0-1, c0+QW+1).
template <typename T, int Q>
__device__ __forceinline__ void q_stage_xhat(T* xs, int h, int w, const double* __restrict__ xhat, int r0, int c0) {
    constexpr int XW = QW + 2, TOT = (QTY * Q + 2) * XW, NST = (TOT + NT - 1) / NT;
    double val[NST];
#pragma unroll
    for (int u = 0; u < NST; ++u) {
        const int idx = threadIdx.x + u * NT;
        val[u] = 0.0;
        if (idx < TOT) {
            const int rr = idx / XW, cc = idx - rr * XW;
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            if (gi >= 0 && gi < h && gj >= 0 && gj < w) val[u] = xhat[gi * w + gj];
        }
    }
#pragma unroll
    for (int u = 0; u < NST; ++u) {
        const int idx = threadIdx.x + u * NT;
        if (idx < TOT) xs[idx] = (T)val[u];
    }
}

// Filter taps and weights of filter j in precision T: k_j (fs*fs) then lambda_j at nf*fs*fs + j.
template <typename T>
__device__ __forceinline__ const T* taps_of(const Stencil& S);
template <>
__device__ __forceinline__ const double* taps_of<double>(const Stencil& S) { return S.taps; }
template <>
__device__ __forceinline__ const float* taps_of<float>(const Stencil& S) { return S.tapsf; }

template <typename T>
__device__ __forceinline__ T d2_at(const Stencil& S, size_t gidx);
template <>
__device__ __forceinline__ double d2_at<double>(const Stencil& S, size_t gidx) { return S.d2[gidx]; }
template <>
__device__ __forceinline__ float d2_at<float>(const Stencil& S, size_t gidx) { return S.d2f[gidx]; }

// H v at the thread's Q pixels (rows r0 + Q ty + k, column c0 + tx) from the staged region
// (and, for TV, the staged xhat), into out[].  Ends with a barrier after its last LDS read.
template <typename T, int R, int CLS, int Q>
__device__ __forceinline__ void q_hvp(T* lds, const Stencil& S, int r0, int c0, T out[Q]) {
    using G = QGeo<R, CLS, Q>;
    using L = QLayout<T, R, CLS, Q>;
    constexpr int QR = Q;
    const T* __restrict__ v = lds + L::o_v;
    T* __restrict__ hb = lds + L::o_h;
    T* __restrict__ t1 = lds + L::o_t1;
    const int tx = threadIdx.x & (QW - 1), ty = threadIdx.x / QW;
    const int h = S.h, w = S.w;
    T g[2 * R + 1];
#pragma unroll
    for (int a = 0; a <= 2 * R; ++a) g[a] = (T)S.g[a];

    // ---- pass 1: rows of the region, hb = horizontal blur of v  (and the TV flux)
    for (int idx = threadIdx.x; idx < G::HR * G::W1; idx += NT) {
        const int rh = idx / G::W1, ch = idx - rh * G::W1;
        const T* src = v + (rh + G::E - 2 * R) * G::RW + ch + G::E - 2 * R;
        T acc = T(0);
#pragma unroll
        for (int b = 0; b <= 2 * R; ++b) acc += g[b] * src[b];
        hb[idx] = acc;
    }
    if constexpr (CLS == TC_TV) {
        const T* __restrict__ xs = lds + L::o_x;
        T* __restrict__ fx = lds + L::o_fx;
        T* __restrict__ fy = lds + L::o_fy;
        constexpr int XW = QW + 2, FW = QW + 1;
        const T gam2 = (T)S.gam2;
        for (int idx = threadIdx.x; idx < G::N_FL; idx += NT) {
            const int rr = idx / FW, cc = idx - rr * FW;
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            T fxv = T(0), fyv = T(0);
            if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
                const T xc = xs[rr * XW + cc];
                const T a = (gj < w - 1) ? xs[rr * XW + cc + 1] - xc : T(0);
                const T b = (gi < h - 1) ? xs[(rr + 1) * XW + cc] - xc : T(0);
                const T* vc = v + (rr - 1 + G::E) * G::RW + (cc - 1 + G::E);
                const T da = (gj < w - 1) ? vc[1] - vc[0] : T(0);
                const T db = (gi < h - 1) ? vc[G::RW] - vc[0] : T(0);
                const T psi2 = a * a + b * b + gam2;
                const T psi = sqrt(psi2);
                const T ip3 = T(1) / (psi2 * psi);
                fxv = ((b * b + gam2) * da - a * b * db) * ip3;
                fyv = ((a * a + gam2) * db - a * b * da) * ip3;
            }
            fx[idx] = fxv;
            fy[idx] = fyv;
        }
    }
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
    for (int idx = threadIdx.x; idx < G::H1 * QW; idx += NT) {
        const int r = idx / QW, c = idx - r * QW;
        const T* src = t1 + r * G::W1 + c;
        T acc = T(0);
#pragma unroll
        for (int b = 0; b <= 2 * R; ++b) acc += g[b] * src[b];
        hb[idx] = acc;
    }
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
        // ---- lambda D^T (flux) at the own pixels
        const T* __restrict__ fx = lds + L::o_fx;
        const T* __restrict__ fy = lds + L::o_fy;
        constexpr int FW = QW + 1;
        const T lam = (T)S.lam;
#pragma unroll
        for (int k = 0; k < QR; ++k) {
            const int f = (QR * ty + k + 1) * FW + (tx + 1);
            out[k] += lam * (-fx[f] + fx[f - 1] - fy[f] + fy[f - FW]);
        }
        __syncthreads();
    } else {
        const T eps = (T)S.eps;
#pragma unroll
        for (int k = 0; k < QR; ++k) out[k] += eps * v[(QR * ty + k + G::E) * G::RW + tx + G::E];
        const int nf = S.nf;
        const T* __restrict__ tp = taps_of<T>(S);
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
                        const T* kj = tp + (j0 + jj) * F2;
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
                    const T* kj = tp + (j0 + jj) * F2;
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
                            const T* kj = tp + (j0 + jj) * f2;
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
                    const T* kj = tp + (j0 + jj) * f2;
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
