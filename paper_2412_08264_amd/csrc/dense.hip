// Dense kernels of the recycle-space refresh: tall-skinny Gram products, tall x small
// products, and single-workgroup small dense algebra (Cholesky with column drop, a
// symmetric eigensolver (Householder tridiagonalisation, multisection, inverse iteration),
// projected GSVD and Ritz-GSV selection).
#include <algorithm>

#include "kernels.h"

namespace bl {

// ------------------------------------------------------------------ Gram: Out = A^T B
// A: n x t1, B: n x t2 (column-major, ld n).  Block (chunk, ti, tj) accumulates a 32 x 32
// output tile over rows [chunk*GRAM_CHUNK, ...); partials are summed in chunk order.
constexpr int GRAM_T = 32;
constexpr int GRAM_ROWS = 32;

__global__ void __launch_bounds__(NT) k_gram(int n, int t1, int t2, const double* __restrict__ A,
                                             const double* __restrict__ B, int chunk_rows,
                                             double* __restrict__ part) {
    __shared__ double As[GRAM_ROWS][GRAM_T + 1];
    __shared__ double Bs[GRAM_ROWS][GRAM_T + 1];
    const int ti = blockIdx.y * GRAM_T, tj = blockIdx.z * GRAM_T;
    const int row0 = blockIdx.x * chunk_rows;
    const int row1 = min(n, row0 + chunk_rows);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // 16 x 16 threads, 2 x 2 outputs each
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int rb = row0; rb < row1; rb += GRAM_ROWS) {
        for (int idx = threadIdx.x; idx < GRAM_ROWS * GRAM_T; idx += NT) {
            const int c = idx / GRAM_ROWS, rr = idx - c * GRAM_ROWS;
            const int row = rb + rr;
            As[rr][c] = (row < row1 && ti + c < t1) ? A[(size_t)(ti + c) * n + row] : 0.0;
            Bs[rr][c] = (row < row1 && tj + c < t2) ? B[(size_t)(tj + c) * n + row] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < GRAM_ROWS; ++rr) {
            const double a0 = As[rr][ty * 2], a1 = As[rr][ty * 2 + 1];
            const double b0 = Bs[rr][tx * 2], b1 = Bs[rr][tx * 2 + 1];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    double* pc = part + (size_t)blockIdx.x * t1 * t2;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            const int i = ti + ty * 2 + u, j = tj + tx * 2 + v;
            if (i < t1 && j < t2) pc[(size_t)j * t1 + i] = acc[u][v];
        }
}

// out[k] = sum over chunks c of part[c * len + k].  A block handles 16 consecutive outputs with
// 16 thread groups; group g sums chunks g, g + 16, ... (8 loads in flight), then the 16 group
// sums are added in group order (a fixed order: deterministic).
constexpr int SC_OUT = 16;
__global__ void __launch_bounds__(NT) k_sum_chunks(int nchunks, int len, const double* __restrict__ part,
                                                   double* __restrict__ out) {
    __shared__ double gs[NT / SC_OUT][SC_OUT];
    const int o = threadIdx.x % SC_OUT, g = threadIdx.x / SC_OUT;
    const int k = blockIdx.x * SC_OUT + o;
    constexpr int NG = NT / SC_OUT;
    double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (k < len) {
        int c = g;
        for (; c + 7 * NG < nchunks; c += 8 * NG) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a8[u] += part[(size_t)(c + u * NG) * len + k];
        }
        for (int u = 0; c < nchunks; c += NG, ++u) a8[u & 7] += part[(size_t)c * len + k];
    }
    gs[g][o] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
    __syncthreads();
    if (g == 0 && k < len) {
        double sum = 0.0;
        for (int q = 0; q < NG; ++q) sum += gs[q][o];
        out[k] = sum;
    }
}

int gram_chunks(int n) {
    int c = (n + 255) / 256;
    return c < 1 ? 1 : (c > 512 ? 512 : c);
}

hipError_t launch_gram(int n, int t1, int t2, const double* A, const double* B, double* part, double* out,
                       hipStream_t stream) {
    return launch_gram_n(n, t1, t2, A, B, gram_chunks(n), part, out, stream);
}

hipError_t launch_gram_n(int n, int t1, int t2, const double* A, const double* B, int nch, double* part,
                         double* out, hipStream_t stream) {
    const int chunk_rows = (n + nch - 1) / nch;
    dim3 grid(nch, (t1 + GRAM_T - 1) / GRAM_T, (t2 + GRAM_T - 1) / GRAM_T);
    hipLaunchKernelGGL(k_gram, grid, dim3(NT), 0, stream, n, t1, t2, A, B, chunk_rows, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int len = t1 * t2;
    hipLaunchKernelGGL(k_sum_chunks, dim3((len + SC_OUT - 1) / SC_OUT), dim3(NT), 0, stream, nch, len, part, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Out = A X (tall x small)
// A: n x t (ld n); X: t x k (ld ldx); Out: n x k (ld n).  A dense contraction, so it runs on the
// FP64 matrix cores (16 x 16 x 4 products): each wave owns 16 rows of Out and up to 128 of its
// columns (8 accumulator tiles), reads its 16 rows of A once per 128 columns, and takes the
// rows of X from LDS, staged 32 at a time.  Lane l holds A[row0 + l % 16][t0 + l / 16] and
// X[t0 + l / 16][c + l % 16]; element r of its accumulator tile is Out[row0 + l / 16 + 4 r][c + l % 16],
// r = 0..3 (the FP64 output layout, checked on the device).
constexpr int GM_COLS = 128;
constexpr int GM_TROWS = 32;
constexpr int GT_TMAX = 256;
typedef double gm_acc __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(NT) k_gemm_tall(int n, int t, int k, const double* __restrict__ A,
                                                  const double* __restrict__ X, int ldx, double* __restrict__ Out) {
    __shared__ double Xs[GM_TROWS][GM_COLS + 2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int row0 = (blockIdx.x * NWAVE + wave) * 16;
    const int arow = row0 + li;
    for (int c0 = 0; c0 < k; c0 += GM_COLS) {
        const int kc = min(GM_COLS, k - c0);
        const int ntile = (kc + 15) / 16;
        gm_acc acc[GM_COLS / 16];
#pragma unroll
        for (int q = 0; q < GM_COLS / 16; ++q) acc[q] = gm_acc{0.0, 0.0, 0.0, 0.0};
        for (int t0 = 0; t0 < t; t0 += GM_TROWS) {
            const int tr = min(GM_TROWS, t - t0);
            // this chunk's 32 rows of A for the wave's 16 rows (8 loads in flight per lane)
            double av[GM_TROWS / 4];
#pragma unroll
            for (int u = 0; u < GM_TROWS / 4; ++u) {
                const int tt = 4 * u + lk;
                av[u] = (tt < tr && arow < n) ? A[(size_t)(t0 + tt) * n + arow] : 0.0;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < GM_TROWS * GM_COLS; idx += NT) {
                const int c = idx / GM_TROWS, r = idx - c * GM_TROWS;
                Xs[r][c] = (r < tr && c < kc) ? X[(size_t)(c0 + c) * ldx + t0 + r] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < GM_TROWS / 4; ++u) {
                if (4 * u >= tr) break;
#pragma unroll
                for (int q = 0; q < GM_COLS / 16; ++q)
                    if (q < ntile)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], Xs[4 * u + lk][16 * q + li], acc[q], 0, 0,
                                                                       0);
            }
        }
#pragma unroll
        for (int q = 0; q < GM_COLS / 16; ++q) {
            const int col = c0 + 16 * q + li;
            if (q >= ntile || col >= k) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + lk + 4 * r;
                if (row < n) Out[(size_t)col * n + row] = acc[q][r];
            }
        }
    }
}

hipError_t launch_gemm_tall(int n, int t, int k, const double* A, const double* X, int ldx, double* Out,
                            hipStream_t stream) {
    if (t > GT_TMAX) return hipErrorInvalidValue;
    if (n <= 0 || k <= 0) return hipSuccess;
    const int rows_per_block = 16 * NWAVE;
    hipLaunchKernelGGL(k_gemm_tall, dim3((n + rows_per_block - 1) / rows_per_block), dim3(NT), 0, stream, n, t, k, A,
                       X, ldx, Out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ small dense (one workgroup)
constexpr int SD_NT = 512;

// Cholesky with column drop on a t x t Gram matrix Gm (column-major, ld t), right-looking in
// column order: the pivot of column j is its diagonal after the updates from the kept
// columns before it (= squared norm of column j after projection); j is dropped when
// pivot_j <= tol^2 Gm_jj.  Writes Xinv (t x tk, ld ldx) with W Xinv = orthonormal basis of
// the kept columns (rows of dropped columns zero) and *tk_out = tk.  A (t*t) is the working
// matrix; with XL the inverse factor is solved into X (t*t, in LDS) and then copied to Xinv,
// so that the solve's accesses stay on chip.  Gm's diagonal is staged in LDS once: the serial
// pivot test of every column reads it.  Instantiated with A and X either in LDS or in global
// memory, never a pointer that may be either (which would make every access a flat one).
template <bool XL, typename AP>
__device__ __forceinline__ void chol_drop(int t, const double* __restrict__ Gm, double tol, AP A, double* X,
                                          int* tk_out, double* Xinv, int ldx) {
    constexpr int NU = 4;   // rows per lane in the inverse (t <= 256)
    constexpr int GC = 4;   // columns of the inverse one wave solves together
    __shared__ int s_tk, s_keep;
    __shared__ double s_d;
    __shared__ int kept[256];
    __shared__ double gdiag[256], rdiag[256];
    const int wv = (int)(threadIdx.x >> 6), ln = (int)(threadIdx.x & 63), nwv = (int)(blockDim.x >> 6);
    if (threadIdx.x == 0) s_tk = 0;
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) A[idx] = Gm[idx];
    for (int j = threadIdx.x; j < t; j += blockDim.x) gdiag[j] = Gm[(size_t)j * t + j];
    __syncthreads();
    for (int j = 0; j < t; ++j) {
        if (threadIdx.x == 0) {
            const double piv = A[(size_t)j * t + j];
            const double gjj = gdiag[j];
            s_keep = (gjj > 0.0 && piv > tol * tol * gjj) ? 1 : 0;
            s_d = s_keep ? sqrt(piv) : 1.0;
            if (s_keep) {
                kept[s_tk] = j;
                s_tk = s_tk + 1;
                A[(size_t)j * t + j] = s_d;
            }
        }
        __syncthreads();
        if (!s_keep) continue;
        const double d = s_d;
        // row j of R: R[j][i] = A[j][i] / d for i > j (A symmetric: use column j)
        for (int i = j + 1 + threadIdx.x; i < t; i += blockDim.x) A[(size_t)i * t + j] /= d;
        __syncthreads();
        // trailing update, one column per wave at a time (no index division)
        const int m = t - j - 1;
        for (int kk = wv; kk < m; kk += nwv) {
            const int k = j + 1 + kk;
            const double akj = A[(size_t)k * t + j];
            for (int ii = ln; ii < m; ii += 64) {
                const int i = j + 1 + ii;
                A[(size_t)k * t + i] -= A[(size_t)i * t + j] * akj;
            }
        }
        __syncthreads();
    }
    const int tk = s_tk;
    double* xb = XL ? X : Xinv;
    const int ldb = XL ? t : ldx;
    for (int idx = threadIdx.x; idx < t * tk; idx += blockDim.x) xb[(size_t)(idx / t) * ldb + idx % t] = 0.0;
    for (int k = threadIdx.x; k < tk; k += blockDim.x) rdiag[k] = 1.0 / A[(size_t)kept[k] * t + kept[k]];
    __syncthreads();
    // R^{-1} (kept rows and columns; R[k][l] = A[kept_l * t + kept_k] for k < l): a wave solves GC
    // columns together, sweeping l downwards; lane ln holds rows ln + 64 u of the right-hand
    // sides, and at step l every lane updates its rows k < l with x_l = b_l / R_ll.
    int kk_row[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = ln + 64 * u;
        kk_row[u] = k < tk ? kept[k] : 0;
    }
    for (int g0 = wv * GC; g0 < tk; g0 += nwv * GC) {
        double b[GC][NU];
#pragma unroll
        for (int c = 0; c < GC; ++c)
#pragma unroll
            for (int u = 0; u < NU; ++u) b[c][u] = (ln + 64 * u == g0 + c) ? 1.0 : 0.0;
        const int top = min(g0 + GC, tk) - 1;
        for (int l = top; l >= 0; --l) {
            const int kl = kept[l];
            const double rl = rdiag[l];
            const int ul = l >> 6, lanel = l & 63;
            double x[GC];
#pragma unroll
            for (int c = 0; c < GC; ++c) {
                double bl = 0.0;
#pragma unroll
                for (int u = 0; u < NU; ++u)
                    if (u == ul) bl = b[c][u];
                const long long bb = __double_as_longlong(bl);
                const int lo = __builtin_amdgcn_readlane((int)bb, lanel);
                const int hi = __builtin_amdgcn_readlane((int)(bb >> 32), lanel);
                x[c] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo) * rl;
            }
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = ln + 64 * u;
                if (k < l) {
                    const double rkl = A[(size_t)kl * t + kk_row[u]];
#pragma unroll
                    for (int c = 0; c < GC; ++c) b[c][u] -= rkl * x[c];
                }
            }
            if (ln < GC && g0 + ln < tk && l <= g0 + ln) {
                double xv = 0.0;
#pragma unroll
                for (int c = 0; c < GC; ++c)
                    if (c == ln) xv = x[c];
                xb[(size_t)(g0 + ln) * ldb + kl] = xv;
            }
        }
    }
    __syncthreads();
    if constexpr (XL) {
        for (int idx = threadIdx.x; idx < t * tk; idx += blockDim.x) Xinv[(size_t)(idx / t) * ldx + idx % t] = X[idx];
        __syncthreads();
    }
    if (threadIdx.x == 0) *tk_out = tk;
}

// The working matrix lives in LDS when it fits (lds >= 1), else in the global scratch R; with
// lds = 2 the inverse factor is solved in LDS too.
__global__ void __launch_bounds__(SD_NT) k_chol_drop(int t, const double* Gm, double tol, double* R, int* tk_out,
                                                     double* Xinv, int ldx, int lds) {
    extern __shared__ double dyn_lds[];
    if (lds == 2) chol_drop<true>(t, Gm, tol, dyn_lds, dyn_lds + (size_t)t * t, tk_out, Xinv, ldx);
    else if (lds == 1) chol_drop<false>(t, Gm, tol, dyn_lds, nullptr, tk_out, Xinv, ldx);
    else chol_drop<false>(t, Gm, tol, gbl(R), nullptr, tk_out, Xinv, ldx);
}

// ------------------------------------------------------------------ symmetric eigensolver
constexpr int EIG_MAX = 256;        // largest order
constexpr int KC = 32;              // rows of G M^{-1} staged per chunk of S^T S

// 1 / a from the hardware reciprocal refined by one Newton step (relative error ~1e-16); used
// where a correctly rounded quotient is not needed (Sturm counts, inverse-iteration solves).
__device__ __forceinline__ double fast_rcp(double a) {
    const double r = __builtin_amdgcn_rcp(a);
    return r * fma(-a, r, 2.0);
}

// Block-wide sum (SD_NT threads); the result is valid in every thread.
__device__ __forceinline__ double sd_sum(double v, double* red) {
    v = wave_sum(v);
    if (SD_NT == 64) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < SD_NT / 64; ++k) s += red[k];
    return s;
}

// Householder tridiagonalisation of a symmetric m x m matrix A (row-major, full storage):
// A <- H_{m-3} ... H_0 A H_0 ... H_{m-3} with H_k = I - tau_k v_k v_k^T acting on indices
// k+1 .. m-1 and mapping column k below the diagonal to a multiple of e_1.  Output: the
// diagonal d and subdiagonal e (e[i] couples i and i+1, e[m-1] = 0); v_k is kept in column k
// of A below the diagonal and tau_k in tau.
__device__ void tridiag(int m, double* A, double* d, double* e, double* tau, double* vv, double* pw, double* red) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int k = 0; k + 2 < m; ++k) {
        const int n2 = m - k - 1;
        double sg = 0.0;
        for (int i = tid; i < n2; i += bs) {
            const double xi = A[(size_t)(k + 1 + i) * m + k];
            vv[i] = xi;
            if (i >= 1) sg += xi * xi;
        }
        const double sig = sd_sum(sg, red);
        const double x0 = A[(size_t)(k + 1) * m + k];
        const double nrm = sqrt(x0 * x0 + sig);
        // v = x - alpha e_1, alpha = -sign(x0) |x|:  v^T v = 2 |x| (|x| + |x0|), tau = 2 / v^T v
        const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0.0 ? -nrm : nrm);
        const double t = nrm == 0.0 ? 0.0 : 1.0 / (nrm * (nrm + fabs(x0)));
        __syncthreads();
        if (tid == 0) {
            vv[0] = x0 - alpha;
            e[k] = alpha;
            tau[k] = t;
        }
        __syncthreads();
        if (t != 0.0) {
            // p = tau A' v, K = tau/2 p.v, w = p - K v, A' -= v w^T + w v^T
            double pv = 0.0;
            for (int i = tid; i < n2; i += bs) {
                // row i of A' read as column i (A' symmetric): consecutive threads, consecutive banks
                const double* col = A + (size_t)(k + 1) * m + (k + 1 + i);
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int j = 0;
                for (; j + 3 < n2; j += 4) {
                    a0 += col[(size_t)j * m] * vv[j];
                    a1 += col[(size_t)(j + 1) * m] * vv[j + 1];
                    a2 += col[(size_t)(j + 2) * m] * vv[j + 2];
                    a3 += col[(size_t)(j + 3) * m] * vv[j + 3];
                }
                for (; j < n2; ++j) a0 += col[(size_t)j * m] * vv[j];
                const double pi = t * ((a0 + a1) + (a2 + a3));
                pw[i] = pi;
                pv += pi * vv[i];
            }
            const double K = 0.5 * t * sd_sum(pv, red);
            __syncthreads();
            for (int i = tid; i < n2; i += bs) pw[i] -= K * vv[i];
            __syncthreads();
            for (int idx = tid; idx < n2 * n2; idx += bs) {
                const int r = idx / n2, c = idx - r * n2;
                A[(size_t)(k + 1 + r) * m + (k + 1 + c)] -= vv[r] * pw[c] + pw[r] * vv[c];
            }
        }
        for (int i = tid; i < n2; i += bs) A[(size_t)(k + 1 + i) * m + k] = vv[i];
        __syncthreads();
    }
    for (int j = tid; j < m; j += bs) d[j] = A[(size_t)j * m + j];
    if (tid == 0) {
        if (m >= 2) e[m - 2] = A[(size_t)(m - 1) * m + (m - 2)];
        e[m - 1] = 0.0;
    }
    __syncthreads();
}

// Eigenvalues of the symmetric tridiagonal (d, e), e2[i] = e[i]^2, by multisection on Sturm
// counts (the number of negative pivots of the LDL^T factorisation of T - x I equals the
// number of eigenvalues below x): lam[k] = k-th smallest.  A group of G lanes of one wave
// (G a power of two, as many as the block has for m eigenvalues) brackets one eigenvalue: per
// round each lane evaluates the count at one of G equally spaced interior points, and the first
// point whose count exceeds k (a ballot over the group) gives the next bracket, G + 1 times
// narrower.  Rounds end when the bracket's midpoint is no longer strictly inside (adjacent
// doubles).  The bracket invariant count(lo) <= k < count(hi) holds whatever the rounding of
// the counts: the new ends are two neighbouring points on either side of the first crossing.
__device__ void tri_bisect(int m, const double* d, const double* e2, double glo, double ghi, double pivmin,
                           double* lam) {
    int G = 64;
    while (G > 1 && G * m > (int)blockDim.x) G >>= 1;
    const int lane = (int)(threadIdx.x & 63);
    const int gi = lane & (G - 1), gbase = lane - gi;
    const unsigned long long gmask = G == 64 ? ~0ull : (((1ull << G) - 1) << gbase);
    const double inv = 1.0 / (double)(G + 1);
    const int ngrp = (int)blockDim.x / G;
    for (int k = (int)threadIdx.x / G; k < m; k += ngrp) {   // uniform within a group
        double lo = glo, hi = ghi;
        for (int round = 0; round < 96; ++round) {
            const double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;   // adjacent doubles: converged
            const double x = lo + (hi - lo) * ((double)(gi + 1) * inv);
            int cnt = 0;
            double q = d[0] - x;
            for (int i = 0;;) {
                if (fabs(q) < pivmin) q = -pivmin;
                cnt += q < 0.0;
                if (++i >= m) break;
                q = (d[i] - x) - e2[i - 1] * fast_rcp(q);
            }
            const unsigned long long above = __ballot(cnt > k) & gmask;
            const int first = above ? (int)__builtin_ctzll(above) - gbase : G;
            const double xl = first == 0 ? lo : lo + (hi - lo) * ((double)first * inv);
            const double xh = first == G ? hi : lo + (hi - lo) * ((double)(first + 1) * inv);
            lo = xl;
            hi = xh;
        }
        if (gi == 0) lam[k] = 0.5 * (lo + hi);
    }
}

// One eigenvector of the tridiagonal (d, e) for the eigenvalue approximation lam by inverse
// iteration: (T - lam I) = P L U with partial pivoting (U with two superdiagonals), three
// solves from a fixed start vector, each followed by Gram-Schmidt against the `nprev`
// vectors prev (earlier members of a cluster of close eigenvalues) and scaling.  Vectors and
// factors are strided by `ld` (element i at [i * ld]) so that the threads of a block, each
// with its own column, access consecutive LDS words.  z: the unit-norm result; w: 4 strided
// arrays (u0^{-1}, u1, u2, multipliers) at w + k * wst; piv: pivot flags (stride ld).
__device__ void tri_invit(int m, const double* d, const double* e, double lam, double tiny, const double* prev,
                          int nprev, double* z, double* w, size_t wst, unsigned char* piv, int ld, int seed) {
    double* iu0 = w;
    double* u1 = w + wst;
    double* u2 = w + 2 * wst;
    double* ml = w + 3 * wst;
    double a = d[0] - lam, c = m > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < m; ++i) {
        const double b = e[i], an = d[i + 1] - lam, cn = i + 2 < m ? e[i + 1] : 0.0;
        const size_t o = (size_t)i * ld;
        if (fabs(a) >= fabs(b)) {
            const double aa = a != 0.0 ? a : tiny;
            const double ia = fast_rcp(aa);
            iu0[o] = ia;
            u1[o] = c;
            u2[o] = 0.0;
            ml[o] = b * ia;
            piv[o] = 0;
            a = an - ml[o] * c;
            c = cn;
        } else {
            const double mli = a * fast_rcp(b);
            iu0[o] = fast_rcp(b);
            u1[o] = an;
            u2[o] = cn;
            ml[o] = mli;
            piv[o] = 1;
            a = c - mli * an;
            c = -mli * cn;
        }
    }
    iu0[(size_t)(m - 1) * ld] = fast_rcp(a != 0.0 ? a : tiny);
    for (int i = 0; i < m; ++i) z[(size_t)i * ld] = 1.0 + 0.25 * (double)(((i + 1) * 7919 + seed * 104729) % 101) / 101.0;
    for (int it = 0; it < 3; ++it) {
        double zi = z[0];
        for (int i = 0; i + 1 < m; ++i) {   // y = L^{-1} P z  (zi carries the running element i)
            double zn = z[(size_t)(i + 1) * ld];
            if (piv[(size_t)i * ld]) {
                const double tmp = zi;
                zi = zn;
                zn = tmp;
            }
            z[(size_t)i * ld] = zi;
            zi = zn - ml[(size_t)i * ld] * zi;
        }
        z[(size_t)(m - 1) * ld] = zi;
        double x1 = 0.0, x2 = 0.0;   // x[i + 1], x[i + 2]
        for (int i = m - 1; i >= 0; --i) {   // U x = y
            const size_t o = (size_t)i * ld;
            const double v = (z[o] - u1[o] * x1 - u2[o] * x2) * iu0[o];
            z[o] = v;
            x2 = x1;
            x1 = v;
        }
        for (int j = 0; j < nprev; ++j) {   // orthogonalise within the cluster
            const double* pj = prev + j;
            double dt = 0.0;
            for (int i = 0; i < m; ++i) dt += pj[(size_t)i * ld] * z[(size_t)i * ld];
            for (int i = 0; i < m; ++i) z[(size_t)i * ld] -= dt * pj[(size_t)i * ld];
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += z[(size_t)i * ld] * z[(size_t)i * ld];
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = 0; i < m; ++i) z[(size_t)i * ld] *= inv;
    }
}

// Symmetric eigenproblem of the m x m matrix A (row-major, destroyed): all eigenvalues in
// ascending order to lam, the eigenvectors of eigenvalues lo .. hi-1 to the columns of Z
// (Z[(k - lo) * m + i] = component i).  Householder tridiagonalisation (in LDS when m^2
// doubles fit), eigenvalues by multisection (tri_bisect), vectors by inverse iteration
// (eigenvalues closer than 1e-7 of the spectrum's width are treated as a cluster, their vectors
// computed in sequence and orthogonalised), and the reflectors applied to the few vectors
// wanted, one wave per vector.
// scr: (hi - lo) * 4 m + m doubles of scratch.
__device__ void eig_range(int m, double* A, int lo, int hi, double* lam, double* Z, double* scr, int ldsd) {
    __shared__ double d[EIG_MAX], e[EIG_MAX], e2[EIG_MAX], tau[EIG_MAX], vv[EIG_MAX], pw[EIG_MAX],
        red[SD_NT / 64];
    __shared__ double s_lo, s_hi, s_piv, s_gap;
    __shared__ int cstart[EIG_MAX];
    extern __shared__ double dyn_lds[];
    const bool in_lds = m * m <= ldsd;
    double* LA = in_lds ? dyn_lds : A;
    if (in_lds) {
        for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) LA[idx] = A[idx];
        __syncthreads();
    }
    tridiag(m, LA, d, e, tau, vv, pw, red);
    for (int i = threadIdx.x; i < m; i += blockDim.x) e2[i] = e[i] * e[i];
    if (threadIdx.x == 0) {   // Gershgorin interval
        double gl = d[0], gh = d[0], me2 = 0.0;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
            gl = fmin(gl, d[i] - r);
            gh = fmax(gh, d[i] + r);
            if (i + 1 < m) me2 = fmax(me2, e[i] * e[i]);
        }
        const double w = fmax(gh - gl, fmax(fabs(gl), fabs(gh)));
        s_lo = gl - 1e-14 * w - 1e-300;
        s_hi = gh + 1e-14 * w + 1e-300;
        s_piv = 2.3e-308 * fmax(1.0, me2);
        s_gap = 1e-7 * w;
    }
    __syncthreads();
    tri_bisect(m, d, e2, s_lo, s_hi, s_piv, lam);
    __syncthreads();
    const int nw = hi - lo;
    if (threadIdx.x == 0) {   // clusters among the wanted eigenvalues
        for (int k = 0; k < nw; ++k) cstart[k] = (k == 0 || lam[lo + k] - lam[lo + k - 1] > s_gap) ? 1 : 0;
    }
    __syncthreads();
    const double tiny = 2.3e-16 * fmax(fabs(s_lo), fabs(s_hi));
    // vectors and inverse-iteration factors: in LDS after LA when they fit (element i of
    // vector k at zs[i * nw + k]), else in the global scratch
    const size_t need = (size_t)5 * m * nw + ((size_t)m * nw + 7) / 8;
    const bool v_lds = in_lds && (size_t)m * m + need <= (size_t)ldsd;
    double* zs = v_lds ? dyn_lds + (size_t)m * m : scr;
    double* ws = zs + (size_t)m * nw;
    unsigned char* pv = reinterpret_cast<unsigned char*>(ws + (size_t)4 * m * nw);
    for (int k = threadIdx.x; k < nw; k += blockDim.x) {
        if (!cstart[k]) continue;
        int len = 1;
        while (k + len < nw && !cstart[k + len]) ++len;
        for (int j = 0; j < len; ++j)
            tri_invit(m, d, e, lam[lo + k + j], tiny, zs + k, j, zs + k + j, ws + k + j, (size_t)m * nw,
                      pv + k + j, nw, lo + k + j);
    }
    __syncthreads();
    // back to the original basis: z <- H_0 H_1 ... H_{m-3} z, one wave per vector (the lanes
    // split each reflection's dot product and update; a block-scope fence orders a lane's
    // update before another lane's read in the next reflection)
    {
        const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6), nwave = (int)(blockDim.x >> 6);
        for (int k = wave; k < nw; k += nwave) {
            double* z = zs + k;
            for (int r = m - 3; r >= 0; --r) {
                const double tr = tau[r];
                if (tr == 0.0) continue;
                const double* hv = LA + (size_t)(r + 1) * m + r;   // v_r[i] at hv[i * m]
                const int len = m - r - 1;
                double a = 0.0;
                for (int i = lane; i < len; i += 64) a += hv[(size_t)i * m] * z[(size_t)(r + 1 + i) * nw];
                const double dt = tr * wave_sum(a);
                for (int i = lane; i < len; i += 64) z[(size_t)(r + 1 + i) * nw] -= dt * hv[(size_t)i * m];
                __threadfence_block();
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nw * m; idx += blockDim.x) {
        const int k = idx / m, i = idx - k * m;
        Z[(size_t)k * m + i] = zs[(size_t)i * nw + k];
    }
    __syncthreads();
}

// Cholesky M = L L^T in place (lower, column-major ld t).  Returns false if not SPD.
// (Instantiated for L in LDS or in global memory, never a pointer that may be either.)
template <typename PL>
__device__ __forceinline__ bool chol_inplace(int t, PL L) {
    __shared__ int s_ok;
    const int wv = (int)(threadIdx.x >> 6), ln = (int)(threadIdx.x & 63), nwv = (int)(blockDim.x >> 6);
    if (threadIdx.x == 0) s_ok = 1;
    __syncthreads();
    for (int j = 0; j < t; ++j) {
        if (threadIdx.x == 0) {
            const double d = L[(size_t)j * t + j];
            if (!(d > 0.0)) s_ok = 0;
            L[(size_t)j * t + j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        if (!s_ok) return false;
        const double dj = L[(size_t)j * t + j];
        for (int i = j + 1 + threadIdx.x; i < t; i += blockDim.x) L[(size_t)j * t + i] /= dj;
        __syncthreads();
        // trailing update: L[i][k] -= L[i][j] L[k][j], j < k <= i; one column k per wave
        for (int k = j + 1 + wv; k < t; k += nwv) {
            const double lkj = L[(size_t)j * t + k];
            for (int i = k + ln; i < t; i += 64) L[(size_t)k * t + i] -= L[(size_t)j * t + i] * lkj;
        }
        __syncthreads();
    }
    return true;
}

// One wave's group of GC columns of X through L y = b, then L^T x = y (L lower, element (i, j)
// at LL[j * ld + i]).  Lane l holds rows l + 64 u of the group in registers; at step j every
// lane updates its rows with x_j, read from the lane that owns row j (readlane), scaled by the
// reciprocal diagonal.  No barrier: the columns and their registers are the wave's own.
template <int GC, typename PL>
__device__ __forceinline__ void solve_group(int t, PL LL, int ld, const double* rdg, double* X, int c0, int gn,
                                            size_t ldc, size_t incx) {
    constexpr int NU = EIG_MAX / 64;
    const int lane = (int)(threadIdx.x & 63);
    const int nu = (t + 63) >> 6;
    double x[GC][NU];
#pragma unroll
    for (int cc = 0; cc < GC; ++cc)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int r = lane + 64 * u;
            x[cc][u] = (cc < gn && r < t) ? X[(size_t)(c0 + cc) * ldc + (size_t)r * incx] : 0.0;
        }
    auto bcast = [&](int row, double (&out)[GC]) {
        const int ur = row >> 6, lr = row & 63;
#pragma unroll
        for (int cc = 0; cc < GC; ++cc) {
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < NU; ++u)
                if (u == ur) v = x[cc][u];
            const long long b = __double_as_longlong(v);
            const int lo = __builtin_amdgcn_readlane((int)b, lr);
            const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lr);
            out[cc] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo) * rdg[row];
        }
    };
    auto settle = [&](int row, const double (&val)[GC]) {   // row takes its solved value
        const int ur = row >> 6, lr = row & 63;
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (u == ur && lane == lr) {
#pragma unroll
                for (int cc = 0; cc < GC; ++cc) x[cc][u] = val[cc];
            }
    };
    for (int jj = 0; jj < t; ++jj) {   // L y = b, column jj of L
        double y[GC];
        bcast(jj, y);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int r = lane + 64 * u;
            if (u < nu && r > jj && r < t) {
                const double l = LL[(size_t)jj * ld + r];
#pragma unroll
                for (int cc = 0; cc < GC; ++cc) x[cc][u] -= l * y[cc];
            }
        }
        settle(jj, y);
    }
    for (int ii = t - 1; ii >= 0; --ii) {   // L^T x = y, row ii of L
        double z[GC];
        bcast(ii, z);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int r = lane + 64 * u;
            if (u < nu && r < ii) {
                const double l = LL[(size_t)r * ld + ii];
#pragma unroll
                for (int cc = 0; cc < GC; ++cc) x[cc][u] -= l * z[cc];
            }
        }
        settle(ii, z);
    }
#pragma unroll
    for (int cc = 0; cc < GC; ++cc)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int r = lane + 64 * u;
            if (cc < gn && r < t) X[(size_t)(c0 + cc) * ldc + (size_t)r * incx] = x[cc][u];
        }
}

template <typename PL>
__device__ __forceinline__ void solve_cols_waves(int t, PL LL, int ld, const double* rdg, double* X, int ncols,
                                                 size_t ldc, size_t incx) {
    const int wave = (int)(threadIdx.x >> 6), nwave = (int)(blockDim.x >> 6);
    const int want = (ncols + nwave - 1) / nwave;   // columns per wave in one pass, at most 8
    const int per = want <= 1 ? 1 : (want <= 2 ? 2 : (want <= 4 ? 4 : 8));
    for (int c0 = wave * per; c0 < ncols; c0 += nwave * per) {
        const int gn = ncols - c0 < per ? ncols - c0 : per;
        if (per == 1) solve_group<1>(t, LL, ld, rdg, X, c0, gn, ldc, incx);
        else if (per == 2) solve_group<2>(t, LL, ld, rdg, X, c0, gn, ldc, incx);
        else if (per == 4) solve_group<4>(t, LL, ld, rdg, X, c0, gn, ldc, incx);
        else solve_group<8>(t, LL, ld, rdg, X, c0, gn, ldc, incx);
    }
}

// X[:, c] <- M^{-1} X[:, c], c < ncols, with M = L L^T (L lower, column-major ld t, t <= 256);
// column c starts at X + c * ldc with element stride incx.  L is staged in LDS when it fits,
// with an odd leading dimension so that the backward sweep's row reads (stride ld) spread over
// the banks.  The columns are dealt to the waves in groups of 1, 2, 4 or 8 (solve_group).
__device__ void solve_cols(int t, const double* L, double* X, int ncols, size_t ldc, size_t incx, int ldsd) {
    extern __shared__ double dyn_lds[];
    __shared__ double rdg[EIG_MAX];   // reciprocal diagonal of L
    const int ldl = t | 1;
    const bool l_in = ldl * t <= ldsd;
    __syncthreads();   // earlier users of the dynamic LDS are done
    if (l_in)
        for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
            const int jc = idx / t, ir = idx - jc * t;
            dyn_lds[(size_t)jc * ldl + ir] = L[idx];
        }
    for (int i = threadIdx.x; i < t; i += blockDim.x) rdg[i] = 1.0 / L[(size_t)i * t + i];
    __syncthreads();
    if (l_in) solve_cols_waves(t, (const double*)dyn_lds, ldl, rdg, X, ncols, ldc, incx);
    else solve_cols_waves(t, gbl(L), t, rdg, X, ncols, ldc, incx);
    __syncthreads();
}

// Projected GSVD of (G, M) (p x t and t x t) and RGen selection of s_eff = min(s, t)
// (`size`: the largest, RGen-L; with p >= t also the smallest or both ends, RGen-S / RGen-M)
// columns.  Output: Xs (t x s_eff, unit columns), VHs (t x s_eff, zero for filled slots),
// mu (s_eff), info = {s_eff, rank_G, status}.  Scratch: sc (gsvd_scratch_doubles).
// Route: Cholesky M = L L^T;  S = G M^{-1};
//   p >= t: eigen of S^T S = V_H diag(mu^2) V_H^T; right vectors X ~ M^{-1} V_H;
//   p <  t: eigen of S S^T (p x p) gives mu and V_H = S^T u / mu; null(G) from a Householder
//           QR of the rank_G columns G^T u_k (u_k the eigenvectors of G G^T with non-zero
//           eigenvalues) = Q R: the remaining slots take the smallest Ritz pairs of N^T M N with
//           N = Q[:, rank_G:], formed as the trailing block of Q^T M Q (Ritz-S).
__global__ void __launch_bounds__(SD_NT) k_gsvd_select(int t, int p, int s, int size, const double* __restrict__ Min,
                                                       const double* __restrict__ G, double* sc, double* Xs,
                                                       double* VHs, double* mu, int* info, int ldsd) {
    extern __shared__ double dyn_lds[];
    __shared__ int s_rank;
    __shared__ double s_beta[EIG_MAX];   // Householder factors of the QR of G^T (p < t <= EIG_MAX)
    __shared__ double red[SD_NT / 64];
    __shared__ double vv[EIG_MAX], pw[EIG_MAX];
    const int s_eff = s < t ? s : t;
    const size_t T2 = (size_t)t * t, P2 = (size_t)p * p, PT = (size_t)p * t, KM = T2 > P2 ? T2 : P2;
    double* L = sc;                 // t*t   Cholesky factor of sym(M)
    double* S = L + T2;             // p*t   G M^{-1}, column-major ld p
    double* K = S + PT;             // S^T S (t*t) | S S^T (p*p)
    double* Vv = K + KM;            // eigenvectors of K
    double* GG = Vv + KM;           // p*p   G G^T
    double* GV = GG + P2;           // p*p
    double* Hv = GV + P2;           // t*p   Householder vectors of G^T
    double* Ms = Hv + PT;           // t*t   sym(M), then Q^T M Q
    double* BV = Ms + T2;           // (t-p)^2 eigenvectors of N^T M N
    double* lamv = BV + T2;         // eigenvalues (t + p)
    double* esc = lamv + t + p;     // eigensolver scratch: 5 t^2 + t
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
        const int j = idx / t, i = idx - j * t;
        const double v = 0.5 * (Min[(size_t)j * t + i] + Min[(size_t)i * t + j]);
        L[idx] = v;
        Ms[idx] = v;
    }
    __syncthreads();
    {
        const bool in_lds = (int)T2 <= ldsd;
        if (in_lds) {
            for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) dyn_lds[idx] = L[idx];
            __syncthreads();
        }
        const bool spd = in_lds ? chol_inplace(t, dyn_lds) : chol_inplace(t, gbl(L));
        if (in_lds) {
            for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) L[idx] = dyn_lds[idx];
            __syncthreads();
        }
        if (!spd) {
            if (threadIdx.x == 0) {
                info[0] = 0;
                info[1] = 0;
                info[2] = BL_E_INDEFINITE;
            }
            return;
        }
    }
    // p < t: S[k, :] = (M^{-1} G[k, :]^T)^T
    if (p < t) {
        for (int idx = threadIdx.x; idx < p * t; idx += blockDim.x) S[idx] = G[idx];
        __syncthreads();
        solve_cols(t, L, S, p, 1, p, ldsd);
    }
    int rankG;
    bool ok = true;
    if (p >= t) {
        // K = S^T S = M^{-1} (G^T G) M^{-1}.  G^T G from chunks of KC rows of G staged in LDS
        // (2 x 2 output blocks per thread, at most 8 blocks per thread per pass over G)
        constexpr int BPT = 8;
        const int tb = (t + 1) / 2, nblk = tb * tb;
        double* Sc = dyn_lds;   // KC x t, row k of the chunk at Sc[k * t]
        for (int g0 = 0; g0 < nblk; g0 += BPT * SD_NT) {
            double acc[BPT][4];
#pragma unroll
            for (int u = 0; u < BPT; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[u][q] = 0.0;
            for (int k0 = 0; k0 < p; k0 += KC) {
                const int kn = (p - k0) < KC ? (p - k0) : KC;
                __syncthreads();
                for (int idx = threadIdx.x; idx < kn * t; idx += blockDim.x) {
                    const int j = idx / kn, k = idx - j * kn;
                    Sc[k * t + j] = G[(size_t)j * p + k0 + k];
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < BPT; ++u) {
                    const int b = g0 + threadIdx.x + u * SD_NT;
                    if (b < nblk) {
                        const int bi = 2 * (b / tb), bj = 2 * (b % tb);
                        const bool i1 = bi + 1 < t, j1 = bj + 1 < t;
                        for (int k = 0; k < kn; ++k) {
                            const double* sr = Sc + k * t;
                            const double a0 = sr[bi], a1 = i1 ? sr[bi + 1] : 0.0;
                            const double b0 = sr[bj], b1 = j1 ? sr[bj + 1] : 0.0;
                            acc[u][0] += a0 * b0;
                            acc[u][1] += a0 * b1;
                            acc[u][2] += a1 * b0;
                            acc[u][3] += a1 * b1;
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < BPT; ++u) {
                const int b = g0 + threadIdx.x + u * SD_NT;
                if (b < nblk) {
                    const int bi = 2 * (b / tb), bj = 2 * (b % tb);
                    K[(size_t)bi * t + bj] = acc[u][0];
                    if (bj + 1 < t) K[(size_t)bi * t + bj + 1] = acc[u][1];
                    if (bi + 1 < t) K[(size_t)(bi + 1) * t + bj] = acc[u][2];
                    if (bi + 1 < t && bj + 1 < t) K[(size_t)(bi + 1) * t + bj + 1] = acc[u][3];
                }
            }
        }
        __syncthreads();
        solve_cols(t, L, K, t, t, 1, ldsd);   // Y = M^{-1} G^T G (columns of Y at K + c t)
        solve_cols(t, L, K, t, 1, t, ldsd);   // K = M^{-1} Y^T (columns of Y^T: rows of Y)
        for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {   // symmetrise
            const int i = idx / t, j = idx - i * t;
            if (i < j) {
                const double v = 0.5 * (K[idx] + K[(size_t)j * t + i]);
                K[idx] = v;
                K[(size_t)j * t + i] = v;
            }
        }
        __syncthreads();
        // all eigenvalues of K (ascending); vectors of the chosen ones: size 0 (L) the s_eff
        // largest (largest first), 1 (S) the s_eff smallest (ascending), 2 (M) ceil(s_eff / 2)
        // smallest then floor(s_eff / 2) largest
        const int lo_e = size == 0 ? t - s_eff : 0, hi_e = size == 1 ? s_eff : t;
        const int nlo = (s_eff + 1) / 2;
        eig_range(t, K, lo_e, hi_e, lamv, Vv, esc, ldsd);
        rankG = t;
        auto eig_of = [&](int c) {   // eigen index of output column c
            return size == 0 ? t - 1 - c : (size == 1 ? c : (c < nlo ? c : t - 1 - (c - nlo)));
        };
        for (int idx = threadIdx.x; idx < s_eff * t; idx += blockDim.x) {
            const int c = idx / t, i = idx - c * t;
            const double v = Vv[(size_t)(eig_of(c) - lo_e) * t + i];
            VHs[(size_t)c * t + i] = v;
            Xs[(size_t)c * t + i] = v;
        }
        for (int c = threadIdx.x; c < s_eff; c += blockDim.x) {
            const double lam = lamv[eig_of(c)];
            mu[c] = lam > 0.0 ? sqrt(lam) : 0.0;
        }
        __syncthreads();
        solve_cols(t, L, Xs, s_eff, t, 1, ldsd);
    } else {
        for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
            const int i = idx / p, j = idx - i * p;
            double v = 0.0, w = 0.0;
            for (int k = 0; k < t; ++k) {
                v += S[(size_t)k * p + i] * S[(size_t)k * p + j];
                w += G[(size_t)k * p + i] * G[(size_t)k * p + j];
            }
            K[idx] = v;
            GG[idx] = w;
        }
        __syncthreads();
        double* lamg = lamv + t;
        eig_range(p, GG, 0, p, lamg, GV, esc, ldsd);   // G G^T = U diag(sigma^2) U^T, ascending
        eig_range(p, K, 0, p, lamv, Vv, esc, ldsd);    // S S^T: all pairs, ascending
        if (threadIdx.x == 0) {
            const double mx2 = fmax(lamg[p - 1], 0.0);
            int r = 0;
            for (int i = 0; i < p; ++i)
                // singular values of G above 1e-6 of the largest: G G^T's rounding (about p eps
                // of its largest eigenvalue) stays far below the cutoff squared
                if (lamg[i] > 1e-12 * mx2) ++r;
            s_rank = r;
        }
        __syncthreads();
        rankG = s_rank;
        const int kg = s_eff < rankG ? s_eff : rankG;
        // v_H = S^T u / |S^T u| for the kg largest pairs (c-th largest: o = p - 1 - c), one
        // element per thread, then a block sum per column for its norm
        for (int c = threadIdx.x; c < kg; c += blockDim.x) {
            const double lam = lamv[p - 1 - c];
            mu[c] = lam > 0.0 ? sqrt(lam) : 0.0;
        }
        for (int idx = threadIdx.x; idx < kg * t; idx += blockDim.x) {
            const int c = idx / t, i = idx - c * t, o = p - 1 - c;
            double v = 0.0;
            for (int k = 0; k < p; ++k) v += S[(size_t)i * p + k] * Vv[(size_t)o * p + k];
            VHs[(size_t)c * t + i] = v;
        }
        __syncthreads();
        for (int c = 0; c < kg; ++c) {
            double part = 0.0;
            for (int i = threadIdx.x; i < t; i += blockDim.x) {
                const double v = VHs[(size_t)c * t + i];
                part += v * v;
            }
            const double nrm = sqrt(sd_sum(part, red));
            for (int i = threadIdx.x; i < t; i += blockDim.x) {
                const double v = VHs[(size_t)c * t + i] / nrm;
                VHs[(size_t)c * t + i] = v;
                Xs[(size_t)c * t + i] = v;
            }
        }
        __syncthreads();
        solve_cols(t, L, Xs, kg, t, 1, ldsd);
        const int nfill = s_eff - kg;
        if (nfill > 0) {
            // null(G) is the orthogonal complement of range(G^T) = span{G^T u_k}, u_k the
            // eigenvectors of G G^T with non-zero eigenvalues (rankG of them, mutually
            // orthogonal): a Householder QR of those rankG columns gives N = Q[:, rankG:],
            // also where G has fewer independent rows than p
            const int r = rankG, nn = t - r;
            for (int idx = threadIdx.x; idx < r * t; idx += blockDim.x) {
                const int j = idx / t, i = idx - j * t;
                const double* u = GV + (size_t)(p - 1 - j) * p;
                double v = 0.0;
                for (int k = 0; k < p; ++k) v += G[(size_t)i * p + k] * u[k];
                Hv[(size_t)j * t + i] = v;
            }
            __syncthreads();
            if (threadIdx.x == 0) {   // Householder QR of the t x r columns, reflectors in Hv
                for (int j = 0; j < r; ++j) {
                    double* v = Hv + (size_t)j * t;
                    double nrm = 0.0;
                    for (int i = j; i < t; ++i) nrm += v[i] * v[i];
                    nrm = sqrt(nrm);
                    const double alpha = v[j] >= 0.0 ? -nrm : nrm;
                    v[j] -= alpha;
                    double vn = 0.0;
                    for (int i = j; i < t; ++i) vn += v[i] * v[i];
                    const double beta = vn > 0.0 ? 2.0 / vn : 0.0;
                    s_beta[j] = beta;
                    for (int i = 0; i < j; ++i) v[i] = 0.0;
                    for (int jj = j + 1; jj < r; ++jj) {
                        double* u = Hv + (size_t)jj * t;
                        double d = 0.0;
                        for (int i = j; i < t; ++i) d += v[i] * u[i];
                        for (int i = j; i < t; ++i) u[i] -= beta * d * v[i];
                    }
                }
            }
            __syncthreads();
            // Q^T M Q = H_{r-1} ... H_0 M H_0 ... H_{r-1}; its trailing block is N^T M N
            {
                const bool in_lds = (int)T2 <= ldsd;
                double* MM = in_lds ? dyn_lds : Ms;   // row-major (M symmetric)
                if (in_lds) {
                    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) MM[idx] = Ms[idx];
                    __syncthreads();
                }
                const int tid = threadIdx.x, bs = blockDim.x;
                for (int j = 0; j < r; ++j) {
                    const double beta = s_beta[j];
                    if (beta == 0.0) continue;
                    for (int i = tid; i < t; i += bs) vv[i] = Hv[(size_t)j * t + i];
                    __syncthreads();
                    double pv = 0.0;
                    for (int i = tid; i < t; i += bs) {
                        const double* row = MM + (size_t)i * t;
                        double acc = 0.0;
                        for (int q = 0; q < t; ++q) acc += row[q] * vv[q];
                        const double pi = beta * acc;
                        pw[i] = pi;
                        pv += pi * vv[i];
                    }
                    const double Kc = 0.5 * beta * sd_sum(pv, red);
                    __syncthreads();
                    for (int i = tid; i < t; i += bs) pw[i] -= Kc * vv[i];
                    __syncthreads();
                    for (int idx = tid; idx < t * t; idx += bs) {
                        const int r = idx / t, c = idx - r * t;
                        MM[idx] -= vv[r] * pw[c] + pw[r] * vv[c];
                    }
                    __syncthreads();
                }
                // B = trailing nn x nn block, into K (row-major)
                for (int idx = threadIdx.x; idx < nn * nn; idx += blockDim.x) {
                    const int rr = idx / nn, c = idx - rr * nn;
                    K[idx] = MM[(size_t)(r + rr) * t + (r + c)];
                }
                __syncthreads();
            }
            eig_range(nn, K, 0, nfill, lamv, BV, esc, ldsd);   // the nfill smallest Ritz pairs
            // fill vectors x = N y = Q [0; y]: apply H_{r-1}, ..., H_0 to [0; y] (element-parallel;
            // the dot v_j . x_f of each reflection is one wave's sum, kept in pw[f])
            for (int f = threadIdx.x; f < nfill; f += blockDim.x) mu[kg + f] = 0.0;
            for (int idx = threadIdx.x; idx < nfill * t; idx += blockDim.x) {
                const int f = idx / t, i = idx - f * t;
                Xs[(size_t)(kg + f) * t + i] = i < r ? 0.0 : BV[(size_t)f * nn + (i - r)];
                VHs[(size_t)(kg + f) * t + i] = 0.0;
            }
            __syncthreads();
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
            for (int j = r - 1; j >= 0; --j) {
                const double* v = Hv + (size_t)j * t;
                for (int f = wave; f < nfill; f += nwave) {
                    const double* x = Xs + (size_t)(kg + f) * t;
                    double a = 0.0;
                    for (int i = j + lane; i < t; i += 64) a += v[i] * x[i];
                    a = wave_sum(a);
                    if (lane == 0) pw[f] = a;
                }
                __syncthreads();
                for (int idx = threadIdx.x; idx < nfill * t; idx += blockDim.x) {
                    const int f = idx / t, i = idx - f * t;
                    if (i >= j) Xs[(size_t)(kg + f) * t + i] -= s_beta[j] * pw[f] * v[i];
                }
                __syncthreads();
            }
        }
    }
    {   // unit columns of X~, one wave per column
        const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6), nwave = (int)(blockDim.x >> 6);
        for (int c = wave; c < s_eff; c += nwave) {
            double* x = Xs + (size_t)c * t;
            double part = 0.0;
            for (int i = lane; i < t; i += 64) part += x[i] * x[i];
            const double nrm = sqrt(wave_sum(part));
            for (int i = lane; i < t; i += 64) x[i] /= nrm;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        info[0] = s_eff;
        info[1] = rankG;
        info[2] = ok ? BL_OK : BL_E_BREAKDOWN;
    }
}

// Ritz (eq. ritz-matrix-decomp) or harmonic Ritz (eq. harmonic-ritz) selection of
// s_eff = min(s, t) vectors from the projected matrices (t x t, column-major; W orthonormal):
//   kind 0: eigenpairs of sym(M), chosen by the Ritz values;
//   kind 1: sym(M) rho = nu (Y^T Y) rho with Y^T Y = L L^T: eigenpairs (nu, z) of
//           K = L^{-1} sym(M) L^{-T}, rho = L^{-T} z, chosen by theta = 1 / nu.
// size 0 (S): the s_eff smallest values, ascending; 1 (L): the largest, descending; 2 (M):
// ceil(s_eff / 2) smallest, then floor(s_eff / 2) largest.  Output: Xs (t x s_eff, unit
// columns), VHs = 0 and mu = 0 (no error estimate), info = {s_eff, 0, status}.
__global__ void __launch_bounds__(SD_NT) k_ritz_select(int t, int s, int kind, int size, const double* __restrict__ Min,
                                                       const double* __restrict__ YtY, double* sc, double* Xs,
                                                       double* VHs, double* mu, int* info, int ldsd) {
    __shared__ int order[EIG_MAX];
    __shared__ int pick[EIG_MAX];
    __shared__ double val[EIG_MAX];
    const int s_eff = s < t ? s : t;
    const size_t T2 = (size_t)t * t;
    double* A = sc;           // sym(M), then K
    double* L = A + T2;       // Cholesky factor of Y^T Y
    double* Bm = L + T2;      // L^{-1} sym(M)
    double* Z = Bm + T2;      // eigenvectors, vector k at Z[k * t]
    double* lam = Z + T2;     // t eigenvalues, ascending
    double* esc = lam + t;    // eigensolver scratch (4 t^2 + t)
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
        const int j = idx / t, i = idx - j * t;
        A[idx] = 0.5 * (Min[(size_t)j * t + i] + Min[(size_t)i * t + j]);
        if (kind == 1) L[idx] = 0.5 * (YtY[(size_t)j * t + i] + YtY[(size_t)i * t + j]);
    }
    __syncthreads();
    if (kind == 1) {
        if (!chol_inplace(t, gbl(L))) {
            if (threadIdx.x == 0) {
                info[0] = 0;
                info[1] = 0;
                info[2] = BL_E_BREAKDOWN;
            }
            return;
        }
        // Bm = L^{-1} A, one column per thread
        for (int c = threadIdx.x; c < t; c += blockDim.x)
            for (int i = 0; i < t; ++i) {
                double acc = A[(size_t)c * t + i];
                for (int k = 0; k < i; ++k) acc -= L[(size_t)k * t + i] * Bm[(size_t)c * t + k];
                Bm[(size_t)c * t + i] = acc / L[(size_t)i * t + i];
            }
        __syncthreads();
        // K = L^{-1} Bm^T (A symmetric), into Z, then symmetrised into A
        for (int c = threadIdx.x; c < t; c += blockDim.x)
            for (int i = 0; i < t; ++i) {
                double acc = Bm[(size_t)i * t + c];
                for (int k = 0; k < i; ++k) acc -= L[(size_t)k * t + i] * Z[(size_t)c * t + k];
                Z[(size_t)c * t + i] = acc / L[(size_t)i * t + i];
            }
        __syncthreads();
        for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
            const int j = idx / t, i = idx - j * t;
            A[idx] = 0.5 * (Z[(size_t)j * t + i] + Z[(size_t)i * t + j]);
        }
        __syncthreads();
    }
    // Ritz S / L need only the s_eff vectors at one end (Ritz values ascend with the
    // eigenvalues); fewer vectors also let the eigensolver keep them in LDS.  Harmonic Ritz
    // and size M take all t.
    const int lo_e = (kind == 0 && size == 1) ? t - s_eff : 0;
    const int hi_e = (kind == 0 && size == 0) ? s_eff : t;
    eig_range(t, A, lo_e, hi_e, lam, Z, esc, ldsd);
    if (threadIdx.x == 0) {
        // values and their ascending order (insertion sort; t <= EIG_MAX)
        for (int k = 0; k < t; ++k) {
            val[k] = kind == 0 ? lam[k] : 1.0 / lam[k];
            order[k] = k;
        }
        for (int k = 1; k < t; ++k) {
            const int o = order[k];
            int q = k - 1;
            while (q >= 0 && val[order[q]] > val[o]) {
                order[q + 1] = order[q];
                --q;
            }
            order[q + 1] = o;
        }
        const int lo = size == 0 ? s_eff : (size == 1 ? 0 : (s_eff + 1) / 2);
        for (int j = 0; j < lo; ++j) pick[j] = order[j];
        for (int j = lo; j < s_eff; ++j) pick[j] = order[t - 1 - (j - lo)];
        if (hi_e - lo_e < t)   // one end only: by eigen index, within the computed range
            for (int j = 0; j < s_eff; ++j) pick[j] = size == 0 ? j : t - 1 - j;
    }
    __syncthreads();
    // vectors: z (Ritz) or rho = L^{-T} z (harmonic Ritz), unit columns; one column per thread
    for (int j = threadIdx.x; j < s_eff; j += blockDim.x) {
        const double* z = Z + (size_t)(pick[j] - lo_e) * t;
        double* x = Xs + (size_t)j * t;
        if (kind == 0) {
            for (int i = 0; i < t; ++i) x[i] = z[i];
        } else {
            for (int i = t - 1; i >= 0; --i) {
                double acc = z[i];
                for (int k = i + 1; k < t; ++k) acc -= L[(size_t)i * t + k] * x[k];
                x[i] = acc / L[(size_t)i * t + i];
            }
        }
        double nrm = 0.0;
        for (int i = 0; i < t; ++i) nrm += x[i] * x[i];
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = 0; i < t; ++i) {
            x[i] *= inv;
            VHs[(size_t)j * t + i] = 0.0;
        }
        mu[j] = 0.0;
    }
    if (threadIdx.x == 0) {
        info[0] = s_eff;
        info[1] = 0;
        info[2] = BL_OK;
    }
}

// Side of the RGen-L vectors: Xs holds the unit right vectors x of the info[0] selected
// columns; the left vector is v = sym(M) x / ||sym(M) x|| (the GSVD's M x = beta v with
// beta > 0).  side 1 (L): x <- v; side 2 (M): x <- x + v.
__global__ void __launch_bounds__(SD_NT) k_rgen_side(int t, int side, const double* __restrict__ Min, double* Xs,
                                                     const int* __restrict__ info) {
    __shared__ double xv[EIG_MAX], vv[EIG_MAX], red[SD_NT / 64];
    const int s_eff = info[0];
    for (int j = 0; j < s_eff; ++j) {
        double* x = Xs + (size_t)j * t;
        for (int i = threadIdx.x; i < t; i += blockDim.x) xv[i] = x[i];
        __syncthreads();
        double part = 0.0;
        for (int i = threadIdx.x; i < t; i += blockDim.x) {
            double acc = 0.0;
            for (int k = 0; k < t; ++k) acc += 0.5 * (Min[(size_t)k * t + i] + Min[(size_t)i * t + k]) * xv[k];
            vv[i] = acc;
            part += acc * acc;
        }
        const double nrm = sqrt(sd_sum(part, red));
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int i = threadIdx.x; i < t; i += blockDim.x) x[i] = side == 1 ? vv[i] * inv : xv[i] + vv[i] * inv;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ inner refresh (eq. subtle-old)
// C = op(A) B for small dense matrices (column-major; op(A) = A, m x k at lda, or A^T with A
// k x m at lda), one output element per thread.
__global__ void __launch_bounds__(NT) k_small_gemm(int m, int k, int ncols, int trans_a, const double* __restrict__ A,
                                                   int lda, const double* __restrict__ Bm, int ldb, double* __restrict__ Cm,
                                                   int ldc) {
    const int idx = blockIdx.x * NT + threadIdx.x;
    if (idx >= m * ncols) return;
    const int i = idx % m, j = idx / m;
    double acc = 0.0;
    if (trans_a)
        for (int q = 0; q < k; ++q) acc += A[(size_t)i * lda + q] * Bm[(size_t)j * ldb + q];
    else
        for (int q = 0; q < k; ++q) acc += A[(size_t)q * lda + i] * Bm[(size_t)j * ldb + q];
    Cm[(size_t)j * ldc + i] = acc;
}

// Y = M0 X for the previous solve's projected Hessian in the basis [U, V] (t0 = s0 + v columns):
// M0 = blockdiag(sym(U^T C), T), T the tridiagonal matrix of the CG coefficients of the stored
// residuals (alpha_j = lz[2j], rho_j = lz[2j+1]):
//   T_aa = 1/alpha_a + (rho_a / rho_{a-1}) / alpha_{a-1},  T_{a,a+1} = -sqrt(rho_{a+1} / rho_a) / alpha_a.
// X: t0 x t (ld t0), Y likewise; UtC: s0 x s0 (column-major).
__global__ void __launch_bounds__(NT) k_inner_y(int s0, int v, int t, const double* __restrict__ UtC,
                                                const double* __restrict__ lz, const double* __restrict__ X,
                                                double* __restrict__ Y) {
    const int t0 = s0 + v;
    const int idx = blockIdx.x * NT + threadIdx.x;
    if (idx >= t0 * t) return;
    const int i = idx % t0, c = idx / t0;
    const double* x = X + (size_t)c * t0;
    double acc = 0.0;
    if (i < s0) {
        for (int q = 0; q < s0; ++q) acc += 0.5 * (UtC[(size_t)q * s0 + i] + UtC[(size_t)i * s0 + q]) * x[q];
    } else {
        const int a = i - s0;
        const double al = lz[2 * a], rh = lz[2 * a + 1];
        double d = 1.0 / al;
        if (a > 0) {
            const double alm = lz[2 * a - 2], rhm = lz[2 * a - 1];
            d += (rh / rhm) / alm;
            acc += -sqrt(rh / rhm) / alm * x[i - 1];
        }
        acc += d * x[i];
        if (a + 1 < v) acc += -sqrt(lz[2 * a + 3] / rh) / al * x[i + 1];
    }
    Y[(size_t)c * t0 + i] = acc;
}

// Leading columns of a stored basis that are semi-orthogonal, from the Gram matrix of [U, V]
// (t0 x t0, V in columns s0 ..): column j of V qualifies while |G_jj - 1| and every |G_ij| with
// i < j in the V block are within tol; out[0] = the first column that breaks it (or all of V).
__global__ void __launch_bounds__(SD_NT) k_semiorth_prefix(int t0, int s0, const double* __restrict__ G, double tol,
                                                           int* __restrict__ out) {
    __shared__ int first;
    const int v = t0 - s0;
    if (threadIdx.x == 0) first = v;
    __syncthreads();
    for (int j = threadIdx.x; j < v; j += blockDim.x) {
        const double* col = G + (size_t)(s0 + j) * t0;
        bool bad = fabs(col[s0 + j] - 1.0) > tol;
        for (int i = 0; i < j && !bad; ++i) bad = fabs(col[s0 + i]) > tol;
        if (bad) atomicMin(&first, j);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[0] = first;
}

hipError_t launch_semiorth_prefix(int t0, int s0, const double* G, double tol, int* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_semiorth_prefix, dim3(1), dim3(SD_NT), 0, stream, t0, s0, G, tol, out);
    return hipGetLastError();
}

hipError_t launch_small_gemm(int m, int k, int ncols, bool trans_a, const double* A, int lda, const double* B, int ldb,
                             double* C, int ldc, hipStream_t stream) {
    if (m <= 0 || ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_small_gemm, dim3((m * ncols + NT - 1) / NT), dim3(NT), 0, stream, m, k, ncols,
                       trans_a ? 1 : 0, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
}

hipError_t launch_inner_y(int s0, int v, int t, const double* UtC, const double* lz, const double* X, double* Y,
                          hipStream_t stream) {
    const int tot = (s0 + v) * t;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inner_y, dim3((tot + NT - 1) / NT), dim3(NT), 0, stream, s0, v, t, UtC, lz, X, Y);
    return hipGetLastError();
}

size_t gsvd_scratch_doubles(int t, int p) {
    const size_t T2 = (size_t)t * t, P2 = (size_t)p * p, PT = (size_t)p * t, KM = T2 > P2 ? T2 : P2;
    const size_t m = t > p ? t : p;
    return T2 + PT + 2 * KM + 2 * P2 + PT + 2 * T2 + (t + p) + 5 * m * m + m + 64;
}

// Largest dynamic LDS per workgroup, queried once (falls back to 64 KiB).
static size_t lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        lim = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lim = (size_t)v;
        lim -= 24576;   // room for the kernels' static LDS (k_gsvd_select: about 18 KiB)
    }
    return lim;
}

hipError_t launch_chol_drop(int t, const double* Gm, double tol, double* R, int* kept, int* tk, double* Xinv,
                            int ldx, hipStream_t stream) {
    (void)kept;   // the kept-column list lives in LDS
    if (t < 0 || t > 256) return hipErrorInvalidValue;   // LDS lists of 256 columns
    const size_t one = (size_t)t * t * sizeof(double);
    const int lds = 2 * one <= lds_limit() ? 2 : (one <= lds_limit() ? 1 : 0);
    const size_t bytes = lds * one;
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)k_chol_drop, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(SD_NT), bytes, stream, t, Gm, tol, R, tk, Xinv, ldx, lds);
    return hipGetLastError();
}

hipError_t launch_gsvd_select(int t, int p, int s, int size, const double* M, const double* G, double* sc,
                              double* Xs, double* VHs, double* mu, int* info, hipStream_t stream) {
    // dynamic LDS: the eigensolver's matrix plus its vectors, the solves' factor plus columns;
    // at least the S^T S chunk
    const size_t want = std::max((size_t)3 * t * t + (size_t)6 * t * t, (size_t)KC * t) * sizeof(double);
    const size_t bytes = std::min(want, lds_limit()) / sizeof(double) * sizeof(double);
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)k_gsvd_select, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_gsvd_select, dim3(1), dim3(SD_NT), bytes, stream, t, p, s, size, M, G, sc, Xs, VHs, mu,
                       info, (int)(bytes / sizeof(double)));
    return hipGetLastError();
}

hipError_t launch_ritz_select(int t, int s, int kind, int size, const double* M, const double* YtY, double* sc,
                              double* Xs, double* VHs, double* mu, int* info, hipStream_t stream) {
    const size_t want = (size_t)6 * t * t * sizeof(double);
    const size_t bytes = std::min(want, lds_limit()) / sizeof(double) * sizeof(double);
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)k_ritz_select, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_ritz_select, dim3(1), dim3(SD_NT), bytes, stream, t, s, kind, size, M, YtY, sc, Xs, VHs, mu,
                       info, (int)(bytes / sizeof(double)));
    return hipGetLastError();
}

hipError_t launch_rgen_side(int t, int side, const double* M, double* Xs, const int* info, hipStream_t stream) {
    hipLaunchKernelGGL(k_rgen_side, dim3(1), dim3(SD_NT), 0, stream, t, side, M, Xs, info);
    return hipGetLastError();
}

}  // namespace bl
