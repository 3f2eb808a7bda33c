// Dense kernels of the recycle-space refresh: tall-skinny Gram products, tall x small
// products, and single-workgroup small dense algebra (Cholesky with column drop,
// parallel cyclic Jacobi, projected GSVD and Ritz-GSV selection).
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

__global__ void k_sum_chunks(int nchunks, int len, const double* __restrict__ part, double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * len + k];
    out[k] = s;
}

int gram_chunks(int n) {
    int c = (n + 255) / 256;
    return c < 1 ? 1 : (c > 512 ? 512 : c);
}

hipError_t launch_gram(int n, int t1, int t2, const double* A, const double* B, double* part, double* out,
                       hipStream_t stream) {
    const int nch = gram_chunks(n);
    const int chunk_rows = (n + nch - 1) / nch;
    dim3 grid(nch, (t1 + GRAM_T - 1) / GRAM_T, (t2 + GRAM_T - 1) / GRAM_T);
    hipLaunchKernelGGL(k_gram, grid, dim3(NT), 0, stream, n, t1, t2, A, B, chunk_rows, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int len = t1 * t2;
    hipLaunchKernelGGL(k_sum_chunks, dim3((len + 255) / 256), dim3(256), 0, stream, nch, len, part, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Out = A X (tall x small)
// A: n x t (ld n); X: t x k (ld ldx); Out: n x k (ld n).  One row per thread, 16 outputs
// at a time, X staged in LDS.
constexpr int GT_K = 16;
constexpr int GT_TMAX = 256;

__global__ void __launch_bounds__(NT) k_gemm_tall(int n, int t, int k, const double* __restrict__ A,
                                                  const double* __restrict__ X, int ldx, double* __restrict__ Out) {
    __shared__ double Xs[GT_TMAX * GT_K];
    const int i = blockIdx.x * NT + threadIdx.x;
    for (int k0 = 0; k0 < k; k0 += GT_K) {
        const int kk = min(GT_K, k - k0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < t * GT_K; idx += NT) {
            const int j = idx / GT_K, c = idx - j * GT_K;
            Xs[idx] = (c < kk) ? X[(size_t)(k0 + c) * ldx + j] : 0.0;
        }
        __syncthreads();
        if (i < n) {
            double acc[GT_K];
#pragma unroll
            for (int c = 0; c < GT_K; ++c) acc[c] = 0.0;
            for (int j = 0; j < t; ++j) {
                const double a = A[(size_t)j * n + i];
#pragma unroll
                for (int c = 0; c < GT_K; ++c) acc[c] += a * Xs[j * GT_K + c];
            }
            for (int c = 0; c < kk; ++c) Out[(size_t)(k0 + c) * n + i] = acc[c];
        }
    }
}

hipError_t launch_gemm_tall(int n, int t, int k, const double* A, const double* X, int ldx, double* Out,
                            hipStream_t stream) {
    if (t > GT_TMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_tall, dim3((n + NT - 1) / NT), dim3(NT), 0, stream, n, t, k, A, X, ldx, Out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ small dense (one workgroup)
constexpr int SD_NT = 512;

// Cholesky with column drop on a t x t Gram matrix Gm (column-major, ld t), right-looking in
// column order: the pivot of column j is its diagonal after the updates from the kept
// columns before it (= squared norm of column j after projection); j is dropped when
// pivot_j <= tol^2 Gm_jj.  Writes Xinv (t x tk, ld ldx) with W Xinv = orthonormal basis of
// the kept columns (rows of dropped columns zero) and *tk_out = tk.  Scratch: A (t*t), kept (t).
__device__ void chol_drop(int t, const double* __restrict__ Gm, double tol, double* A, int* kept, int* tk_out,
                          double* Xinv, int ldx) {
    __shared__ int s_tk, s_keep;
    __shared__ double s_d;
    __shared__ int s_kept[256];
    kept = s_kept;
    if (threadIdx.x == 0) s_tk = 0;
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) A[idx] = Gm[idx];
    __syncthreads();
    for (int j = 0; j < t; ++j) {
        if (threadIdx.x == 0) {
            const double piv = A[(size_t)j * t + j];
            const double gjj = Gm[(size_t)j * t + j];
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
        const int m = t - j - 1;
        for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
            const int kk = idx / m, ii = idx - kk * m;
            const int k = j + 1 + kk, i = j + 1 + ii;
            A[(size_t)k * t + i] -= A[(size_t)i * t + j] * A[(size_t)k * t + j];
        }
        __syncthreads();
    }
    const int tk = s_tk;
    for (int idx = threadIdx.x; idx < t * tk; idx += blockDim.x) Xinv[(size_t)(idx / t) * ldx + idx % t] = 0.0;
    __syncthreads();
    // R (kept rows/cols) upper triangular: Rk[k][l] = A[kept_l * t + kept_k] (k < l), diag A[kept_k*t+kept_k]
    for (int mcol = threadIdx.x; mcol < tk; mcol += blockDim.x) {
        double* x = Xinv + (size_t)mcol * ldx;
        for (int k = mcol; k >= 0; --k) {
            const int ck = kept[k];
            double v = (k == mcol) ? 1.0 : 0.0;
            for (int l = k + 1; l <= mcol; ++l) v -= A[(size_t)kept[l] * t + ck] * x[kept[l]];
            x[ck] = v / A[(size_t)ck * t + ck];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *tk_out = tk;
}

// The working matrix lives in LDS when it fits (lds != 0), else in the global scratch R.
__global__ void __launch_bounds__(SD_NT) k_chol_drop(int t, const double* Gm, double tol, double* R, int* kept,
                                                     int* tk_out, double* Xinv, int ldx, int lds) {
    extern __shared__ double dyn_lds[];
    chol_drop(t, Gm, tol, lds ? dyn_lds : R, kept, tk_out, Xinv, ldx);
}

// Parallel cyclic Jacobi on a symmetric m x m matrix A (row-major, in place -> eigenvalues on
// the diagonal), eigenvectors accumulated in V (row-major, V[i*m + k] = component i of
// vector k).  Round-robin pairing; m is padded to even with a decoupled index.
__device__ void jacobi_eigh(int m, double* A, double* V, double* cs, int* pairs, int max_sweeps) {
    const int me = (m + 1) & ~1;      // even count; index m (if padded) is a dummy
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) V[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
    __shared__ double s_off, s_norm;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal Frobenius norm relative to the full norm
        {
            __shared__ double r_off[SD_NT / 64], r_nrm[SD_NT / 64];
            double off = 0.0, nrm = 0.0;
            for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
                const double v = A[idx];
                nrm += v * v;
                if (idx / m != idx % m) off += v * v;
            }
            off = wave_sum(off);
            nrm = wave_sum(nrm);
            if ((threadIdx.x & 63) == 0) {
                r_off[threadIdx.x >> 6] = off;
                r_nrm[threadIdx.x >> 6] = nrm;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double a = 0.0, b = 0.0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                    a += r_off[w];
                    b += r_nrm[w];
                }
                s_off = a;
                s_norm = b;
            }
            __syncthreads();
        }
        if (s_off <= 1e-30 * s_norm || s_off == 0.0) break;
        for (int rnd = 0; rnd < me - 1; ++rnd) {
            const int np = me / 2;
            for (int k = threadIdx.x; k < np; k += blockDim.x) {
                int a, b;
                if (k == 0) {
                    a = 0;
                    b = (rnd % (me - 1)) + 1;
                } else {
                    a = ((k + rnd) % (me - 1)) + 1;
                    b = ((me - 1 - k + rnd) % (me - 1)) + 1;
                }
                const int p = a < b ? a : b, q = a < b ? b : a;
                pairs[2 * k] = p;
                pairs[2 * k + 1] = q;
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[p * m + q];
                    if (apq != 0.0) {
                        const double tau = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                cs[2 * k] = c;
                cs[2 * k + 1] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = threadIdx.x; idx < np * m; idx += blockDim.x) {
                const int k = idx / m, j = idx - k * m;
                const int p = pairs[2 * k], q = pairs[2 * k + 1];
                if (q >= m) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                const double ap = A[p * m + j], aq = A[q * m + j];
                A[p * m + j] = c * ap - s * aq;
                A[q * m + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int idx = threadIdx.x; idx < np * m; idx += blockDim.x) {
                const int k = idx / m, i = idx - k * m;
                const int p = pairs[2 * k], q = pairs[2 * k + 1];
                if (q >= m) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                const double ap = A[i * m + p], aq = A[i * m + q];
                A[i * m + p] = c * ap - s * aq;
                A[i * m + q] = s * ap + c * aq;
                const double vp = V[i * m + p], vq = V[i * m + q];
                V[i * m + p] = c * vp - s * vq;
                V[i * m + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
}

// Cholesky M = L L^T in place (lower, column-major ld t).  Returns false if not SPD.
__device__ bool chol_inplace(int t, double* L) {
    __shared__ int s_ok;
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
        // trailing update: L[i][k] -= L[i][j] L[k][j], j < k <= i
        const int m = t - j - 1;
        for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
            const int kk = idx / m, ii = idx - kk * m;
            const int k = j + 1 + kk, i = j + 1 + ii;
            if (i >= k) L[(size_t)k * t + i] -= L[(size_t)j * t + i] * L[(size_t)j * t + k];
        }
        __syncthreads();
    }
    return true;
}

// x <- M^{-1} x with M = L L^T (single thread, one right-hand side of length t).
__device__ void chol_solve(int t, const double* L, double* x) {
    for (int i = 0; i < t; ++i) {
        double v = x[i];
        for (int k = 0; k < i; ++k) v -= L[(size_t)k * t + i] * x[k];
        x[i] = v / L[(size_t)i * t + i];
    }
    for (int i = t - 1; i >= 0; --i) {
        double v = x[i];
        for (int k = i + 1; k < t; ++k) v -= L[(size_t)i * t + k] * x[k];
        x[i] = v / L[(size_t)i * t + i];
    }
}

// Projected GSVD of (G, M) (p x t and t x t) and RGen-L(R) selection of s_eff = min(s, t)
// columns.  Output: Xs (t x s_eff, unit columns), VHs (t x s_eff, zero for filled slots),
// mu (s_eff), info = {s_eff, rank_G, status}.  Scratch: sc (see sizes in the host).
// Route: Cholesky M = L L^T;  S = G M^{-1};
//   p >= t: eigen of S^T S = V_H diag(mu^2) V_H^T; right vectors X ~ M^{-1} V_H;
//   p <  t: eigen of S S^T (p x p) gives mu and V_H = S^T u / mu; null(G) from Householder QR
//           of G^T; the remaining slots take the smallest Ritz pairs of N^T M N (Ritz-S).
// Run the symmetric Jacobi solver on (A, V) (m x m, global scratch), staging both in LDS
// when `lds` (2 m^2 doubles fit).
__device__ void jacobi_staged(int m, double* A, double* V, double* cs, int* pairs, int lds) {
    extern __shared__ double dyn_lds[];
    if (!lds) {
        jacobi_eigh(m, A, V, cs, pairs, 40);
        return;
    }
    double* LA = dyn_lds;
    double* LV = dyn_lds + (size_t)m * m;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) LA[idx] = A[idx];
    __syncthreads();
    jacobi_eigh(m, LA, LV, cs, pairs, 40);
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        A[idx] = LA[idx];
        V[idx] = LV[idx];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(SD_NT) k_gsvd_select(int t, int p, int s, const double* __restrict__ Min,
                                                       const double* __restrict__ G, double* sc, double* Xs,
                                                       double* VHs, double* mu, int* info, int lds) {
    extern __shared__ double dyn_lds[];
    __shared__ double cs[SD_NT];
    __shared__ int pairs[SD_NT];
    __shared__ int s_rank;
    __shared__ double s_beta[64];
    const int s_eff = s < t ? s : t;
    const size_t T2 = (size_t)t * t, P2 = (size_t)p * p, PT = (size_t)p * t;
    double* L = sc;                 // t*t   Cholesky factor of sym(M)
    double* S = L + T2;             // p*t   G M^{-1}, column-major ld p
    double* K = S + PT;             // t*t or p*p   S^T S  |  S S^T
    double* Vv = K + T2 + P2;       // t*t or p*p   eigenvectors of K
    double* GG = Vv + T2 + P2;      // p*p   G G^T
    double* GV = GG + P2;           // p*p
    double* Hv = GV + P2;           // t*p   Householder vectors of G^T
    double* Nb = Hv + PT;           // t*t   basis of null(G)
    double* Ms = Nb + T2;           // t*t   sym(M)
    double* MN = Ms + T2;           // t*t   M N
    double* B = MN + T2;            // t*t   N^T M N
    double* BV = B + T2;            // t*t
    int* order = reinterpret_cast<int*>(BV + T2);   // t + p ints
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
        const int j = idx / t, i = idx - j * t;
        const double v = 0.5 * (Min[(size_t)j * t + i] + Min[(size_t)i * t + j]);
        L[idx] = v;
        Ms[idx] = v;
    }
    __syncthreads();
    {
        double* LL = lds ? dyn_lds : L;   // factor in LDS, then copy back
        if (lds)
            for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) LL[idx] = L[idx];
        __syncthreads();
        const bool spd = chol_inplace(t, LL);
        if (lds) {
            for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) L[idx] = LL[idx];
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
    // S[k, :] = (M^{-1} G[k, :]^T)^T, one row per thread
    for (int k = threadIdx.x; k < p; k += blockDim.x) {
        double* row = S + k;   // stride p
        for (int j = 0; j < t; ++j) row[(size_t)j * p] = G[(size_t)j * p + k];
        for (int i = 0; i < t; ++i) {
            double v = row[(size_t)i * p];
            for (int q = 0; q < i; ++q) v -= L[(size_t)q * t + i] * row[(size_t)q * p];
            row[(size_t)i * p] = v / L[(size_t)i * t + i];
        }
        for (int i = t - 1; i >= 0; --i) {
            double v = row[(size_t)i * p];
            for (int q = i + 1; q < t; ++q) v -= L[(size_t)i * t + q] * row[(size_t)q * p];
            row[(size_t)i * p] = v / L[(size_t)i * t + i];
        }
    }
    __syncthreads();
    int rankG;
    if (p >= t) {
        for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
            const int i = idx / t, j = idx - i * t;
            double v = 0.0;
            for (int k = 0; k < p; ++k) v += S[(size_t)i * p + k] * S[(size_t)j * p + k];
            K[idx] = v;
        }
        __syncthreads();
        jacobi_staged(t, K, Vv, cs, pairs, lds);
        if (threadIdx.x == 0) {
            for (int i = 0; i < t; ++i) order[i] = i;
            for (int i = 1; i < t; ++i) {   // descending mu^2, stable
                const int oi = order[i];
                const double vi = K[oi * t + oi];
                int j = i - 1;
                while (j >= 0 && K[order[j] * t + order[j]] < vi) {
                    order[j + 1] = order[j];
                    --j;
                }
                order[j + 1] = oi;
            }
            s_rank = t;
        }
        __syncthreads();
        rankG = s_rank;
        for (int c = threadIdx.x; c < s_eff; c += blockDim.x) {
            const int o = order[c];
            const double lam = K[o * t + o];
            mu[c] = lam > 0.0 ? sqrt(lam) : 0.0;
            double* x = Xs + (size_t)c * t;
            for (int i = 0; i < t; ++i) {
                VHs[(size_t)c * t + i] = Vv[i * t + o];
                x[i] = Vv[i * t + o];
            }
            chol_solve(t, L, x);
        }
        __syncthreads();
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
        jacobi_staged(p, K, Vv, cs, pairs, lds);
        jacobi_staged(p, GG, GV, cs, pairs, lds);
        if (threadIdx.x == 0) {
            double mx2 = 0.0;
            for (int i = 0; i < p; ++i) mx2 = fmax(mx2, GG[i * p + i]);
            int r = 0;
            for (int i = 0; i < p; ++i)
                if (GG[i * p + i] > 1e-16 * mx2) ++r;   // singular values of G above 1e-8 of the largest
            s_rank = r;
            for (int i = 0; i < p; ++i) order[i] = i;
            for (int i = 1; i < p; ++i) {
                const int oi = order[i];
                const double vi = K[oi * p + oi];
                int j = i - 1;
                while (j >= 0 && K[order[j] * p + order[j]] < vi) {
                    order[j + 1] = order[j];
                    --j;
                }
                order[j + 1] = oi;
            }
        }
        __syncthreads();
        rankG = s_rank;
        const int kg = s_eff < rankG ? s_eff : rankG;
        for (int c = threadIdx.x; c < kg; c += blockDim.x) {
            const int o = order[c];
            const double lam = K[o * p + o];
            mu[c] = lam > 0.0 ? sqrt(lam) : 0.0;
            double* vh = VHs + (size_t)c * t;
            double* x = Xs + (size_t)c * t;
            double nrm = 0.0;
            for (int i = 0; i < t; ++i) {
                double v = 0.0;
                for (int k = 0; k < p; ++k) v += S[(size_t)i * p + k] * Vv[k * p + o];
                vh[i] = v;
                nrm += v * v;
            }
            nrm = sqrt(nrm);
            for (int i = 0; i < t; ++i) {
                vh[i] /= nrm;
                x[i] = vh[i];
            }
            chol_solve(t, L, x);
        }
        __syncthreads();
        const int nfill = s_eff - kg;
        if (nfill > 0 && p <= 64) {
            const int nn = t - p;
            if (threadIdx.x == 0) {   // Householder QR of G^T (t x p), reflectors in Hv
                for (int j = 0; j < p; ++j)
                    for (int i = 0; i < t; ++i) Hv[(size_t)j * t + i] = G[(size_t)i * p + j];
                for (int j = 0; j < p; ++j) {
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
                    for (int jj = j + 1; jj < p; ++jj) {
                        double* u = Hv + (size_t)jj * t;
                        double d = 0.0;
                        for (int i = j; i < t; ++i) d += v[i] * u[i];
                        for (int i = j; i < t; ++i) u[i] -= beta * d * v[i];
                    }
                }
            }
            __syncthreads();
            for (int c = threadIdx.x; c < nn; c += blockDim.x) {   // N = Q[:, p:]
                double* col = Nb + (size_t)c * t;
                for (int i = 0; i < t; ++i) col[i] = (i == p + c) ? 1.0 : 0.0;
                for (int j = p - 1; j >= 0; --j) {
                    const double* v = Hv + (size_t)j * t;
                    double d = 0.0;
                    for (int i = j; i < t; ++i) d += v[i] * col[i];
                    for (int i = j; i < t; ++i) col[i] -= s_beta[j] * d * v[i];
                }
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < t * nn; idx += blockDim.x) {
                const int c = idx / t, i = idx - c * t;
                double v = 0.0;
                for (int k = 0; k < t; ++k) v += Ms[(size_t)k * t + i] * Nb[(size_t)c * t + k];
                MN[idx] = v;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < nn * nn; idx += blockDim.x) {
                const int i = idx / nn, j = idx - i * nn;
                double v = 0.0;
                for (int k = 0; k < t; ++k) v += Nb[(size_t)i * t + k] * MN[(size_t)j * t + k];
                B[idx] = v;
            }
            __syncthreads();
            jacobi_staged(nn, B, BV, cs, pairs, lds);
            if (threadIdx.x == 0) {
                for (int i = 0; i < nn; ++i) order[i] = i;
                for (int i = 1; i < nn; ++i) {   // ascending Ritz values
                    const int oi = order[i];
                    const double vi = B[oi * nn + oi];
                    int j = i - 1;
                    while (j >= 0 && B[order[j] * nn + order[j]] > vi) {
                        order[j + 1] = order[j];
                        --j;
                    }
                    order[j + 1] = oi;
                }
            }
            __syncthreads();
            for (int f = threadIdx.x; f < nfill; f += blockDim.x) {
                const int c = kg + f;
                const int o = order[f];
                mu[c] = 0.0;
                double* x = Xs + (size_t)c * t;
                for (int i = 0; i < t; ++i) {
                    double v = 0.0;
                    for (int k = 0; k < nn; ++k) v += Nb[(size_t)k * t + i] * BV[k * nn + o];
                    x[i] = v;
                    VHs[(size_t)c * t + i] = 0.0;
                }
            }
            __syncthreads();
        }
    }
    for (int c = threadIdx.x; c < s_eff; c += blockDim.x) {   // unit columns of X~
        double* x = Xs + (size_t)c * t;
        double nrm = 0.0;
        for (int i = 0; i < t; ++i) nrm += x[i] * x[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < t; ++i) x[i] /= nrm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        info[0] = s_eff;
        info[1] = rankG;
        info[2] = BL_OK;
    }
}

size_t gsvd_scratch_doubles(int t, int p) {
    const size_t T2 = (size_t)t * t, P2 = (size_t)p * p, PT = (size_t)p * t;
    return T2 + PT + 2 * (T2 + P2) + 2 * P2 + PT + 6 * T2 + (t + p) + 64;
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
        lim -= 16384;   // room for the kernels' static LDS
    }
    return lim;
}

hipError_t launch_chol_drop(int t, const double* Gm, double tol, double* R, int* kept, int* tk, double* Xinv,
                            int ldx, hipStream_t stream) {
    const size_t bytes = (size_t)t * t * sizeof(double);
    const int lds = bytes <= lds_limit() ? 1 : 0;
    if (lds && bytes > 65536)
        (void)hipFuncSetAttribute((const void*)k_chol_drop, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(SD_NT), lds ? bytes : 0, stream, t, Gm, tol, R, kept, tk, Xinv, ldx,
                       lds);
    return hipGetLastError();
}

hipError_t launch_gsvd_select(int t, int p, int s, const double* M, const double* G, double* sc, double* Xs,
                              double* VHs, double* mu, int* info, hipStream_t stream) {
    // Jacobi problems are at most t x t (t x t for p >= t; p x p and (t-p) x (t-p) otherwise)
    const int m = t;
    const size_t bytes = 2 * (size_t)m * m * sizeof(double);
    const int lds = bytes <= lds_limit() ? 1 : 0;
    if (lds && bytes > 65536)
        (void)hipFuncSetAttribute((const void*)k_gsvd_select, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_gsvd_select, dim3(1), dim3(SD_NT), lds ? bytes : 0, stream, t, p, s, M, G, sc, Xs, VHs, mu,
                       info, lds);
    return hipGetLastError();
}

}  // namespace bl
