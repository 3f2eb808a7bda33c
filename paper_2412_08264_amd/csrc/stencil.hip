// Stencil kernels: Hessian-vector products, the fused CG apply step, residual set-up,
// filter-state precompute, the hypergradient map J, the lower-level gradient and A.
#include "kernels.h"
#include "stencil.h"
#include "tile.h"

namespace bl {

__device__ __forceinline__ void tile_origin(const Stencil& S, int tile, int& r0, int& c0) {
    r0 = (tile / S.tiles_x) * TH;
    c0 = (tile % S.tiles_x) * TW;
}

// Per-block partial record of nv values; value k of this thread given by `val(k)`.
template <typename Val>
__device__ __forceinline__ void write_partials(double* part, int nv, double*, Val val) {
    block_partials(part, nv, val);
}

// ------------------------------------------------------------------ filter state
// d1_j = phi'(K_j xhat), d2_j = phi''(K_j xhat) (FP64 maps, plus FP32 copies of d2).
__global__ void __launch_bounds__(NT) k_filter_state(Stencil S, const double* __restrict__ xhat,
                                                     double* __restrict__ d1, double* __restrict__ d2,
                                                     float* __restrict__ d2f) {
    const int i = blockIdx.x * NT + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= S.n) return;
    const int gi = i / S.w, gj = i - gi * S.w, F = S.fs / 2;
    const double* kj = S.taps + j * S.fs * S.fs;
    double s = 0.0;
    for (int a = 0; a < S.fs; ++a) {
        const int ii = gi + a - F;
        if (ii < 0 || ii >= S.h) continue;
        for (int b = 0; b < S.fs; ++b) {
            const int jj = gj + b - F;
            if (jj < 0 || jj >= S.w) continue;
            s += kj[a * S.fs + b] * xhat[ii * S.w + jj];
        }
    }
    double p1, p2;
    if (S.penalty == BL_PEN_LOG) {
        const double den = 1.0 + s * s;
        p1 = 2.0 * s / den;
        p2 = 2.0 * (1.0 - s * s) / (den * den);
    } else {
        p1 = 2.0 * s;
        p2 = 2.0;
    }
    const size_t o = (size_t)j * S.n + i;
    d1[o] = p1;
    d2[o] = p2;
    d2f[o] = (float)p2;
}

// ------------------------------------------------------------------ J for smoothed TV
// Column c of G (2 x ncols): [-lam sum <u/psi, D w_c>, lam gam2 sum <u/psi^3, D w_c>], u = D xhat.
__global__ void __launch_bounds__(NT) k_jac_tv(Stencil S, const double* __restrict__ xhat,
                                               const double* __restrict__ wv, double* __restrict__ part) {
    __shared__ double red[NWAVE];
    const double* w = wv + (size_t)blockIdx.y * S.n;
    double s0 = 0.0, s1 = 0.0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < S.n; i += gridDim.x * NT) {
        const int gi = i / S.w, gj = i - gi * S.w;
        const double a = (gj < S.w - 1) ? xhat[i + 1] - xhat[i] : 0.0;
        const double b = (gi < S.h - 1) ? xhat[i + S.w] - xhat[i] : 0.0;
        const double da = (gj < S.w - 1) ? w[i + 1] - w[i] : 0.0;
        const double db = (gi < S.h - 1) ? w[i + S.w] - w[i] : 0.0;
        const double psi2 = a * a + b * b + S.gam2;
        const double psi = sqrt(psi2);
        const double dot = a * da + b * db;
        s0 += dot / psi;
        s1 += dot / (psi2 * psi);
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        double* pr = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        pr[0] = -S.lam * s0;
        pr[1] = S.lam * S.gam2 * s1;
    }
}

// ------------------------------------------------------------------ J for filters
// Column c of G = J W (p x ncols), per block over a band of 8 x 32 tiles:
//   [J w]_{w_j}      = -lam_j <d1_j, K_j w>
//   [J w]_{k_j[a,b]} = -lam_j (<d1_j, S_ab w> + <d2_j . K_j w, S_ab xhat>)
// (S_ab: shift by (a - F, b - F), zero outside the image).  Per tile, each thread forms K_j w
// at one pixel for every filter from one window of w (the taps are uniform loads) and stores
// d1_j and t_j = d2_j . K_j w; then items (j, a, r) (filter, tap row, tile row) sweep the 32
// columns of row r with sliding windows of w and xhat held in registers, accumulating the FS
// tap sums of both terms.  The accumulators stay in registers across the block's tiles and are
// summed over the 8 tile rows (8 adjacent lanes) by a group sum at the end, in a fixed order.
constexpr int JF_BLOCKS = 64;
template <int FS>
__global__ void __launch_bounds__(NT) k_jac_filters(Stencil S, const double* __restrict__ xhat,
                                                    const double* __restrict__ wv, const double* __restrict__ d1,
                                                    const double* __restrict__ d2, double* __restrict__ part) {
    constexpr int F = FS / 2, F2 = FS * FS;
    constexpr int WW = TW + 2 * F, HH = TH + 2 * F;
    constexpr int NITEM = MAX_NF * FS * TH;
    constexpr int IPT = (NITEM + NT - 1) / NT;
    __shared__ double ws[HH * WW], xs[HH * WW];
    __shared__ double d1s[MAX_NF][TH * TW], tss[MAX_NF][TH * TW];
    __shared__ double acc_s[MAX_NF * (1 + F2)];
    __shared__ double wred[NWAVE][MAX_NF];
    const int nf = S.nf, p = nf * (1 + F2);
    const size_t n = (size_t)S.n;
    const double* __restrict__ w = wv + (size_t)blockIdx.y * n;
    const double* __restrict__ tp = S.taps;
    double A1[IPT][FS], A2[IPT][FS], wacc[MAX_NF];
#pragma unroll
    for (int u = 0; u < IPT; ++u)
#pragma unroll
        for (int b = 0; b < FS; ++b) A1[u][b] = A2[u][b] = 0.0;
#pragma unroll
    for (int j = 0; j < MAX_NF; ++j) wacc[j] = 0.0;
    const int pr_ = threadIdx.x / TW, pc = threadIdx.x % TW;   // the thread's pixel of a tile
    const int ntiles = S.tiles_x * S.tiles_y;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int r0, c0;
        tile_origin(S, tile, r0, c0);
        __syncthreads();   // the previous tile's sweep is done with the LDS arrays
        for (int idx = threadIdx.x; idx < HH * WW; idx += NT) {
            const int rr = idx / WW, cc = idx - rr * WW;
            const int gi = r0 - F + rr, gj = c0 - F + cc;
            const bool in = gi >= 0 && gi < S.h && gj >= 0 && gj < S.w;
            ws[idx] = in ? w[(size_t)gi * S.w + gj] : 0.0;
            xs[idx] = in ? xhat[(size_t)gi * S.w + gj] : 0.0;
        }
        __syncthreads();
        {
            const int gi = r0 + pr_, gj = c0 + pc;
            const bool in = gi < S.h && gj < S.w;
            double kw[MAX_NF];
#pragma unroll
            for (int j = 0; j < MAX_NF; ++j) kw[j] = 0.0;
#pragma unroll
            for (int a = 0; a < FS; ++a) {
                double win[FS];
#pragma unroll
                for (int b = 0; b < FS; ++b) win[b] = ws[(pr_ + a) * WW + pc + b];
#pragma unroll
                for (int j = 0; j < MAX_NF; ++j) {
                    if (j >= nf) break;
#pragma unroll
                    for (int b = 0; b < FS; ++b) kw[j] += tp[j * F2 + a * FS + b] * win[b];
                }
            }
            const size_t o = in ? (size_t)gi * S.w + gj : 0;
#pragma unroll
            for (int j = 0; j < MAX_NF; ++j) {
                if (j >= nf) break;
                const double a1 = in ? d1[(size_t)j * n + o] : 0.0;
                const double a2 = in ? d2[(size_t)j * n + o] : 0.0;
                d1s[j][threadIdx.x] = a1;
                tss[j][threadIdx.x] = a2 * kw[j];
                wacc[j] += a1 * kw[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int item = threadIdx.x + u * NT;
            const int r = item % TH, ja = item / TH, a = ja % FS, j = ja / FS;
            if (j < nf) {
                const double* wrow = ws + (r + a) * WW;
                const double* xrow = xs + (r + a) * WW;
                const double* drow = d1s[j] + r * TW;
                const double* trow = tss[j] + r * TW;
                double wwin[FS], xwin[FS];
#pragma unroll
                for (int b = 0; b + 1 < FS; ++b) {
                    wwin[b] = wrow[b];
                    xwin[b] = xrow[b];
                }
#pragma unroll
                for (int c = 0; c < TW; ++c) {
                    wwin[FS - 1] = wrow[c + FS - 1];
                    xwin[FS - 1] = xrow[c + FS - 1];
                    const double dd = drow[c], tt = trow[c];
#pragma unroll
                    for (int b = 0; b < FS; ++b) {
                        A1[u][b] += dd * wwin[b];
                        A2[u][b] += tt * xwin[b];
                    }
#pragma unroll
                    for (int b = 0; b + 1 < FS; ++b) {
                        wwin[b] = wwin[b + 1];
                        xwin[b] = xwin[b + 1];
                    }
                }
            }
        }
    }
    // weight terms: block sums of wacc_j
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < MAX_NF; ++j) {
        const double v = wave_sum(wacc[j]);
        if (lane == 0) wred[wave][j] = v;
    }
    // tap terms: both terms, then the 8 tile rows (lanes 8g .. 8g + 7 share (j, a))
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int item = threadIdx.x + u * NT;
        const int r = item % TH, ja = item / TH, a = ja % FS, j = ja / FS;
#pragma unroll
        for (int b = 0; b < FS; ++b) {
            const double v = group_sum(A1[u][b] + A2[u][b], 8);
            if (r == 0 && j < nf) acc_s[j * (1 + F2) + 1 + a * FS + b] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nf) {
        double v = 0.0;
        for (int q = 0; q < NWAVE; ++q) v += wred[q][threadIdx.x];
        acc_s[threadIdx.x * (1 + F2)] = v;
    }
    __syncthreads();
    double* pr = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * p;
    for (int k = threadIdx.x; k < p; k += NT) {
        const int j = k / (1 + F2);
        pr[k] = -S.lamj[j] * acc_s[k];
    }
}

// Sum the per-block records of J into G (p x ncols, column-major), optional zero-mean
// projection of each filter's tap block.
__global__ void k_jac_reduce(const double* __restrict__ part, int nblocks, int p, int ncols, double* __restrict__ G,
                             int project, int fs2) {
    const int c = blockIdx.x;
    extern __shared__ double colv[];
    for (int k = threadIdx.x; k < p; k += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += part[((size_t)c * nblocks + b) * p + k];
        colv[k] = s;
    }
    __syncthreads();
    if (project && fs2 > 0) {
        const int nfil = p / (1 + fs2);
        for (int j = threadIdx.x; j < nfil; j += blockDim.x) {
            double m = 0.0;
            for (int a = 0; a < fs2; ++a) m += colv[j * (1 + fs2) + 1 + a];
            m /= fs2;
            for (int a = 0; a < fs2; ++a) colv[j * (1 + fs2) + 1 + a] -= m;
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < p; k += blockDim.x) G[(size_t)c * p + k] = colv[k];
}

// ------------------------------------------------------------------ lower-level gradient
// grad = 2 A^T (A x - y) + [TV] lam D^T(D x / psi) | [filters] eps x + sum_j lam_j K_j^T phi'(K_j x)
// and block partials of Phi and ||grad||^2 (last block: st_out[0] = Phi, [1] = ||grad||^2).
__global__ void __launch_bounds__(NT) k_lower_grad(Stencil S, const double* __restrict__ x,
                                                   const double* __restrict__ y, double* __restrict__ grad,
                                                   double* part) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    const TileLayout L = tile_layout(S.R, S.reg, S.fs);
    const int R = S.R, E = L.E, RW = L.RW, RH = L.RH;
    int r0, c0;
    tile_origin(S, xcd_tile(blockIdx.x, gridDim.x), r0, c0);
    double* v = lds + L.o_v;
    stage_region<double>(v, S, L, r0, c0, [&](int i) { return x[i]; });
    __syncthreads();
    double* h1 = lds + L.o_h1;
    double* t1 = lds + L.o_t1;
    double* out = lds + L.o_out;
    double phi_loc = 0.0;
    const int W1 = TW + 2 * R, H1 = TH + 2 * R;
    for (int idx = threadIdx.x; idx < RH * W1; idx += NT) {
        const int rr = idx / W1, cc = idx - rr * W1;
        const double* src = v + rr * RW + cc + E - 2 * R;
        double acc = 0.0;
        for (int b = 0; b <= 2 * R; ++b) acc += S.g[b] * src[b];
        h1[idx] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < H1 * W1; idx += NT) {      // residual A x - y on tile + R
        const int rr = idx / W1, cc = idx - rr * W1;
        const double* src = h1 + (rr + E - 2 * R) * W1 + cc;
        double acc = 0.0;
        for (int a = 0; a <= 2 * R; ++a) acc += S.g[a] * src[a * W1];
        const int gi = r0 - R + rr, gj = c0 - R + cc;
        double res = 0.0;
        if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) {
            res = acc - y[gi * S.w + gj];
            if (rr >= R && rr < R + TH && cc >= R && cc < R + TW) phi_loc += res * res;
        }
        t1[idx] = res;
    }
    __syncthreads();
    double* h2 = h1;
    for (int idx = threadIdx.x; idx < H1 * TW; idx += NT) {
        const int rr = idx / TW, cc = idx - rr * TW;
        const double* src = t1 + rr * W1 + cc;
        double acc = 0.0;
        for (int b = 0; b <= 2 * R; ++b) acc += S.g[b] * src[b];
        h2[idx] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
        const int rr = idx / TW, cc = idx - rr * TW;
        const double* src = h2 + rr * TW + cc;
        double acc = 0.0;
        for (int a = 0; a <= 2 * R; ++a) acc += S.g[a] * src[a * TW];
        out[idx] = 2.0 * acc;
    }
    if (S.reg == BL_REG_TV) {
        double* fx = lds + L.o_fx;
        double* fy = lds + L.o_fy;
        const int FW = TW + 1;
        for (int idx = threadIdx.x; idx < (TH + 1) * FW; idx += NT) {
            const int rr = idx / FW, cc = idx - rr * FW;
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            double fxv = 0.0, fyv = 0.0;
            if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) {
                const double* vc = v + (rr - 1 + E) * RW + (cc - 1 + E);
                const double a = (gj < S.w - 1) ? vc[1] - vc[0] : 0.0;
                const double b = (gi < S.h - 1) ? vc[RW] - vc[0] : 0.0;
                const double psi = sqrt(a * a + b * b + S.gam2);
                fxv = a / psi;
                fyv = b / psi;
                if (rr >= 1 && cc >= 1) phi_loc += S.lam * psi;
            }
            fx[idx] = fxv;
            fy[idx] = fyv;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
            const int rr = idx / TW, cc = idx - rr * TW;
            const int f = (rr + 1) * FW + (cc + 1);
            out[idx] += S.lam * (-fx[f] + fx[f - 1] - fy[f] + fy[f - FW]);
        }
        __syncthreads();
    } else {
        const int F = L.F, fs = S.fs, TWF = TW + 2 * F, THF = TH + 2 * F;
        double* tb = lds + L.o_t;
        for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
            const int rr = idx / TW, cc = idx - rr * TW;
            const double xv = v[(rr + E) * RW + (cc + E)];
            out[idx] += S.eps * xv;
            if (r0 + rr < S.h && c0 + cc < S.w) phi_loc += 0.5 * S.eps * xv * xv;
        }
        __syncthreads();
        for (int j = 0; j < S.nf; ++j) {
            const double* kj = S.taps + j * fs * fs;
            const double lj = S.lamj[j];
            for (int idx = threadIdx.x; idx < THF * TWF; idx += NT) {
                const int rr = idx / TWF, cc = idx - rr * TWF;
                const int gi = r0 - F + rr, gj = c0 - F + cc;
                double val = 0.0;
                if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) {
                    const double* src = v + (rr + E - 2 * F) * RW + (cc + E - 2 * F);
                    double sresp = 0.0;
                    for (int a = 0; a < fs; ++a)
                        for (int b = 0; b < fs; ++b) sresp += kj[a * fs + b] * src[a * RW + b];
                    if (S.penalty == BL_PEN_LOG) {
                        val = 2.0 * sresp / (1.0 + sresp * sresp);
                        if (rr >= F && rr < F + TH && cc >= F && cc < F + TW) phi_loc += lj * log1p(sresp * sresp);
                    } else {
                        val = 2.0 * sresp;
                        if (rr >= F && rr < F + TH && cc >= F && cc < F + TW) phi_loc += lj * sresp * sresp;
                    }
                }
                tb[idx] = val;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
                const int rr = idx / TW, cc = idx - rr * TW;
                const double* src = tb + (rr + 2 * F) * TWF + (cc + 2 * F);
                double acc = 0.0;
                for (int a = 0; a < fs; ++a)
                    for (int b = 0; b < fs; ++b) acc += kj[a * fs + b] * src[-a * TWF - b];
                out[idx] += lj * acc;
            }
            __syncthreads();
        }
    }
    double gn = 0.0;
    for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
        const int gi = r0 + idx / TW, gj = c0 + idx % TW;
        if (gi < S.h && gj < S.w) {
            grad[gi * S.w + gj] = out[idx];
            gn += out[idx] * out[idx];
        }
    }
    block_partials(part, 2, [&](int k) { return k == 0 ? phi_loc : gn; });
}

// ------------------------------------------------------------------ y = A x + noise e
__global__ void __launch_bounds__(NT) k_forward(Stencil S, const double* __restrict__ x, const double* __restrict__ e,
                                                double noise, double* __restrict__ y) {
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i >= S.n) return;
    const int gi = i / S.w, gj = i - gi * S.w, R = S.R;
    double acc = 0.0;
    for (int a = -R; a <= R; ++a) {
        const int ii = gi + a;
        if (ii < 0 || ii >= S.h) continue;
        double row = 0.0;
        for (int b = -R; b <= R; ++b) {
            const int jj = gj + b;
            if (jj < 0 || jj >= S.w) continue;
            row += S.g[b + R] * x[ii * S.w + jj];
        }
        acc += S.g[a + R] * row;
    }
    y[i] = acc + noise * e[i];
}

// ------------------------------------------------------------------ launchers
// Dynamic LDS above 64 KiB (large blur radii) must be enabled per kernel.
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static inline dim3 tiles_grid(const Stencil& S, int ncols) { return dim3(S.tiles_x * S.tiles_y, ncols); }
int tiles_of(const Stencil& S) { return S.tiles_x * S.tiles_y; }

// Kernels are instantiated per blur radius (0..MAX_R) and arithmetic type.
hipError_t launch_hvp(const Stencil& S, bool fp32, const double* xhat, const double* v, double* out, int ncols,
                      int rows, hipStream_t st) {
    switch (rows) {
        case QTY * 1: return launch_hvp_q<1>(S, fp32, xhat, v, out, ncols, st);
        case QTY * 2: return launch_hvp_q<2>(S, fp32, xhat, v, out, ncols, st);
        case QTY * 4: return launch_hvp_q<4>(S, fp32, xhat, v, out, ncols, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_filter_state(const Stencil& S, const double* xhat, double* d1, double* d2, float* d2f,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_filter_state, dim3((S.n + NT - 1) / NT, S.nf), dim3(NT), 0, stream, S, xhat, d1, d2, d2f);
    return hipGetLastError();
}

int jac_blocks(const Stencil& S) {
    if (S.reg == BL_REG_TV) return (S.n + NT * 8 - 1) / (NT * 8) < 256 ? (S.n + NT * 8 - 1) / (NT * 8) : 256;
    const int ntiles = S.tiles_x * S.tiles_y;
    return ntiles < JF_BLOCKS ? ntiles : JF_BLOCKS;
}

hipError_t launch_jac(const Stencil& S, const double* xhat, const double* w, int ncols, const double* d1,
                      const double* d2, double* part, double* G, int project, hipStream_t stream) {
    const int nb = jac_blocks(S);
    int p;
    if (S.reg == BL_REG_TV) {
        p = 2;
        hipLaunchKernelGGL(k_jac_tv, dim3(nb, ncols), dim3(NT), 0, stream, S, xhat, w, part);
    } else {
        p = S.nf * (1 + S.fs * S.fs);
        const dim3 grid(nb, ncols);
        switch (S.fs) {
            case 1: hipLaunchKernelGGL(k_jac_filters<1>, grid, dim3(NT), 0, stream, S, xhat, w, d1, d2, part); break;
            case 3: hipLaunchKernelGGL(k_jac_filters<3>, grid, dim3(NT), 0, stream, S, xhat, w, d1, d2, part); break;
            case 5: hipLaunchKernelGGL(k_jac_filters<5>, grid, dim3(NT), 0, stream, S, xhat, w, d1, d2, part); break;
            case 7: hipLaunchKernelGGL(k_jac_filters<7>, grid, dim3(NT), 0, stream, S, xhat, w, d1, d2, part); break;
            default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int fs2 = S.reg == BL_REG_TV ? 0 : S.fs * S.fs;
    hipLaunchKernelGGL(k_jac_reduce, dim3(ncols), dim3(NT), p * sizeof(double), stream, part, nb, p, ncols, G, project,
                       fs2);
    return hipGetLastError();
}

hipError_t launch_lower_grad(const Stencil& S, const double* x, const double* y, double* grad, double* part,
                             hipStream_t stream) {
    allow_lds(k_lower_grad, tile_lds_bytes<double>(S.R, S.reg, S.fs));
    hipLaunchKernelGGL(k_lower_grad, tiles_grid(S, 1), dim3(NT), tile_lds_bytes<double>(S.R, S.reg, S.fs), stream, S,
                       x, y, grad, part);
    return hipGetLastError();
}

hipError_t launch_forward(const Stencil& S, const double* x, const double* e, double noise, double* y,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_forward, dim3((S.n + NT - 1) / NT), dim3(NT), 0, stream, S, x, e, noise, y);
    return hipGetLastError();
}

}  // namespace bl
