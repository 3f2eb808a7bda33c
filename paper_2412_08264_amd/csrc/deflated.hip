// Deflated CG (Saad, Yeung, Erhel and Guyomarc'h, 2000) for one Hessian system in FP64, with the
// refresh's recycle space U and C = H U as the deflation space: the reading of the recycled
// solver beside the Galerkin form of the batch kernels (Section 2.2.2 defines only RMINRES).
// With E = U^T C (symmetric positive definite, inverted once per solve):
//   set-up:  r = g - H w0;  c = E^{-1} U^T r;  w = w0 + U c;  r -= C c          (U^T r = 0)
//   step j:  mu_j = E^{-1} C^T r_j;  p_j = r_j + beta_{j-1} p_{j-1} - U mu_j;  q_j = H p_j;
//            alpha_j = rho_j / (p_j . q_j);  w += alpha_j p_j;  r -= alpha_j q_j.
// Two launches per step, no grid synchronisation (per-block records reduced by the next launch):
//   apply  (tiles of 32 x 8)  rho_j, C^T r_j (and Z^T r_j on tested iterations) from the update's
//                             records; the stop test of iterate j; beta; mu_j; the stencil input
//                             y = r_j + beta p_{j-1} on the tile and its halo (no column of U is
//                             read there: H p_j = H y - C mu_j, p_j = y - U mu_j at the thread's
//                             own pixel); record [p_j . q_j].
//   update (pixel blocks)     alpha_j; w += alpha_j p_j; r -= alpha_j q_j; record [r . r, C^T r,
//                             Z^T r when the next test evaluates the error estimate].
// Per step the columns of U and C are read once each in the apply and C once more in the update.
#include "batch_tile.h"

namespace bl {

__device__ __forceinline__ void d_tile_origin(const Stencil& S, int& r0, int& c0) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    r0 = (t / S.tiles_x) * QTY;
    c0 = (t % S.tiles_x) * QW;
}

// ------------------------------------------------------------------ r = g - H w; record [g.g, U^T r]
template <int R, int CLS>
__global__ void __launch_bounds__(NT) k_d_residual(Stencil S, DeflArgs a) {
    using L = QLayout<double, R, CLS, 1>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    int r0, c0;
    d_tile_origin(S, r0, c0);
    const Own<1> o = own_pixels<1>(S.h, S.w, r0, c0);
    const double gv = o.in[0] ? a.g[o.g[0]] : 0.0;
    q_stage<double, R, CLS, 1>(lds + L::o_v, S.h, S.w, r0, c0, [&](int gi) { return a.w[gi]; });
    const TvX<1> X = tv_x<CLS, 1>(S.h, S.w, a.xhat, r0, c0);
    __syncthreads();
    double hv[1];
    q_hvp<double, R, CLS, 1>(lds, S, r0, c0, hv, X);
    const double rv = o.in[0] ? gv - hv[0] : 0.0;
    if (o.in[0]) a.r[o.g[0]] = rv;
    block_partials(a.rec_res, 1 + a.s, [&](int k) -> double {
        if (!o.in[0]) return 0.0;
        return k == 0 ? gv * gv : a.U[(size_t)(k - 1) * S.n + o.g[0]] * rv;
    });
}

// ------------------------------------------------------------------ E^{-1}
// Einv = (sym(U^T C))^{-1} from the Gram product UtC (s x s), one workgroup: Cholesky by one
// thread (s <= 64), then one column of the inverse per thread.  A non-positive pivot sets
// info[0] = BL_E_INDEFINITE.
__global__ void __launch_bounds__(NT) k_d_einv(int s, const double* __restrict__ UtC, double* __restrict__ L,
                                               double* __restrict__ Einv, int* __restrict__ info) {
    __shared__ int ok;
    if (threadIdx.x == 0) {
        ok = 1;
        for (int j = 0; j < s && ok; ++j)
            for (int i = j; i < s; ++i) {
                double v = 0.5 * (UtC[(size_t)j * s + i] + UtC[(size_t)i * s + j]);
                for (int k = 0; k < j; ++k) v -= L[(size_t)k * s + i] * L[(size_t)k * s + j];
                if (i == j) {
                    if (!(v > 0.0)) {
                        ok = 0;
                        break;
                    }
                    L[(size_t)j * s + j] = sqrt(v);
                } else {
                    L[(size_t)j * s + i] = v / L[(size_t)j * s + j];
                }
            }
        info[0] = ok ? BL_OK : BL_E_INDEFINITE;
    }
    __syncthreads();
    if (!ok) return;
    for (int c = threadIdx.x; c < s; c += NT) {   // solve L L^T x = e_c into column c
        double* x = Einv + (size_t)c * s;
        for (int i = 0; i < s; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[(size_t)k * s + i] * x[k];
            x[i] = v / L[(size_t)i * s + i];
        }
        for (int i = s - 1; i >= 0; --i) {
            double v = x[i];
            for (int k = i + 1; k < s; ++k) v -= L[(size_t)i * s + k] * x[k];
            x[i] = v / L[(size_t)i * s + i];
        }
    }
}

// ------------------------------------------------------------------ set-up
// c = E^{-1} U^T r (records of the residual launch), w += U c, r -= C c; settings into the state;
// record [r.r, C^T r, Z^T r] (iterate 0 is always tested).
__global__ void __launch_bounds__(NT) k_d_init(DeflArgs a, StateInit in, int fold) {
    __shared__ double tot[NT];
    __shared__ double cv[S_MAX];
    const int s = a.s, n = a.n;
    reduce_partials(fold ? a.fold : a.rec_res, fold ? FOLD_BLOCKS : a.ntiles, 1 + s, tot);
    for (int k = threadIdx.x; k < s; k += NT) {
        double v = 0.0;
        for (int q = 0; q < s; ++q) v += a.Einv[(size_t)q * s + k] * tot[1 + q];
        cv[k] = v;
    }
    SolveState* st = a.st;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 0;
        st->status = BL_OK;
        st->iters = 0;
        st->gnorm = sqrt(tot[0]);
        st->tol = in.tol;
        st->hg_tol = in.hg_tol;
        st->max_iter = in.max_iter;
        st->check_every = in.check_every;
        st->stop = in.stop;
        st->s = in.s;
        st->v_cap = in.v_cap;
        st->store_basis = in.store_basis;
        st->hgerr_on = in.hgerr_on;
        st->est = NAN;
    }
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < S_MAX; k += NT) st->mu[k] = (k < s && a.mu) ? a.mu[k] : 0.0;
    __syncthreads();
    const int i = blockIdx.x * NT + threadIdx.x;
    const bool inb = i < n;
    double ri = 0.0;
    if (inb) {
        a.w[i] += combo(a.U, n, i, cv, s);
        ri = a.r[i] - combo(a.C, n, i, cv, s);
        a.r[i] = ri;
    }
    block_partials(a.rec_upd, 1 + s + a.nz, [&](int k) -> double {
        if (!inb) return 0.0;
        if (k == 0) return ri * ri;
        if (k <= s) return a.C[(size_t)(k - 1) * n + i] * ri;
        return a.Z[(size_t)(k - 1 - s) * n + i] * ri;
    });
}

// ------------------------------------------------------------------ apply, step j
// `zw` values of Z^T r_j in the update records (0 or nz); `fold`: those records were folded.
template <int R, int CLS>
__global__ void __launch_bounds__(NT) k_d_apply(Stencil S, DeflArgs a, int j, int zw, int fold) {
    using L = QLayout<double, R, CLS, 1>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    __shared__ double tot[NT];
    __shared__ double mus[S_MAX];
    __shared__ int sdone;
    SolveState* st = a.st;
    if (threadIdx.x == 0) sdone = st->done;
    int r0, c0;
    d_tile_origin(S, r0, c0);
    const Own<1> o = own_pixels<1>(S.h, S.w, r0, c0);
    const int n = S.n, s = a.s;
    const double* __restrict__ p_old = a.p[(j + 1) & 1];
    double* __restrict__ p_new = a.p[j & 1];
    const TestSettings ts = test_settings(st);
    const double rho_prev = j > 0 ? uni(st->rho2[(j - 1) & 1]) : 1.0;
    const double mu_lane = mu_of_lane(st, ts.s);
    reduce_partials(fold ? a.fold : a.rec_upd, fold ? FOLD_BLOCKS : a.npix, 1 + s + zw, tot);
    if (sdone) return;
    const double rho = tot[0];
    const Decision dec = decide(ts, j, rho, tot + 1 + s, zw > 0, mu_lane);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho2[j & 1] = rho;
        if (zw) st->est = dec.est;
        st->iters = j;
        if (j == 0) st->res0 = sqrt(rho);
        if (dec.done) {
            st->status = dec.status;
            st->done = 1;
        }
    }
    if (dec.done) return;
    const double beta = j == 0 ? 0.0 : rho / rho_prev;
    for (int k = threadIdx.x; k < s; k += NT) {   // mu_j = E^{-1} C^T r_j
        double v = 0.0;
        for (int q = 0; q < s; ++q) v += a.Einv[(size_t)q * s + k] * tot[1 + q];
        mus[k] = v;
    }
    q_stage<double, R, CLS, 1>(lds + L::o_v, S.h, S.w, r0, c0,
                               [&](int gi) { return j == 0 ? a.r[gi] : a.r[gi] + beta * p_old[gi]; });
    const TvX<1> X = tv_x<CLS, 1>(S.h, S.w, a.xhat, r0, c0);
    __syncthreads();
    const double yi = o.in[0] ? (j == 0 ? a.r[o.g[0]] : a.r[o.g[0]] + beta * p_old[o.g[0]]) : 0.0;
    const double ri = o.in[0] ? a.r[o.g[0]] : 0.0;
    double hv[1];
    q_hvp<double, R, CLS, 1>(lds, S, r0, c0, hv, X);
    double pi = 0.0, qi = 0.0;
    if (o.in[0]) {
        pi = yi - combo(a.U, n, o.g[0], mus, s);
        qi = hv[0] - combo(a.C, n, o.g[0], mus, s);
        p_new[o.g[0]] = pi;
        a.q[o.g[0]] = qi;
        if (uni(st->store_basis) && j < uni(st->v_cap))
            a.V[(size_t)j * n + o.g[0]] = ri / sqrt(rho);
    }
    block_partials(a.rec_app, 1, [&](int) -> double { return pi * qi; });
}

// ------------------------------------------------------------------ update, step j
// `zw` values of Z^T r_{j+1} go into this launch's record (0 or nz); `fold`: the apply records
// were folded.
__global__ void __launch_bounds__(NT) k_d_update(DeflArgs a, int j, int zw, int fold) {
    __shared__ double tot[NT];
    __shared__ int sdone;
    SolveState* st = a.st;
    if (threadIdx.x == 0) sdone = st->done;
    const int s = a.s, n = a.n;
    const int i = blockIdx.x * NT + threadIdx.x;
    const bool inb = i < n;
    const double* __restrict__ p = a.p[j & 1];
    const double rho = uni(st->rho2[j & 1]);
    reduce_partials(fold ? a.fold : a.rec_app, fold ? FOLD_BLOCKS : a.ntiles, 1, tot);
    if (sdone) return;
    const double sigma = tot[0];
    if (!(sigma > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->status = (sigma != sigma || fabs(sigma) == INFINITY) ? BL_E_NONFINITE : BL_E_INDEFINITE;
            st->iters = j;
            st->done = 1;
        }
        return;
    }
    const double alpha = rho / sigma;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->alpha = alpha;
    double ri = 0.0;
    if (inb) {
        a.w[i] += alpha * p[i];
        ri = a.r[i] - alpha * a.q[i];
        a.r[i] = ri;
    }
    block_partials(a.rec_upd, 1 + s + zw, [&](int k) -> double {
        if (!inb) return 0.0;
        if (k == 0) return ri * ri;
        if (k <= s) return a.C[(size_t)(k - 1) * n + i] * ri;
        return a.Z[(size_t)(k - 1 - s) * n + i] * ri;
    });
}

// ------------------------------------------------------------------ launchers
hipError_t launch_d_residual(const Stencil& S, const DeflArgs& a, hipStream_t stream) {
    q_dispatch(S.R, tile_class(S.reg, S.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        const size_t lds = QLayout<double, RR, CC, 1>::bytes;
        allow_lds_b(k_d_residual<RR, CC>, lds);
        hipLaunchKernelGGL((k_d_residual<RR, CC>), dim3(a.ntiles), dim3(NT), lds, stream, S, a);
    });
    return hipGetLastError();
}

hipError_t launch_d_einv(int s, const double* UtC, double* Lscr, double* Einv, int* info, hipStream_t stream) {
    hipLaunchKernelGGL(k_d_einv, dim3(1), dim3(NT), 0, stream, s, UtC, Lscr, Einv, info);
    return hipGetLastError();
}

hipError_t launch_d_init(const DeflArgs& a, const StateInit& in, bool fold, hipStream_t stream) {
    hipLaunchKernelGGL(k_d_init, dim3(a.npix), dim3(NT), 0, stream, a, in, (int)fold);
    return hipGetLastError();
}

hipError_t launch_d_apply(const Stencil& S, const DeflArgs& a, int j, int zw, bool fold, hipStream_t stream) {
    q_dispatch(S.R, tile_class(S.reg, S.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        const size_t lds = QLayout<double, RR, CC, 1>::bytes;
        allow_lds_b(k_d_apply<RR, CC>, lds);
        hipLaunchKernelGGL((k_d_apply<RR, CC>), dim3(a.ntiles), dim3(NT), lds, stream, S, a, j, zw, (int)fold);
    });
    return hipGetLastError();
}

hipError_t launch_d_update(const DeflArgs& a, int j, int zw, bool fold, hipStream_t stream) {
    hipLaunchKernelGGL(k_d_update, dim3(a.npix), dim3(NT), 0, stream, a, j, zw, (int)fold);
    return hipGetLastError();
}

}  // namespace bl
