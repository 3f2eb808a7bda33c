// Tile-grid kernels of the batched recycled CG (residual and apply), templated on the rows
// per thread Q of the Hessian-vector tile (tiles of 32 x 8Q pixels) and on whether the solves
// of the launch have a recycle space (REC; plain CG launches carry no projection code), with
// the device helpers the batch kernels share.  Each tile height is instantiated in a
// translation unit of its own.
#pragma once

#include <type_traits>

#include "kernels.h"
#include "tile.h"

namespace bl {

__device__ __forceinline__ void slot_stencil(Stencil& S, const Slot& sl) {
    S.h = sl.h;
    S.w = sl.width;
    S.n = sl.n;
    S.tiles_x = sl.tiles_x;
    S.lam = sl.lam;
    S.gam2 = sl.gam2;
    S.taps = sl.taps;
    S.tapsf = sl.tapsf;
    S.lamj = sl.lamj;
    S.d2 = sl.d2;
    S.d2f = sl.d2f;
}

template <int Q>
__device__ __forceinline__ void slot_tile(const Slot& sl, int local, int& r0, int& c0) {
    const int t = xcd_tile(local, sl.ntiles);
    r0 = (t / sl.tiles_x) * (QTY * Q);
    c0 = (t % sl.tiles_x) * QW;
}

// The thread's Q pixels: rows r0 + Q ty + k of column c0 + tx.
template <int Q>
struct Own {
    int g[Q];
    bool in[Q];
};
template <int Q>
__device__ __forceinline__ Own<Q> own_pixels(int h, int w, int r0, int c0) {
    Own<Q> o;
    const int tx = threadIdx.x & (QW - 1), ty = threadIdx.x / QW, gj = c0 + tx;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int gi = r0 + Q * ty + k;
        o.in[k] = gi < h && gj < w;
        o.g[k] = o.in[k] ? gi * w + gj : 0;
    }
    return o;
}

// Records a consumer reads: the producer's per-block array, or its folded record.
__device__ __forceinline__ const double* slot_rec(const Slot& sl, int which, int& nb) {
    if (which == 0) {
        nb = sl.fold_res ? FOLD_BLOCKS : sl.ntiles;
        return sl.fold_res ? sl.fold : sl.rec_res;
    }
    if (which == 1) {
        nb = sl.fold_app ? FOLD_BLOCKS : sl.ntiles;
        return sl.fold_app ? sl.fold + FOLD_BLOCKS * NV_RED : sl.rec_app;
    }
    nb = sl.fold_upd ? FOLD_BLOCKS : sl.npix;
    return sl.fold_upd ? sl.fold + 2 * FOLD_BLOCKS * NV_RED : sl.rec_upd;
}

// ------------------------------------------------------------------ residual g - H w
// r = g - H w in FP64 and the record [g.g, C^T r].  With `periodic` set (a scheduled
// residual replacement) a slot that has already stopped is left alone.
template <int R, int CLS, int Q, bool REC>
__global__ void __launch_bounds__(NT) k_b_residual(Stencil base, const Slot* __restrict__ slots, BatchMap M,
                                                   int periodic) {
    using L = QLayout<double, R, CLS, Q>;
    constexpr int QR = Q;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    const int2 m = map_block(M, blockIdx.x);
    const Slot& sl = slots[m.x];
    if (m.y >= sl.ntiles || (periodic && sl.st->done)) return;
    Stencil S = base;
    slot_stencil(S, sl);
    int r0, c0;
    slot_tile<Q>(sl, m.y, r0, c0);
    const Own<Q> o = own_pixels<Q>(S.h, S.w, r0, c0);
    double gv[QR];
#pragma unroll
    for (int k = 0; k < QR; ++k) gv[k] = o.in[k] ? sl.g[o.g[k]] : 0.0;
    q_stage<double, R, CLS, Q>(lds + L::o_v, S.h, S.w, r0, c0, [&](int gi) { return sl.w[gi]; });
    const TvX<Q> X = tv_x<CLS, Q>(S.h, S.w, sl.xhat, r0, c0);
    __syncthreads();
    double hv[QR];
    q_hvp<double, R, CLS, Q>(lds, S, r0, c0, hv, X);
    double ov[QR];
#pragma unroll
    for (int k = 0; k < QR; ++k) {
        ov[k] = o.in[k] ? gv[k] - hv[k] : 0.0;
        if (o.in[k]) sl.r[o.g[k]] = ov[k];
    }
    block_partials_in(reinterpret_cast<double*>(smem_raw),
        sl.rec_res, REC ? 1 + sl.s : 1,
        [&](int k) {
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < QR; ++u)
                if (o.in[u]) acc += k == 0 ? gv[u] * gv[u] : sl.C[(size_t)(k - 1) * S.n + o.g[u]] * ov[u];
            return acc;
        },
        m.y);
}

// Iteration j = step - j0, first half: stop test from the update records, beta, p, q = H p,
// V store, record [p.q, C^T q].  After a residual replacement whose true residual exceeds the
// previous recursive one the direction restarts (p = r): keeping it would let the stale
// direction dominate (beta = rho_true / rho_rec >> 1) and stall at the accuracy of the FP32
// operator; restarting turns the replacement into a step of iterative refinement.
// A slot stopped by an earlier launch leaves before its record reduction (stopped_before);
// one stopped by this launch's decision leaves after it, as every block takes that decision.
// TV on short tiles (8 or 16 rows, the small images, where latency decides): the loads that
// do not depend on the scalars of this iteration (the thread's r, p and columns of C, the halo
// of r and p, x_hat) are issued before the record reduction, so their latency overlaps it; the
// stencil input r + beta p is formed from registers afterwards.  Filters: the first columns
// of C (about 20 values per thread) are loaded before the stencil, whose arithmetic then
// hides them (measured: 7-13% per iteration over loading them after the stencil).
template <int CLS, int Q, bool REC>
__host__ __device__ constexpr int c_prefetch() {
    return !REC ? 1 : (CLS != TC_TV ? (Q == 1 ? 20 : (Q == 2 ? 10 : 5)) : (Q == 1 ? 24 : (Q == 2 ? 10 : 8)));
}

template <typename T, int R, int CLS, int Q, bool REC>
__global__ void __launch_bounds__(NT) k_b_apply(Stencil base, const Slot* __restrict__ slots, BatchMap M,
                                                StepRef sr) {
    using L = QLayout<T, R, CLS, Q>;
    using G = QGeo<R, CLS, Q>;
    constexpr int QR = Q;
    constexpr bool EARLY = CLS == TC_TV && Q < 4;   // (tall tiles: registers would cost occupancy)
    constexpr int CP = c_prefetch<CLS, Q, REC>();
    constexpr int NST = EARLY ? (G::N_V + NT - 1) / NT : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    __shared__ double tot[NT];
    const int2 m = map_block(M, blockIdx.x);
    const Slot& sl = slots[m.x];
    if (m.y >= sl.ntiles) return;
    SolveState* st = sl.st;
    const int mark = stop_mark(st);
    const int step = step_of(sr), j = step - sl.j0;
    const int s = REC ? sl.s : 0, nz = REC ? sl.nz : 0;
    const int h = sl.h, w = sl.width, n = sl.n;
    const gbl_t<const double> __restrict__ r = gbl((const double*)sl.r);
    const gbl_t<const double> __restrict__ p_old = gbl((const double*)sl.p[j & 1]);
    const gbl_t<double> __restrict__ p_new = gbl(sl.p[(j + 1) & 1]);
    const gbl_t<const double> gC = gbl(sl.C);
    int r0, c0;
    slot_tile<Q>(sl, m.y, r0, c0);
    const Own<Q> o = own_pixels<Q>(h, w, r0, c0);
    // p_old is read whatever the iteration and selected away below when the direction restarts
    double ri[QR], pr[QR], cpre[CP][QR], hr[NST], hp[NST];
    TvX<Q> X{};
#pragma unroll
    for (int k = 0; k < QR; ++k) {
        ri[k] = o.in[k] ? r[o.g[k]] : 0.0;
        pr[k] = o.in[k] ? p_old[o.g[k]] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CP; ++c)
#pragma unroll
        for (int k = 0; k < QR; ++k) cpre[c][k] = (o.in[k] && c < s) ? gC[(size_t)c * n + o.g[k]] : 0.0;
    if constexpr (EARLY) {
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = threadIdx.x + u * NT;
            hr[u] = hp[u] = 0.0;
            if (idx < G::N_V) {
                const int rr = idx / G::RW, cc = idx - rr * G::RW;
                const int gi = r0 - G::E + rr, gj = c0 - G::E + cc;
                if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
                    hr[u] = r[gi * w + gj];
                    hp[u] = p_old[gi * w + gj];
                }
            }
        }
    }
    int nb;
    const double* rec = slot_rec(sl, 2, nb);
    // scalars written by earlier launches, read before the reduction so that nothing after it
    // waits on them
    const gbl_t<const SolveState> sg = gbl((const SolveState*)st);
    const TestSettings ts = test_settings(st);
    const int zw = REC ? zr_width(ts.check_every, nz, j) : 0;
    const double rho_prev = j > 0 ? uni(sg->rho2[(j - 1) & 1]) : 1.0;
    const bool store_basis = uni(sg->store_basis) && j >= 0 && j < uni(sg->v_cap);
    const int rr_j = uni(sg->rr_j);
    const double mu_lane = REC ? mu_of_lane(st, ts.s) : 0.0;
    if (stopped_before(mark, step)) return;
    reduce_partials(rec, nb, 1 + zw, tot);
    const double rho = tot[0];
    const bool restart = j > 0 && rr_j == j && rho > rho_prev;
    const Decision dec = decide(ts, j, rho, tot + 1, zw > 0, mu_lane);
    if (m.y == 0) {
        for (int k = threadIdx.x; k < zw; k += NT) st->zr[k] = tot[1 + k];
        if (threadIdx.x == 0) {
            st->rho2[j & 1] = rho;
            if (store_basis && sl.lz) sl.lz[2 * j + 1] = rho;
            if (zw) st->est = dec.est;
            st->iters = j;
            if (j == 0) st->res0 = sqrt(rho);
            if (dec.done) {
                st->status = dec.status;
                st->done = 1;
                st->stop_at = step + 1;
            }
        }
    }
    if (dec.done) return;
    // x_hat for the flux blocks: read after the decision, held through the first pass only
    if constexpr (EARLY) X = tv_xload<Q>(h, w, sl.xhat, r0, c0);
    Stencil S = base;
    slot_stencil(S, sl);
    const bool first = (j == 0) || restart;
    const double beta = first ? 0.0 : rho / rho_prev;
    double pi[QR];
#pragma unroll
    for (int k = 0; k < QR; ++k) pi[k] = first ? 0.0 : pr[k];
    if constexpr (EARLY) {
        T* v = lds + L::o_v;
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = threadIdx.x + u * NT;
            if (idx < G::N_V) v[idx] = (T)(first ? hr[u] : hr[u] + beta * hp[u]);
        }
    } else {
        q_stage<T, R, CLS, Q>(lds + L::o_v, S.h, S.w, r0, c0,
                              [&](int g) { return first ? r[g] : r[g] + beta * p_old[g]; });
        if constexpr (CLS == TC_TV) X = tv_xload<Q>(h, w, sl.xhat, r0, c0);
    }
    __syncthreads();
    T hv[QR];
    q_hvp<T, R, CLS, Q>(lds, S, r0, c0, hv, X);
    double pv[QR], qq[QR];
    const double inv = store_basis ? 1.0 / sqrt(rho) : 0.0;
#pragma unroll
    for (int k = 0; k < QR; ++k) {
        const double pn = first ? ri[k] : ri[k] + beta * pi[k];
        qq[k] = o.in[k] ? (double)hv[k] : 0.0;
        pv[k] = o.in[k] ? pn : 0.0;
        if (o.in[k]) {
            p_new[o.g[k]] = pn;
            gbl(sl.q)[o.g[k]] = qq[k];
            if (store_basis) gbl(sl.V)[(size_t)j * S.n + o.g[k]] = ri[k] * inv;
        }
    }
    block_partials_in(reinterpret_cast<double*>(smem_raw),
        sl.rec_app, 1 + s,
        [&](int k) {
            double acc = 0.0;
            if (k == 0) {
#pragma unroll
                for (int u = 0; u < QR; ++u) acc += pv[u] * qq[u];
                return acc;
            }
            const int c = k - 1;
            if (c < CP) {
#pragma unroll
                for (int cc = 0; cc < CP; ++cc)
                    if (cc == c) {
#pragma unroll
                        for (int u = 0; u < QR; ++u) acc += cpre[cc][u] * qq[u];
                    }
            } else {
#pragma unroll
                for (int u = 0; u < QR; ++u)
                    if (o.in[u]) acc += gC[(size_t)c * S.n + o.g[u]] * qq[u];
            }
            return acc;
        },
        m.y);
}

// ------------------------------------------------------------------ fused FP64 step
// One launch per iteration of the recycled CG of an FP64 solve (Chronopoulos and Gear's
// single-reduction form of CG, with the residual norm recomputed each step).  Launch j:
//   j = 0   the set-up's records [r_0.r_0, Z^T r_0]: the test of iterate 0; p_0 = r_0, q_0 = H p_0.
//   j >= 1  the records of launch j - 1 [sigma, rho, r.q, q.q, e = C^T q, Z^T r] (all of iterate
//           j - 1): the test of iterate j - 1 (from j = 2; launch 0 tested iterate 0), then
//           alpha = rho / sigma, the projected residual's norm from the recurrence
//           rho^ = rho - 2 alpha (r.q) + alpha^2 (q.q - e.e)   (C^T r = 0, C^T C = I),
//           beta = rho^ / rho; on the own pixels r_j = r - alpha (q - C e), w += alpha p,
//           p_j = r_j + beta p; the stencil input y = r - alpha q + beta p on the tile and its
//           halo (p_j = y + alpha C e, so H p_j = H y + alpha (H C) e with H C formed once per
//           solve: no column of C is read on the halo), q_j = H y + alpha (H C e) on the own pixels.
//   record  [p_j.q_j, r_j.r_j, r_j.q_j, q_j.q_j, C^T q_j, Z^T r_j when iterate j is tested], in the
//           record buffer of j's parity: launch j + 1 reads them while writing the other.
// C^T q_j = C^T (H y) + alpha (C^T H C) e: the blocks reduce C^T (H y) from the stencil output, and
// block 0 adds alpha M e with M = C^T H C (s x s, formed with H C), so each column of C and of
// H C is read once per launch, in rounds of a few columns (no column is held in registers
// across the stencil, except the first few, loaded before the record reduction on 8-row tiles).
// alpha uses the explicit r.r of the previous launch, and so does every test: the recurrence
// only enters beta.  r, q and p alternate between two buffers by iteration parity; stored
// basis columns and CG coefficients of iterate j - 1 are written by launch j.
template <int CLS, int Q>
__host__ __device__ constexpr int f_prefetch() {
    return Q == 1 ? (CLS == TC_TV ? 16 : 8) : 0;
}

// ONE: a launch of a single solve, whose descriptor comes by value with the kernel arguments
// (loaded with them, instead of from the descriptor array after the block's slot is known).
template <int R, int CLS, int Q, bool REC, bool ONE>
__global__ void __launch_bounds__(NT) k_f_step(Stencil base, const Slot* __restrict__ slots, BatchMap M,
                                               StepRef sr, Slot one) {
    using L = QLayout<double, R, CLS, Q>;
    using G = QGeo<R, CLS, Q>;
    constexpr int QR = Q;
    constexpr bool EARLY = CLS == TC_TV && Q < 4;
    constexpr int PF = REC ? f_prefetch<CLS, Q>() : 0;   // columns of C and H C loaded up front
    constexpr int PFA = PF > 0 ? PF : 1;
    constexpr int CH = Q == 1 ? 8 : (Q == 2 ? 4 : 2);      // columns per later round of loads
    constexpr int NST = EARLY ? (G::N_V + NT - 1) / NT : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    __shared__ double tot[NT];
    const int2 m = ONE ? make_int2(M.slot[0], (int)blockIdx.x) : map_block(M, blockIdx.x);
    const Slot& sl = ONE ? one : slots[m.x];
    if (m.y >= sl.ntiles) return;
    SolveState* st = sl.st;
    const int mark = stop_mark(st);
    const int step = step_of(sr), j = step - sl.j0;
    const int s = REC ? sl.s : 0, nz = REC ? sl.nz : 0;
    const int h = sl.h, w = sl.width, n = sl.n;
    const bool first = j == 0;
    const gbl_t<const double> __restrict__ r0b = gbl((j & 1) ? sl.r : sl.r2);   // iterate j - 1 (j >= 1)
    const gbl_t<const double> __restrict__ q0b = gbl((j & 1) ? sl.q : sl.q2);
    const gbl_t<const double> __restrict__ p0b = gbl(sl.p[(j + 1) & 1]);
    const gbl_t<double> __restrict__ r1b = gbl((j & 1) ? sl.r2 : sl.r);          // iterate j
    const gbl_t<double> __restrict__ q1b = gbl((j & 1) ? sl.q2 : sl.q);
    const gbl_t<double> __restrict__ p1b = gbl(sl.p[j & 1]);
    const gbl_t<const double> __restrict__ rin = first ? gbl(sl.r) : r0b;
    const gbl_t<const double> gC = gbl(sl.C), gHC = gbl(sl.HC), gM = gbl(sl.M), gZ = gbl(sl.Z);
    const gbl_t<double> gW = gbl(sl.w), gV = gbl(sl.V), gLZ = gbl(sl.lz);
    int r0, c0;
    slot_tile<Q>(sl, m.y, r0, c0);
    const Own<Q> o = own_pixels<Q>(h, w, r0, c0);
    double ri[QR], qi[QR], pi[QR], wi[QR], cpre[PFA][QR], hpre[PFA][QR], hr[NST], hq[NST], hp[NST];
    TvX<Q> X{};
    // the columns of C and H C do not depend on the step index: issued first, they need not wait
    // for the step counter (H C enters only through alpha e, zero at j = 0)
#pragma unroll
    for (int c = 0; c < PFA; ++c)
#pragma unroll
        for (int k = 0; k < QR; ++k) {
            const bool ld = PF > 0 && o.in[k] && c < s;
            cpre[c][k] = ld ? gC[(size_t)c * n + o.g[k]] : 0.0;
            hpre[c][k] = ld ? gHC[(size_t)c * n + o.g[k]] : 0.0;
        }
#pragma unroll
    for (int k = 0; k < QR; ++k) {
        ri[k] = o.in[k] ? rin[o.g[k]] : 0.0;
        qi[k] = (o.in[k] && !first) ? q0b[o.g[k]] : 0.0;
        pi[k] = (o.in[k] && !first) ? p0b[o.g[k]] : 0.0;
        wi[k] = (o.in[k] && !first) ? gW[o.g[k]] : 0.0;
    }
    if constexpr (EARLY) {
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = threadIdx.x + u * NT;
            hr[u] = hq[u] = hp[u] = 0.0;
            if (idx < G::N_V) {
                const int rr = idx / G::RW, cc = idx - rr * G::RW;
                const int gi = r0 - G::E + rr, gj = c0 - G::E + cc;
                if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
                    hr[u] = rin[gi * w + gj];
                    if (!first) {
                        hq[u] = q0b[gi * w + gj];
                        hp[u] = p0b[gi * w + gj];
                    }
                }
            }
        }
    }
    // records of launch j - 1 are in the buffer of its parity (or folded); launch j writes the other
    int nb;
    const double* rec = slot_rec(sl, first ? 2 : 1, nb);
    if (!first && !sl.fold_app && ((j - 1) & 1)) rec = sl.rec_app2;
    double* rec_out = (j & 1) ? sl.rec_app2 : sl.rec_app;
    const gbl_t<const SolveState> sg = gbl((const SolveState*)st);
    const TestSettings ts = test_settings(st);
    const int zin = first ? zr_width(ts.check_every, nz, 0) : (j >= 2 ? zr_width(ts.check_every, nz, j - 1) : 0);
    const int nin = first ? 1 + zin : 4 + s + zin;
    const bool keep = j >= 1 && uni(sg->store_basis) && j - 1 < uni(sg->v_cap);
    const bool acc_mine = m.y == 0 && j >= 1 && (int)threadIdx.x < s;
    const double zacc0 = acc_mine ? sg->zacc[threadIdx.x] : 0.0;
    const double mu_lane = REC ? mu_of_lane(st, ts.s) : 0.0;
    // recycled steps on 8-row tiles (small images, latency-bound): 32 loads in flight per thread
    // cover the records of a 256 x 256 image in one round
    if (stopped_before(mark, step)) return;
    reduce_partials<(REC && Q == 1) ? 32 : 8>(rec, nb, nin, tot);
    double alpha = 0.0, beta = 0.0, rho_prev = 0.0;
    const double* e = tot + 4;
    bool stop = false;
    if (first || j >= 2) {   // test of iterate 0 (launch 0) or of iterate j - 1
        const int it = first ? 0 : j - 1;
        const double rho_t = first ? tot[0] : tot[1];
        const Decision dec = decide(ts, it, rho_t, first ? tot + 1 : tot + 4 + s, zin > 0, mu_lane);
        if (m.y == 0 && threadIdx.x == 0) {
            st->rho2[it & 1] = rho_t;
            if (zin) st->est = dec.est;
            st->iters = it;
            if (first) st->res0 = sqrt(rho_t);
            if (dec.done) {
                st->status = dec.status;
                st->done = 1;
                st->stop_at = step + 1;
            }
        }
        stop = dec.done;
    }
    if (!first && !stop) {
        const double sigma = tot[0];
        rho_prev = tot[1];
        if (!(sigma > 0.0)) {
            if (m.y == 0 && threadIdx.x == 0) {
                st->status = (sigma != sigma || fabs(sigma) == INFINITY) ? BL_E_NONFINITE : BL_E_INDEFINITE;
                st->iters = j - 1;
                st->done = 1;
                st->stop_at = step + 1;
            }
            stop = true;
        } else {
            alpha = rho_prev / sigma;
            double ee = 0.0;
            for (int k = 0; k < s; ++k) ee += e[k] * e[k];
            const double rho_hat = rho_prev - 2.0 * alpha * tot[2] + alpha * alpha * (tot[3] - ee);
            beta = rho_hat / rho_prev;
        }
    }
    if (stop) return;
    // block 0: corrs[k] = alpha (M e)_k, the part of record value 4 + k that no pixel carries.
    // G lanes share row k of M (all of their loads in one round), summed by a group sum.
    __shared__ double corrs[S_MAX];
    if constexpr (REC) {
        if (m.y == 0 && !first) {
            const int G = s <= 32 ? 8 : 4;
            const int k = (int)threadIdx.x / G, jl = (int)threadIdx.x & (G - 1);
            double part = 0.0;
            if (k < s) {
#pragma unroll 1
                for (int u0 = 0; u0 < 16; u0 += 8) {   // (one round for s <= 32)
                    if (jl + u0 * G >= s) break;
                    double mv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int l = jl + (u0 + u) * G;
                        mv[u] = l < s ? gM[(size_t)l * s + k] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int l = jl + (u0 + u) * G;
                        if (l < s) part += mv[u] * e[l];
                    }
                }
            }
            part = group_sum(part, G);
            if (k < s && jl == 0) corrs[k] = alpha * part;
        }
    }
    if (m.y == 0 && j >= 1) {
        if (acc_mine) st->zacc[threadIdx.x] = zacc0 - alpha * e[threadIdx.x];
        if (threadIdx.x == 0 && keep && sl.lz) {
            gLZ[2 * (j - 1)] = alpha;
            gLZ[2 * (j - 1) + 1] = rho_prev;
        }
    }
    Stencil S = base;
    slot_stencil(S, sl);
    auto yof = [&](double rv, double qv, double pv) { return first ? rv : rv - alpha * qv + beta * pv; };
    if constexpr (EARLY) {
        double* v = lds + L::o_v;
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = threadIdx.x + u * NT;
            if (idx < G::N_V) v[idx] = yof(hr[u], hq[u], hp[u]);
        }
        X = tv_xload<Q>(h, w, sl.xhat, r0, c0);
    } else {
        if (first)
            q_stage<double, R, CLS, Q>(lds + L::o_v, S.h, S.w, r0, c0, [&](int g) { return rin[g]; });
        else
            q_stage<double, R, CLS, Q>(lds + L::o_v, S.h, S.w, r0, c0,
                                       [&](int g) { return rin[g] - alpha * q0b[g] + beta * p0b[g]; });
        if constexpr (CLS == TC_TV) X = tv_xload<Q>(h, w, sl.xhat, r0, c0);
    }
    __syncthreads();
    double hv[QR];
    q_hvp<double, R, CLS, Q>(lds, S, r0, c0, hv, X);
    // The record.  Taller tiles (Q >= 2): per-wave sums by DPP (wave_total) into the tile's LDS.
    // 8-row tiles (one pixel per thread, one wave per SIMD at 256 x 256, where every dependent
    // instruction shows): the values go through LDS eight at a time, transposed, so each is
    // summed by 32 lanes over 8 entries and one 32-lane DPP sum instead of a full wave sum per
    // value; two alternating buffers of 8 x 256 values, one barrier per round.
    constexpr bool LDS_RED = Q == 1;
    __shared__ double recv[NV_RED];
    double* wred = lds;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto put = [&](int k, double v) {
        const double t = wave_total(v);
        if (lane == 0) wred[wave * NV_RED + k] = t;
    };
    int rbuf = 0;
    auto sum8 = [&](const double (&v)[8], int nval, int base) {
        double* buf = lds + rbuf * 8 * NT;
        rbuf ^= 1;
#pragma unroll
        for (int k = 0; k < 8; ++k) buf[k * NT + threadIdx.x] = v[k];
        __syncthreads();
        const int k = threadIdx.x >> 5, jl = threadIdx.x & 31;
        double acc = 0.0;
        if (k < nval) {
            const double* b = buf + k * NT + jl;
            acc = ((b[0] + b[32]) + (b[64] + b[96])) + ((b[128] + b[160]) + (b[192] + b[224]));
        }
        acc = group_sum_last(acc, 32);
        if (jl == 31 && k < nval) recv[base + k] = acc;
    };
    // columns of C and H C: C e and (H C) e of the previous step's e at the own pixels, and the
    // record values C^T (H y)
    double ce[QR], hce[QR];
#pragma unroll
    for (int k = 0; k < QR; ++k) ce[k] = hce[k] = 0.0;
    if constexpr (REC) {
        auto column = [&](int c, const double* cv, const double* hcv) {
            const double ec = first ? 0.0 : e[c];
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < QR; ++k) {
                ce[k] += cv[k] * ec;
                hce[k] += hcv[k] * ec;
                d += cv[k] * hv[k];
            }
            return d;
        };
        if constexpr (LDS_RED) {
            static_assert(PF % 8 == 0 && CH == 8, "rounds of 8 columns");
#pragma unroll
            for (int r = 0; r < PF / 8; ++r) {
                if (8 * r >= s) break;
                double v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = 8 * r + i < s ? column(8 * r + i, cpre[8 * r + i], hpre[8 * r + i]) : 0.0;
                sum8(v, s - 8 * r < 8 ? s - 8 * r : 8, 4 + 8 * r);
            }
        } else {
#pragma unroll
            for (int c = 0; c < PF; ++c)
                if (c < s) put(4 + c, column(c, cpre[c], hpre[c]));
        }
        for (int c0r = PF; c0r < s; c0r += CH) {
            double cv[CH][QR], hcv[CH][QR];
#pragma unroll
            for (int i = 0; i < CH; ++i)
#pragma unroll
                for (int k = 0; k < QR; ++k) {
                    const bool ld = o.in[k] && c0r + i < s;
                    cv[i][k] = ld ? gC[(size_t)(c0r + i) * n + o.g[k]] : 0.0;
                    hcv[i][k] = (ld && !first) ? gHC[(size_t)(c0r + i) * n + o.g[k]] : 0.0;
                }
            if constexpr (LDS_RED) {
                double v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = c0r + i < s ? column(c0r + i, cv[i], hcv[i]) : 0.0;
                sum8(v, s - c0r < 8 ? s - c0r : 8, 4 + c0r);
            } else {
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    if (c0r + i < s) put(4 + c0r + i, column(c0r + i, cv[i], hcv[i]));
            }
        }
    }
    // own pixels: the new vectors
    double rn[QR], pn[QR], qn[QR];
#pragma unroll
    for (int k = 0; k < QR; ++k) {
        const double y = yof(ri[k], qi[k], pi[k]);
        rn[k] = o.in[k] ? (first ? ri[k] : ri[k] - alpha * qi[k] + alpha * ce[k]) : 0.0;
        pn[k] = o.in[k] ? y + alpha * ce[k] : 0.0;
        qn[k] = o.in[k] ? hv[k] + alpha * hce[k] : 0.0;
        if (o.in[k]) {
            if (!first) {
                r1b[o.g[k]] = rn[k];
                gW[o.g[k]] = wi[k] + alpha * pi[k];
                if (keep) gV[(size_t)(j - 1) * n + o.g[k]] = ri[k] / sqrt(rho_prev);
            }
            p1b[o.g[k]] = pn[k];
            q1b[o.g[k]] = qn[k];
        }
    }
    {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int k = 0; k < QR; ++k) {
            a0 += pn[k] * qn[k];
            a1 += rn[k] * rn[k];
            a2 += rn[k] * qn[k];
            a3 += qn[k] * qn[k];
        }
        if constexpr (LDS_RED) {
            const double v[8] = {a0, a1, a2, a3, 0.0, 0.0, 0.0, 0.0};
            sum8(v, 4, 0);
        } else {
            put(0, a0);
            put(1, a1);
            put(2, a2);
            put(3, a3);
        }
    }
    // Z^T r_j when iterate j is tested (launch j + 1 tests it)
    const int zw = j >= 1 ? zr_width(ts.check_every, nz, j) : 0;
    if constexpr (REC) {
        for (int z0 = 0; z0 < zw; z0 += CH) {
            double zv[CH][QR];
#pragma unroll
            for (int i = 0; i < CH; ++i)
#pragma unroll
                for (int k = 0; k < QR; ++k)
                    zv[i][k] = (o.in[k] && z0 + i < zw) ? gZ[(size_t)(z0 + i) * n + o.g[k]] : 0.0;
            if constexpr (LDS_RED) {
                double v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    double d = 0.0;
#pragma unroll
                    for (int k = 0; k < QR; ++k) d += zv[i][k] * rn[k];
                    v[i] = z0 + i < zw ? d : 0.0;
                }
                sum8(v, zw - z0 < 8 ? zw - z0 : 8, 4 + s + z0);
            } else {
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    if (z0 + i >= zw) break;
                    double d = 0.0;
#pragma unroll
                    for (int k = 0; k < QR; ++k) d += zv[i][k] * rn[k];
                    put(4 + s + z0 + i, d);
                }
            }
        }
    }
    __syncthreads();
    const int nv = 4 + s + zw;
    for (int k = threadIdx.x; k < nv; k += NT) {
        double sum;
        if constexpr (LDS_RED) {
            sum = recv[k];
        } else {
            sum = 0.0;
#pragma unroll
            for (int wv = 0; wv < NWAVE; ++wv) sum += wred[wv * NV_RED + k];
        }
        if (REC && m.y == 0 && !first && k >= 4 && k < 4 + s) sum += corrs[k - 4];
        gbl(rec_out)[(size_t)m.y * nv + k] = sum;
    }
}

// ------------------------------------------------------------------ out[:, c] = H v[:, c]
// One 32 x 8Q tile of one column per block (grid: tiles x columns): the refresh's Y = H W and
// the stand-alone product of the ABI.
template <typename T, int R, int CLS, int Q>
__global__ void __launch_bounds__(NT) k_hvp(Stencil S, const double* __restrict__ xhat,
                                            const double* __restrict__ v, double* __restrict__ out) {
    constexpr int QH = QTY * Q;
    using L = QLayout<T, R, CLS, Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int qtx = (S.w + QW - 1) / QW;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int r0 = (t / qtx) * QH, c0 = (t % qtx) * QW;
    const double* vc = v + (size_t)blockIdx.y * S.n;
    q_stage<T, R, CLS, Q>(lds + L::o_v, S.h, S.w, r0, c0, [&](int i) { return vc[i]; });
    const TvX<Q> X = tv_x<CLS, Q>(S.h, S.w, xhat, r0, c0);
    __syncthreads();
    T hv[Q];
    q_hvp<T, R, CLS, Q>(lds, S, r0, c0, hv, X);
    double* oc = out + (size_t)blockIdx.y * S.n;
    const int tx = threadIdx.x & (QW - 1), ty = threadIdx.x / QW, gj = c0 + tx;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int gi = r0 + Q * ty + k;
        if (gi < S.h && gj < S.w) oc[gi * S.w + gj] = (double)hv[k];
    }
}

template <typename K>
static void allow_lds_b(K kernel, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static inline dim3 map_grid(const BatchMap& M) { return dim3(M.off[M.ns]); }

template <int Q>
hipError_t launch_b_residual_q(const Stencil& base, bool rec, const Slot* slots, const BatchMap& M, int periodic,
                               hipStream_t stream) {
    q_dispatch(base.R, tile_class(base.reg, base.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        const size_t lds = QLayout<double, RR, CC, Q>::bytes;
        auto go = [&](auto kern) {
            allow_lds_b(kern, lds);
            hipLaunchKernelGGL(kern, map_grid(M), dim3(NT), lds, stream, base, slots, M, periodic);
        };
        if (rec) go(k_b_residual<RR, CC, Q, true>);
        else go(k_b_residual<RR, CC, Q, false>);
    });
    return hipGetLastError();
}

template <int Q>
hipError_t launch_b_apply_q(const Stencil& base, bool rec, bool fp32, const Slot* slots, const BatchMap& M,
                            StepRef sr, hipStream_t stream) {
    q_dispatch(base.R, tile_class(base.reg, base.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        auto go = [&](auto kern, size_t lds) {
            allow_lds_b(kern, lds);
            hipLaunchKernelGGL(kern, map_grid(M), dim3(NT), lds, stream, base, slots, M, sr);
        };
        constexpr size_t l32 = QLayout<float, RR, CC, Q>::bytes, l64 = QLayout<double, RR, CC, Q>::bytes;
        if (fp32) {
            if (rec) go(k_b_apply<float, RR, CC, Q, true>, l32);
            else go(k_b_apply<float, RR, CC, Q, false>, l32);
        } else {
            if (rec) go(k_b_apply<double, RR, CC, Q, true>, l64);
            else go(k_b_apply<double, RR, CC, Q, false>, l64);
        }
    });
    return hipGetLastError();
}

template <int Q>
hipError_t launch_f_step_q(const Stencil& base, bool rec, const Slot* slots, const BatchMap& M, StepRef sr,
                           const Slot* one, hipStream_t stream) {
    q_dispatch(base.R, tile_class(base.reg, base.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        // 8-row tiles reduce their record through two buffers of 8 x NT doubles in the tile's LDS
        constexpr size_t tile = QLayout<double, RR, CC, Q>::bytes, red = Q == 1 ? 2 * 8 * NT * sizeof(double) : 0;
        const size_t lds = tile > red ? tile : red;
        const bool single = one && M.ns == 1;
        const Slot arg = single ? *one : Slot{};
        auto go = [&](auto kern) {
            allow_lds_b(kern, lds);
            hipLaunchKernelGGL(kern, map_grid(M), dim3(NT), lds, stream, base, slots, M, sr, arg);
        };
        if (rec) single ? go(k_f_step<RR, CC, Q, true, true>) : go(k_f_step<RR, CC, Q, true, false>);
        else single ? go(k_f_step<RR, CC, Q, false, true>) : go(k_f_step<RR, CC, Q, false, false>);
    });
    return hipGetLastError();
}

template <int Q>
hipError_t launch_hvp_q(const Stencil& S, bool fp32, const double* xhat, const double* v, double* out, int ncols,
                        hipStream_t st) {
    const dim3 grid(((S.w + QW - 1) / QW) * ((S.h + QTY * Q - 1) / (QTY * Q)), ncols);
    q_dispatch(S.R, tile_class(S.reg, S.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        if (fp32) {
            const size_t lds = QLayout<float, RR, CC, Q>::bytes;
            allow_lds_b(k_hvp<float, RR, CC, Q>, lds);
            hipLaunchKernelGGL((k_hvp<float, RR, CC, Q>), grid, dim3(NT), lds, st, S, xhat, v, out);
        } else {
            const size_t lds = QLayout<double, RR, CC, Q>::bytes;
            allow_lds_b(k_hvp<double, RR, CC, Q>, lds);
            hipLaunchKernelGGL((k_hvp<double, RR, CC, Q>), grid, dim3(NT), lds, st, S, xhat, v, out);
        }
    });
    return hipGetLastError();
}

}  // namespace bl
