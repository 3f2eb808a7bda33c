// RMINRES (Section 2.2.2, Algorithm 3) for one Hessian system in FP64: two fused launches per
// Lanczos step, no grid synchronisation (per-block records reduced by the next launch, as in
// the recycled-CG kernels).
//
// Step k = 1, 2, ...:
//   apply  (tiles of 32 x 8)  beta_k = ||u_k|| from the previous launch's records; the stop test
//                             of iterate k - 2 (iterate 0 at k = 1); the Givens rotation of
//                             column k - 1 of T; v_k = u_k / beta_k; q = H v_k; record
//                             [v_k . q, C^T q].
//   update (pixel blocks)     alpha_k and e_k = C^T q from the apply records;
//                             u_{k+1} = (q - C e_k) - alpha_k v_k - beta_k v_{k-1};
//                             the solution update of step k - 1; record [u_{k+1} . u_{k+1},
//                             Z^T r_{k-1} when iterate k - 1 is tested].
// The rotation of column k needs beta_{k+1}, which the update's records give, so the solution
// update trails the Lanczos step by one launch pair, and iterate j is tested by the apply launch
// of step j + 2.  The solve stops with the tested iterate, which is then the current w.
//
// Differences in form from the printed algorithm (same quantities in exact arithmetic):
//   * alpha_k = v_k . H v_k: v_k is orthogonal to C, so projecting H v_k first changes nothing;
//   * b~_k = U mh_k is kept in the s coordinates of U: mh_k = (e_k - gamma mh_{k-2}
//     - delta mh_{k-1}) / eps~ and zacc += c zeta mh_k, applied once at the end as w -= U zacc
//     (the minus sign of the recycle part that eq. zk_answer fixes);
//   * the explicit residual r_k = V_{k+1} Q_k^T (zeta_k e_{k+1}) (Q_k the product of the
//     rotations) obeys r_k = s_k^2 r_{k-1} + c_k zeta_k v_{k+1}: one vector instead of the seven
//     that Appendix A's recurrence r_k = r_{k-1} - c zeta H (v~ - b~) keeps.
#include "batch_tile.h"

namespace bl {

// Stop decision for iterate j from its residual norm |zeta_j| and, when the record holds it,
// Z^T r_j.  Same order as the recycled-CG test: non-finite; exact zero; only every
// check_every iterates: the error estimate or the residual test; then the iteration limit.
__device__ __forceinline__ Decision m_decide(const MinresState* st, int j, double res, const double* zr,
                                             bool have_zr) {
    Decision d{false, BL_OK, NAN};
    if (st->hgerr_on && have_zr) {
        double acc = 0.0;
        for (int k = 0; k < st->s; ++k) {
            const double t = st->mu[k] * zr[k];
            acc += t * t;
        }
        d.est = sqrt(acc);
    }
    if (!(res == res) || res == INFINITY) {
        d.done = true;
        d.status = BL_E_NONFINITE;
        return d;
    }
    bool met;
    if (res == 0.0) met = true;
    else if (j % st->check_every) met = false;
    else if (st->stop == BL_STOP_HGERR && st->hgerr_on) met = d.est <= st->hg_tol;
    else met = res <= st->tol * st->gnorm;
    if (met) {
        d.done = true;
    } else if (j >= st->max_iter) {
        d.done = true;
        d.status = BL_E_NOT_CONVERGED;
    }
    return d;
}

__device__ __forceinline__ void tile_origin(const Stencil& S, int& r0, int& c0) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    r0 = (t / S.tiles_x) * QTY;
    c0 = (t % S.tiles_x) * QW;
}

// ------------------------------------------------------------------ r = g - H w
// Record [g.g, C^T r].
template <int R, int CLS>
__global__ void __launch_bounds__(NT) k_m_residual(Stencil S, MinresArgs a) {
    using L = QLayout<double, R, CLS, 1>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    int r0, c0;
    tile_origin(S, r0, c0);
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
        return k == 0 ? gv * gv : a.C[(size_t)(k - 1) * S.n + o.g[0]] * rv;
    });
}

// ------------------------------------------------------------------ set-up
// c0 = C^T r (records), w += U c0, r -= C c0, u_1 = r, u_0 = v~ = 0; record [r.r, Z^T r].
// Block 0 writes the solve's settings and the starting values of the recurrences.
__global__ void __launch_bounds__(NT) k_m_init(MinresArgs a, MinresInit in, int fold) {
    __shared__ double tot[NT];
    const int s = a.s, n = a.n;
    reduce_partials(fold ? a.fold : a.rec_res, fold ? FOLD_BLOCKS : a.ntiles, 1 + s, tot);
    MinresState* st = a.st;
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < S_MAX; k += NT) {
            st->zacc[k] = 0.0;
            st->mu[k] = (k < s && in.mu) ? in.mu[k] : 0.0;
            for (int q = 0; q < 4; ++q) {
                st->e[q][k] = 0.0;
                st->mh[q][k] = 0.0;
            }
        }
        if (threadIdx.x == 0) {
            st->done = 0;
            st->status = BL_OK;
            st->iters = 0;
            st->v_cur = 0;
            st->res = 0.0;
            st->res0 = 0.0;
            st->est = NAN;
            st->gnorm = sqrt(tot[0]);
            st->tol = in.tol;
            st->hg_tol = in.hg_tol;
            st->max_iter = in.max_iter;
            st->check_every = in.check_every;
            st->stop = in.stop;
            st->s = in.s;
            st->nz = in.nz;
            st->hgerr_on = in.hgerr_on;
            st->store = in.store;
            st->v_cap = in.v_cap;
            for (int q = 0; q < 4; ++q) {
                st->beta[q] = st->alpha[q] = st->zeta[q] = 0.0;
                st->gam[q] = st->del[q] = st->epst[q] = 0.0;
                st->c[q] = st->sn[q] = 0.0;
            }
            st->beta[0] = 1.0;   // u_0 = 0, so v_0 = u_0 / beta_0 = 0
            st->c[0] = 1.0;      // rotation 0: identity; rotation -1 (slot 3): zero
        }
    }
    const double* c0 = tot + 1;
    const int i = blockIdx.x * NT + threadIdx.x;
    const bool inb = i < n;
    double ri = 0.0;
    if (inb) {
        a.w[i] += combo(a.U, n, i, c0, s);
        ri = a.r[i] - combo(a.C, n, i, c0, s);
        a.r[i] = ri;
        a.u[1][i] = ri;
        a.u[0][i] = 0.0;
        a.m[0][i] = 0.0;
        a.m[1][i] = 0.0;
    }
    block_partials(a.rec_upd, 1 + a.nz, [&](int k) -> double {
        if (!inb) return 0.0;
        return k == 0 ? ri * ri : a.Z[(size_t)(k - 1) * n + i] * ri;
    });
}

// ------------------------------------------------------------------ apply, step k
// `nvb` values per record of the previous launch (1, or 1 + nz when iterate k - 2 is tested;
// 1 + nz at k = 1); `fold`: those records were folded.
// Loads that do not depend on this step's scalars are issued before the record reduction: the
// columns of C at the thread's pixel (the first MCP), x_hat, and for TV the staged region of u_k
// (the stencil input v_k = u_k / beta_k is formed from registers once beta_k is known).
// REC: the solve has a recycle space (s > 0); without one no registers hold columns of C.
template <int R, int CLS, bool REC>
__global__ void __launch_bounds__(NT) k_m_apply(Stencil S, MinresArgs a, int k, int nvb, int fold) {
    using L = QLayout<double, R, CLS, 1>;
    using G = QGeo<R, CLS, 1>;
    constexpr int MCP = REC ? 24 : 1;
    constexpr bool EARLY = CLS == TC_TV;
    constexpr int NST = EARLY ? (G::N_V + NT - 1) / NT : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    __shared__ double tot[NT];
    __shared__ int sdone;
    MinresState* st = a.st;
    if (threadIdx.x == 0) sdone = st->done;
    int r0, c0;
    tile_origin(S, r0, c0);
    const Own<1> o = own_pixels<1>(S.h, S.w, r0, c0);
    const double* __restrict__ uk = a.u[k % 3];
    const int n = S.n, s = REC ? a.s : 0;
    double cpre[MCP], hu[NST];
    TvX<1> X{};
#pragma unroll
    for (int c = 0; c < MCP; ++c) cpre[c] = (o.in[0] && c < s) ? a.C[(size_t)c * n + o.g[0]] : 0.0;
    const double uown = o.in[0] ? uk[o.g[0]] : 0.0;
    if constexpr (EARLY) {
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = threadIdx.x + u * NT;
            hu[u] = 0.0;
            if (idx < G::N_V) {
                const int rr = idx / G::RW, cc = idx - rr * G::RW;
                const int gi = r0 - G::E + rr, gj = c0 - G::E + cc;
                if (gi >= 0 && gi < S.h && gj >= 0 && gj < S.w) hu[u] = uk[gi * S.w + gj];
            }
        }
    }
    reduce_partials(fold ? a.fold : a.rec_upd, fold ? FOLD_BLOCKS : a.npix, nvb, tot);
    if (sdone) return;
    if constexpr (EARLY) X = tv_xload<1>(S.h, S.w, a.xhat, r0, c0);
    const double bk = sqrt(tot[0]);
    // stop test of iterate j (zeta_0 = beta_1)
    const int j = k == 1 ? 0 : (k >= 3 ? k - 2 : -1);
    const double res = k == 1 ? bk : (j >= 0 ? fabs(st->zeta[j & 3]) : 0.0);
    Decision dec{false, BL_OK, NAN};
    if (j >= 0) dec = m_decide(st, j, res, tot + 1, nvb > 1);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (lead) {
        st->beta[k & 3] = bk;
        if (k == 1) {
            st->zeta[0] = bk;
            st->res0 = bk;
        }
        if (j >= 0) {
            st->iters = j;
            st->res = res;
            if (nvb > 1) st->est = dec.est;
            if (dec.done) {
                st->status = dec.status;
                st->done = 1;
            }
        }
    }
    if (dec.done) return;
    // rotation of column k - 1: the two previous rotations, then a new one annihilating beta_k
    if (k >= 2) {
        const int km = k - 1;
        const double a_ = st->alpha[km & 3], b_ = st->beta[km & 3];
        const double c1 = st->c[(km - 1) & 3], s1 = st->sn[(km - 1) & 3];
        const double c2 = st->c[(km - 2) & 3], s2 = st->sn[(km - 2) & 3];
        const double gamma = s2 * b_;
        const double delta = c1 * c2 * b_ + s1 * a_;
        const double eps = -s1 * c2 * b_ + c1 * a_;
        const double et = hypot(eps, bk);
        if (!(et > 0.0)) {
            if (lead) {
                st->status = et == 0.0 ? BL_E_BREAKDOWN : BL_E_NONFINITE;
                st->iters = k - 2 > 0 ? k - 2 : 0;
                st->done = 1;
            }
            return;
        }
        const double ck = eps / et, sk = bk / et;
        if (lead) {
            st->c[km & 3] = ck;
            st->sn[km & 3] = sk;
            st->zeta[km & 3] = -sk * st->zeta[(km - 1) & 3];
            st->gam[km & 3] = gamma;
            st->del[km & 3] = delta;
            st->epst[km & 3] = et;
        }
    }
    // v_k = u_k / beta_k and q = H v_k
    auto vof = [&](double uv) { return bk > 0.0 ? uv / bk : 0.0; };
    if constexpr (EARLY) {
        double* v = lds + L::o_v;
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = threadIdx.x + u * NT;
            if (idx < G::N_V) v[idx] = vof(hu[u]);
        }
    } else {
        q_stage<double, R, CLS, 1>(lds + L::o_v, S.h, S.w, r0, c0, [&](int gi) { return vof(uk[gi]); });
        if constexpr (CLS == TC_TV) X = tv_xload<1>(S.h, S.w, a.xhat, r0, c0);
    }
    __syncthreads();
    double hv[1];
    q_hvp<double, R, CLS, 1>(lds, S, r0, c0, hv, X);
    const double vi = o.in[0] ? vof(uown) : 0.0;
    const double qi = o.in[0] ? hv[0] : 0.0;
    if (o.in[0]) {
        a.q[o.g[0]] = qi;
        if (st->store && k - 1 < st->v_cap) a.V[(size_t)(k - 1) * n + o.g[0]] = vi;
    }
    block_partials(a.rec_app, 1 + s, [&](int kk) -> double {
        if (!o.in[0]) return 0.0;
        if (kk == 0) return vi * qi;
        const int c = kk - 1;
        double cv = 0.0;
#pragma unroll
        for (int u = 0; u < MCP; ++u)
            if (u == c) cv = cpre[u];
        if (c >= MCP) cv = a.C[(size_t)c * n + o.g[0]];
        return cv * qi;
    });
}

// ------------------------------------------------------------------ update, step k
// `zr` values of Z^T r_{k-1} go into this launch's record (0 or nz); `fold`: the apply records
// were folded.  WIDE: the records are reduced with all of a thread's loads in flight at once
// (for grids of few blocks, where latency decides; costs registers).
template <bool REC, bool WIDE>
__global__ void __launch_bounds__(NT) k_m_update(MinresArgs a, int k, int zr, int fold) {
    constexpr int MPRE = REC ? 24 : 1;
    __shared__ double tot[NT];
    __shared__ int sdone;
    MinresState* st = a.st;
    if (threadIdx.x == 0) sdone = st->done;
    const int s = REC ? a.s : 0, n = a.n;
    const int i = blockIdx.x * NT + threadIdx.x;
    const bool in = i < n;
    // loads that do not depend on this step's scalars, issued before the reduction
    const double qi = in ? a.q[i] : 0.0;
    const double uk = in ? a.u[k % 3][i] : 0.0;
    const double uk1 = in ? a.u[(k + 2) % 3][i] : 0.0;
    double wi = 0.0, ri = 0.0, mA = 0.0, mB = 0.0;
    if (k >= 2 && in) {
        wi = a.w[i];
        ri = a.r[i];
        mA = a.m[k & 1][i];         // v~_{k-2}
        mB = a.m[(k + 1) & 1][i];   // v~_{k-3}
    }
    double cpre[MPRE];
#pragma unroll
    for (int c = 0; c < MPRE; ++c) cpre[c] = (in && c < s) ? a.C[(size_t)c * n + i] : 0.0;
    // scalars of earlier launches (this step's beta and the rotation of column k - 1 come from
    // the apply launch): read before the reduction
    const int km = k - 1;
    const double bk = st->beta[k & 3], bk1 = st->beta[km & 3];
    double ck = 0.0, sk = 0.0, zk = 0.0, gam = 0.0, del = 0.0, ept = 1.0, zkm = 0.0;
    if (k >= 2) {
        ck = st->c[km & 3];
        sk = st->sn[km & 3];
        zk = st->zeta[km & 3];
        gam = st->gam[km & 3];
        del = st->del[km & 3];
        ept = st->epst[km & 3];
        zkm = st->zeta[(km - 1) & 3];
    }
    const bool lead0 = blockIdx.x == 0;
    // block 0 carries the recycle-space coordinates: e_{k-1} and mh of the two steps before
    const bool mine = lead0 && k >= 2 && (int)threadIdx.x < s;
    const double e_km = mine ? st->e[km & 3][threadIdx.x] : 0.0;
    const double mh1 = mine ? st->mh[(km - 1) & 3][threadIdx.x] : 0.0;
    const double mh2 = mine ? st->mh[(km - 2) & 3][threadIdx.x] : 0.0;
    reduce_partials<WIDE ? 32 : 8>(fold ? a.fold : a.rec_app, fold ? FOLD_BLOCKS : a.ntiles, 1 + s, tot);
    if (sdone) return;
    const double alpha = tot[0];
    const double* e = tot + 1;
    const double vk = bk > 0.0 ? uk / bk : 0.0;
    const double vk1 = bk1 > 0.0 ? uk1 / bk1 : 0.0;
    double ce = 0.0;
#pragma unroll
    for (int c = 0; c < MPRE; ++c)
        if (c < s) ce += cpre[c] * e[c];
    for (int c = MPRE; c < s; ++c) ce += (in ? a.C[(size_t)c * n + i] : 0.0) * e[c];
    const double un = (qi - ce) - alpha * vk - bk * vk1;
    if (in) a.u[(k + 1) % 3][i] = un;
    double rn = ri;
    if (k >= 2) {
        // solution update of step k - 1 with its rotation
        const double tau = ck * zkm;
        const double mn = (vk1 - gam * mB - del * mA) / ept;
        rn = sk * sk * ri + ck * zk * vk;
        if (in) {
            a.m[km & 1][i] = mn;
            a.w[i] = wi + tau * mn;
            a.r[i] = rn;
        }
        if (mine) {
            const double mh = (e_km - gam * mh2 - del * mh1) / ept;
            st->mh[km & 3][threadIdx.x] = mh;
            st->zacc[threadIdx.x] += tau * mh;
        }
    }
    if (lead0) {
        for (int t = threadIdx.x; t < s; t += NT) st->e[k & 3][t] = e[t];
        if (threadIdx.x == 0) st->alpha[k & 3] = alpha;
    }
    block_partials(a.rec_upd, 1 + zr, [&](int kk) -> double {
        if (!in) return 0.0;
        return kk == 0 ? un * un : a.Z[(size_t)(kk - 1) * n + i] * rn;
    });
}

// ------------------------------------------------------------------ w -= U zacc
__global__ void __launch_bounds__(NT) k_m_finish(MinresArgs a) {
    __shared__ double z[S_MAX];
    for (int t = threadIdx.x; t < a.s; t += NT) z[t] = a.st->zacc[t];
    __syncthreads();
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i < a.n) a.w[i] -= combo(a.U, a.n, i, z, a.s);
}

// ------------------------------------------------------------------ record fold
// Block f reduces records f * nb / FOLD_BLOCKS .. (f + 1) * nb / FOLD_BLOCKS - 1 (in order)
// into folded record f; consumers then reduce the FOLD_BLOCKS folded records.
__global__ void __launch_bounds__(NT) k_m_fold(const double* __restrict__ rec, int nb, int nv,
                                               double* __restrict__ out) {
    __shared__ double tot[NT];
    const int f = blockIdx.x;
    const int b0 = (int)((long)f * nb / FOLD_BLOCKS), b1 = (int)((long)(f + 1) * nb / FOLD_BLOCKS);
    reduce_partials(rec + (size_t)b0 * nv, b1 - b0, nv, tot);
    for (int k = threadIdx.x; k < nv; k += NT) out[(size_t)f * nv + k] = tot[k];
}

// ------------------------------------------------------------------ launchers
hipError_t launch_m_residual(const Stencil& S, const MinresArgs& a, hipStream_t stream) {
    q_dispatch(S.R, tile_class(S.reg, S.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        const size_t lds = QLayout<double, RR, CC, 1>::bytes;
        allow_lds_b(k_m_residual<RR, CC>, lds);
        hipLaunchKernelGGL((k_m_residual<RR, CC>), dim3(a.ntiles), dim3(NT), lds, stream, S, a);
    });
    return hipGetLastError();
}

hipError_t launch_m_init(const MinresArgs& a, const MinresInit& in, bool fold, hipStream_t stream) {
    hipLaunchKernelGGL(k_m_init, dim3(a.npix), dim3(NT), 0, stream, a, in, (int)fold);
    return hipGetLastError();
}

hipError_t launch_m_apply(const Stencil& S, const MinresArgs& a, int k, int nvb, bool fold, hipStream_t stream) {
    q_dispatch(S.R, tile_class(S.reg, S.fs), [&](auto rc, auto cc) {
        constexpr int RR = decltype(rc)::value, CC = decltype(cc)::value;
        const size_t lds = QLayout<double, RR, CC, 1>::bytes;
        auto go = [&](auto kern) {
            allow_lds_b(kern, lds);
            hipLaunchKernelGGL(kern, dim3(a.ntiles), dim3(NT), lds, stream, S, a, k, nvb, (int)fold);
        };
        if (a.s > 0) go(k_m_apply<RR, CC, true>);
        else go(k_m_apply<RR, CC, false>);
    });
    return hipGetLastError();
}

hipError_t launch_m_update(const MinresArgs& a, int k, int zr, bool fold, hipStream_t stream) {
    if (a.s > 0 && a.npix <= 16 * 256)
        hipLaunchKernelGGL((k_m_update<true, true>), dim3(a.npix), dim3(NT), 0, stream, a, k, zr, (int)fold);
    else if (a.s > 0)
        hipLaunchKernelGGL((k_m_update<true, false>), dim3(a.npix), dim3(NT), 0, stream, a, k, zr, (int)fold);
    else
        hipLaunchKernelGGL((k_m_update<false, false>), dim3(a.npix), dim3(NT), 0, stream, a, k, zr, (int)fold);
    return hipGetLastError();
}

hipError_t launch_m_finish(const MinresArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(k_m_finish, dim3(a.npix), dim3(NT), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_m_fold(const double* rec, int nb, int nv, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_m_fold, dim3(FOLD_BLOCKS), dim3(NT), 0, stream, rec, nb, nv, out);
    return hipGetLastError();
}

}  // namespace bl
