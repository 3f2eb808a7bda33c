// Recycled-CG kernels over a batch of independent solves ("slots").
//
// A launch covers every active slot: block b works for slot map[b].x on its local tile or
// pixel block map[b].y.  Slots differ in image size, recycle dimension, iteration index and
// stop state; they share the operator class (regulariser, blur, filter size, precision).
// No kernel synchronises its blocks: each kernel writes one partial record per block into
// its slot's record array; the next kernel reduces the records of its slot in every block
// (fixed order), so a slot's scalars and decisions are identical in every block and do
// not depend on the other slots.  Block 0 of a slot stores the scalars for the host.
#include "batch_tile.h"

namespace bl {

// Set-up: c0 = C^T r (records), w += U c0, r -= C c0, record [r.r, Z^T r].
__global__ void __launch_bounds__(NT) k_b_init(const Slot* __restrict__ slots, BatchMap M) {
    __shared__ double tot[NT];
    const int2 m = map_block(M, blockIdx.x);
    const Slot& sl = slots[m.x];
    if (m.y >= sl.npix) return;
    const int s = sl.s, nz = sl.nz, n = sl.n;
    int nb;
    const double* rec = slot_rec(sl, 0, nb);
    reduce_partials(rec, nb, 1 + s, tot);
    if (m.y == 0 && threadIdx.x == 0) sl.st->gnorm = sqrt(tot[0]);
    const double* c0 = tot + 1;
    const int i = m.y * NT + threadIdx.x;
    const bool in = i < n;
    double ri = 0.0;
    if (in) {
        sl.w[i] += combo(sl.U, n, i, c0, s);
        ri = sl.r[i] - combo(sl.C, n, i, c0, s);
        sl.r[i] = ri;
    }
    block_partials(
        sl.rec_upd, 1 + zr_width(sl.st, nz, 0),
        [&](int k) -> double {
            if (!in) return 0.0;
            return k == 0 ? ri * ri : sl.Z[(size_t)(k - 1) * n + i] * ri;
        },
        m.y);
}

// Iteration j, second half: sigma, e from the apply records; alpha = rho_j / sigma;
// w += alpha p;  r -= alpha (q - C e);  z -= alpha e;  record [r.r, Z^T r] (Z^T r only when
// the test of iteration j + 1 evaluates the error estimate).
// REC: some slot of the launch has a recycle space; without one (plain CG only) no registers
// hold columns of C or Z.  A slot with s = 0 computes the same values either way.
// WIDE: the records are reduced with all of a thread's loads in flight at once (a single
// memory round trip; costs registers): for launches of few blocks, where latency decides.
template <bool REC, bool WIDE>
__global__ void __launch_bounds__(NT) k_b_update(const Slot* __restrict__ slots, BatchMap M, StepRef sr) {
    constexpr int UPRE = REC ? 24 : 1;
    __shared__ double tot[NT];
    const int2 m = map_block(M, blockIdx.x);
    const Slot& sl = slots[m.x];
    if (m.y >= sl.npix) return;
    SolveState* st = sl.st;
    const int mark = stop_mark(st);
    const int step = step_of(sr), j = step - sl.j0;
    const int s = REC ? sl.s : 0, n = sl.n;
    const int i = m.y * NT + threadIdx.x;
    const bool in = i < n;
    const gbl_t<const double> p = gbl((const double*)sl.p[(j + 1) & 1]), gq = gbl((const double*)sl.q);
    const gbl_t<const double> gC = gbl(sl.C), gZ = gbl(sl.Z);
    const gbl_t<double> gw = gbl(sl.w), gr = gbl(sl.r);
    const double wi = in ? gw[i] : 0.0, pi = in ? p[i] : 0.0, ri0 = in ? gr[i] : 0.0, qi = in ? gq[i] : 0.0;
    double cpre[UPRE], zpre[UPRE];
#pragma unroll
    for (int k = 0; k < UPRE; ++k) cpre[k] = (in && k < s) ? gC[(size_t)k * n + i] : 0.0;
    const gbl_t<const SolveState> sg = gbl((const SolveState*)st);
    const int zw = REC ? zr_width(st, sl.nz, j + 1) : 0;
#pragma unroll
    for (int k = 0; k < UPRE; ++k) zpre[k] = (in && k < zw) ? gZ[(size_t)k * n + i] : 0.0;
    int nb;
    const double* rec = slot_rec(sl, 1, nb);
    // scalars of earlier launches, read before the reduction: rho_j (the apply of this
    // iteration) and, in block 0, the recycle coefficient accumulated so far
    const double rho = uni(sg->rho2[j & 1]);
    const bool keep_lz = m.y == 0 && sl.lz && uni(sg->store_basis) && j < uni(sg->v_cap);
    const bool acc_mine = m.y == 0 && (int)threadIdx.x < s;
    const double zacc0 = acc_mine ? sg->zacc[threadIdx.x] : 0.0;
    // the apply launch of this step runs first: a stop it decided counts too
    if (stopped_before(mark, step + 1)) return;
    reduce_partials<WIDE ? 32 : 8>(rec, nb, 1 + s, tot);
    const double sigma = tot[0];
    if (!(sigma > 0.0)) {
        if (m.y == 0 && threadIdx.x == 0) {
            st->status = (sigma != sigma || fabs(sigma) == INFINITY) ? BL_E_NONFINITE : BL_E_INDEFINITE;
            st->iters = j;
            st->done = 1;
            st->stop_at = step + 1;
        }
        return;
    }
    const double alpha = rho / sigma;
    const double* e = tot + 1;
    if (acc_mine) st->zacc[threadIdx.x] = zacc0 - alpha * e[threadIdx.x];
    if (m.y == 0 && threadIdx.x == 0) st->alpha = alpha;
    if (keep_lz && threadIdx.x == 0) sl.lz[2 * j] = alpha;
    double ce = 0.0;
#pragma unroll
    for (int k = 0; k < UPRE; ++k)
        if (k < s) ce += cpre[k] * e[k];
    for (int k = UPRE; k < s; ++k) ce += (in ? gC[(size_t)k * n + i] : 0.0) * e[k];
    const double ri = ri0 - alpha * (qi - ce);
    if (in) {
        gw[i] = wi + alpha * pi;
        gr[i] = ri;
    }
    block_partials(
        sl.rec_upd, 1 + zw,
        [&](int k) -> double {
            if (!in) return 0.0;
            if (k == 0) return ri * ri;
            const int c = k - 1;
            double zv = 0.0;
#pragma unroll
            for (int u = 0; u < UPRE; ++u)
                if (u == c) zv = zpre[u];
            if (c >= UPRE) zv = gZ[(size_t)c * n + i];
            return zv * ri;
        },
        m.y);
}

// Residual replacement: r holds t = g - H w (record [g.g, C^T t]): z := C^T t,
// r := t - C z, and the slot resumes at iteration step - j0, whose apply step re-tests the
// replaced residual.  With `periodic` set a slot that has already stopped is left alone.
__global__ void __launch_bounds__(NT) k_b_replace(const Slot* __restrict__ slots, BatchMap M, int periodic,
                                                  StepRef sr) {
    __shared__ double tot[NT];
    const int2 m = map_block(M, blockIdx.x);
    const Slot& sl = slots[m.x];
    if (m.y >= sl.npix || (periodic && sl.st->done)) return;
    const int s = sl.s, nz = sl.nz, n = sl.n;
    int nb;
    const double* rec = slot_rec(sl, 0, nb);
    reduce_partials(rec, nb, 1 + s, tot);
    const double* c = tot + 1;
    if (m.y == 0) {
        for (int k = threadIdx.x; k < s; k += NT) sl.st->zacc[k] = c[k];
        if (threadIdx.x == 0) {
            sl.st->done = 0;
            sl.st->stop_at = 0;
            sl.st->status = BL_OK;
            sl.st->rr_j = step_of(sr) - sl.j0;
        }
    }
    const int i = m.y * NT + threadIdx.x;
    const bool in = i < n;
    double ri = 0.0;
    if (in) {
        ri = sl.r[i] - combo(sl.C, n, i, c, s);
        sl.r[i] = ri;
    }
    block_partials(
        sl.rec_upd, 1 + zr_width(sl.st, nz, step_of(sr) - sl.j0),
        [&](int k) -> double {
            if (!in) return 0.0;
            return k == 0 ? ri * ri : sl.Z[(size_t)(k - 1) * n + i] * ri;
        },
        m.y);
}

// w += U z.
__global__ void __launch_bounds__(NT) k_b_finish(const Slot* __restrict__ slots, BatchMap M) {
    __shared__ double z[S_MAX];
    const int2 m = map_block(M, blockIdx.x);
    const Slot& sl = slots[m.x];
    if (m.y >= sl.npix) return;
    const int s = sl.s;
    for (int k = threadIdx.x; k < s; k += NT) z[k] = sl.st->zacc[k];
    __syncthreads();
    const int i = m.y * NT + threadIdx.x;
    if (i < sl.n) sl.w[i] += combo(sl.U, sl.n, i, z, s);
}

// Fold the records of kind `which` (0 residual, 1 apply, 2 update, read by the test of step
// sr; 3: the input of a fused step, the set-up's records at its step 0 and the previous step's
// after): FOLD_BLOCKS blocks per listed slot; block f reduces the records f * nb / FOLD_BLOCKS ..
// (f + 1) * nb / FOLD_BLOCKS - 1 (in order) into folded record f, and consumers then reduce the
// FOLD_BLOCKS folded records (two levels, fixed order: deterministic).
__global__ void __launch_bounds__(NT) k_b_fold(const Slot* __restrict__ slots, BatchMap M, int which, StepRef sr) {
    __shared__ double tot[NT];
    const Slot& sl = slots[M.slot[blockIdx.x / FOLD_BLOCKS]];
    // the records of a step (kinds 1 to 3) are read by no one once the slot has stopped (kind 1
    // follows the apply launch of its own step)
    if (which != 0 && stopped_before(stop_mark(sl.st), step_of(sr) + (which == 1 ? 1 : 0))) return;
    const int f = blockIdx.x % FOLD_BLOCKS;
    int nb, nv;
    const double* rec;
    if (which == 3) {
        const int j = step_of(sr) - sl.j0;
        if (j == 0) {
            if (!sl.fold_upd) return;
            which = 2;
            nb = sl.npix;
            nv = 1 + zr_width(sl.st, sl.nz, 0);
            rec = sl.rec_upd;
        } else {
            if (!sl.fold_app) return;
            which = 1;
            nb = sl.ntiles;
            nv = 4 + sl.s + (j >= 2 ? zr_width(sl.st, sl.nz, j - 1) : 0);
            rec = ((j - 1) & 1) ? sl.rec_app2 : sl.rec_app;
        }
    } else if (which == 0) {
        nb = sl.ntiles;
        nv = 1 + sl.s;
        rec = sl.rec_res;
    } else if (which == 1) {
        nb = sl.ntiles;
        nv = 1 + sl.s;
        rec = sl.rec_app;
    } else {
        nb = sl.npix;
        nv = 1 + zr_width(sl.st, sl.nz, step_of(sr) - sl.j0);
        rec = sl.rec_upd;
    }
    const int b0 = (int)((long)f * nb / FOLD_BLOCKS), b1 = (int)((long)(f + 1) * nb / FOLD_BLOCKS);
    reduce_partials(rec + (size_t)b0 * nv, b1 - b0, nv, tot);
    double* out = sl.fold + (size_t)which * FOLD_BLOCKS * NV_RED + (size_t)f * nv;
    for (int k = threadIdx.x; k < nv; k += NT) out[k] = tot[k];
}

// Admission: descriptor `v` into slots[idx]; a zeroed SolveState with the settings of `init`
// and the selected generalized singular values mu (s values, device; may be null when s = 0).
__global__ void __launch_bounds__(NT) k_b_admit(Slot* __restrict__ slots, int idx, Slot v, StateInit init,
                                                const double* __restrict__ mu) {
    SolveState* st = v.st;
    int* words = reinterpret_cast<int*>(st);
    for (int k = threadIdx.x; k < (int)(sizeof(SolveState) / sizeof(int)); k += NT) words[k] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        slots[idx] = v;
        st->tol = init.tol;
        st->hg_tol = init.hg_tol;
        st->max_iter = init.max_iter;
        st->check_every = init.check_every;
        st->stop = init.stop;
        st->s = init.s;
        st->v_cap = init.v_cap;
        st->store_basis = init.store_basis;
        st->hgerr_on = init.hgerr_on;
        st->rr_j = -1;
    }
    for (int k = threadIdx.x; k < init.s; k += NT) st->mu[k] = mu[k];
}

// Restart index: the slot's next apply step runs iteration j = step - j0.
__global__ void k_b_set_j0(Slot* __restrict__ slots, int idx, int j0) {
    if (threadIdx.x == 0) slots[idx].j0 = j0;
}

// Scalar headers of the listed slots into out[slot index * HDR_BYTES] (4-byte words; out is
// pinned host memory that the host reads after the chunk's poll event), and the step counter
// advanced past the chunk (adv steps; no other block of this kernel reads it).
__global__ void __launch_bounds__(NT) k_b_headers(const Slot* __restrict__ slots, BatchMap M, int* __restrict__ out,
                                                  int* __restrict__ ctr, int adv) {
    constexpr int WPS = HDR_BYTES / 4;
    const int t = blockIdx.x * NT + threadIdx.x;
    if (t == 0) ctr[0] += adv;
    const int k = t / WPS, wd = t - k * WPS;
    if (k >= M.ns) return;
    const int idx = M.slot[k];
    out[(size_t)idx * WPS + wd] = reinterpret_cast<const int*>(slots[idx].st)[wd];
}

hipError_t launch_b_residual(const Stencil& base, int rows, bool rec, const Slot* slots, const BatchMap& M,
                             int periodic, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    switch (rows) {
        case QTY * 1: return launch_b_residual_q<1>(base, rec, slots, M, periodic, stream);
        case QTY * 2: return launch_b_residual_q<2>(base, rec, slots, M, periodic, stream);
        case QTY * 4: return launch_b_residual_q<4>(base, rec, slots, M, periodic, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_b_apply(const Stencil& base, int rows, bool rec, bool fp32, const Slot* slots, const BatchMap& M,
                          StepRef sr, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    switch (rows) {
        case QTY * 1: return launch_b_apply_q<1>(base, rec, fp32, slots, M, sr, stream);
        case QTY * 2: return launch_b_apply_q<2>(base, rec, fp32, slots, M, sr, stream);
        case QTY * 4: return launch_b_apply_q<4>(base, rec, fp32, slots, M, sr, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_f_step(const Stencil& base, int rows, bool rec, const Slot* slots, const BatchMap& M, StepRef sr,
                         const Slot* one, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    switch (rows) {
        case QTY * 1: return launch_f_step_q<1>(base, rec, slots, M, sr, one, stream);
        case QTY * 2: return launch_f_step_q<2>(base, rec, slots, M, sr, one, stream);
        case QTY * 4: return launch_f_step_q<4>(base, rec, slots, M, sr, one, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_b_init(const Slot* slots, const BatchMap& M, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_init, map_grid(M), dim3(NT), 0, stream, slots, M);
    return hipGetLastError();
}
hipError_t launch_b_update(const Slot* slots, const BatchMap& M, StepRef sr, bool rec, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    // a grid of at most 16 blocks per compute unit waits on memory latency, not bandwidth
    const bool wide = rec && map_grid(M).x <= 16 * 256;
    if (wide)
        hipLaunchKernelGGL((k_b_update<true, true>), map_grid(M), dim3(NT), 0, stream, slots, M, sr);
    else if (rec)
        hipLaunchKernelGGL((k_b_update<true, false>), map_grid(M), dim3(NT), 0, stream, slots, M, sr);
    else
        hipLaunchKernelGGL((k_b_update<false, false>), map_grid(M), dim3(NT), 0, stream, slots, M, sr);
    return hipGetLastError();
}
hipError_t launch_b_replace(const Slot* slots, const BatchMap& M, int periodic, StepRef sr, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_replace, map_grid(M), dim3(NT), 0, stream, slots, M, periodic, sr);
    return hipGetLastError();
}
hipError_t launch_b_finish(const Slot* slots, const BatchMap& M, hipStream_t stream) {
    if (M.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_finish, map_grid(M), dim3(NT), 0, stream, slots, M);
    return hipGetLastError();
}
hipError_t launch_b_fold(const Slot* slots, const BatchMap& list, int which, StepRef sr, hipStream_t stream) {
    if (list.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_fold, dim3(list.ns * FOLD_BLOCKS), dim3(NT), 0, stream, slots, list, which, sr);
    return hipGetLastError();
}
hipError_t launch_b_admit(Slot* slots, int idx, const Slot& v, const StateInit& init, const double* mu,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_b_admit, dim3(1), dim3(NT), 0, stream, slots, idx, v, init, mu);
    return hipGetLastError();
}
hipError_t launch_b_set_j0(Slot* slots, int idx, int j0, hipStream_t stream) {
    hipLaunchKernelGGL(k_b_set_j0, dim3(1), dim3(64), 0, stream, slots, idx, j0);
    return hipGetLastError();
}
hipError_t launch_b_headers(const Slot* slots, const BatchMap& list, int* out, int* ctr, int adv,
                            hipStream_t stream) {
    const int words = list.ns * (HDR_BYTES / 4);
    hipLaunchKernelGGL(k_b_headers, dim3(words > 0 ? (words + NT - 1) / NT : 1), dim3(NT), 0, stream, slots, list, out,
                       ctr, adv);
    return hipGetLastError();
}

}  // namespace bl
