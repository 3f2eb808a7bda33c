// Elementwise kernels of recycled CG with fused reductions and device-side stop tests.
#include "kernels.h"

namespace bl {

// Stop decision after a residual update (thread 0 of the last block).  Order of tests:
// exact zero residual; only every check_every iterations; error estimate (when enabled)
// or relative residual; then the iteration limit.
__device__ void stop_logic(SolveState* st, double rho_new, bool at_init) {
    double est = NAN;
    if (st->hgerr_on) {
        double acc = 0.0;
        for (int k = 0; k < st->s; ++k) {
            const double t = st->mu[k] * st->zr[k];
            acc += t * t;
        }
        est = sqrt(acc);
    }
    st->est = est;
    if (!(rho_new == rho_new) || fabs(rho_new) == INFINITY) {
        st->status = BL_E_NONFINITE;
        st->done = 1;
        st->rho = rho_new;
        return;
    }
    if (!at_init) st->beta = rho_new / st->rho;
    const int it = st->iters;
    bool met;
    if (rho_new == 0.0) met = true;
    else if (it % st->check_every) met = false;
    else if (st->stop == BL_STOP_HGERR && st->hgerr_on) met = est <= st->hg_tol;
    else met = sqrt(rho_new) <= st->tol * st->gnorm;
    if (met) {
        st->done = 1;
        st->status = BL_OK;
    } else if (it >= st->max_iter) {
        st->done = 1;
        st->status = BL_E_NOT_CONVERGED;
    }
    st->rho = rho_new;
}

// Reductions r.r and (with the error estimate) Z^T r of this thread's pixels.
template <typename Body>
__device__ __forceinline__ void residual_reductions(const double* __restrict__ Z, int n, int nz, double* part,
                                                    double* red, Body body) {
    // body(i) updates pixel i and returns r_i
    double rr = 0.0;
    double zr[8];
    const int chunks = (nz + 7) / 8;
    // first pass computes r and r.r, Z^T r in groups of 8 columns
    for (int ch = 0; ch < (chunks > 0 ? chunks : 1); ++ch) {
#pragma unroll
        for (int k = 0; k < 8; ++k) zr[k] = 0.0;
        for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
            double ri = body(i, ch == 0);
            if (ch == 0) rr += ri * ri;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int col = ch * 8 + k;
                if (col < nz) zr[k] += Z[(size_t)col * n + i] * ri;
            }
        }
        if (ch == 0) {
            const double s = block_sum(rr, red);
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * (1 + nz)] = s;
        }
        for (int k = 0; k < 8; ++k) {
            const int col = ch * 8 + k;
            if (col >= nz) break;
            const double s = block_sum(zr[k], red);
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * (1 + nz) + 1 + col] = s;
        }
    }
}

// w = w0 + U c0;  r = r - C c0;  then r.r, Z^T r and the stop test at j = 0.
__global__ void __launch_bounds__(NT) k_cg_init(int n, double* __restrict__ w, double* __restrict__ r,
                                                const double* __restrict__ U, const double* __restrict__ C,
                                                const double* __restrict__ Z, SolveState* st, double* part,
                                                unsigned* counter) {
    __shared__ double red[NWAVE];
    __shared__ double c0[S_MAX];
    __shared__ double tot[1 + S_MAX];
    const int s = st->s;
    for (int k = threadIdx.x; k < s; k += NT) c0[k] = st->c0[k];
    __syncthreads();
    const int nz = st->hgerr_on ? s : 0;
    residual_reductions(Z, n, nz, part, red, [&](int i, bool write) {
        if (!write) return r[i];
        double uc = 0.0, cc = 0.0;
        for (int k = 0; k < s; ++k) {
            uc += U[(size_t)k * n + i] * c0[k];
            cc += C[(size_t)k * n + i] * c0[k];
        }
        w[i] += uc;
        const double ri = r[i] - cc;
        r[i] = ri;
        return ri;
    });
    if (!last_block(counter, gridDim.x)) return;
    reduce_partials(part, gridDim.x, 1 + nz, tot, red);
    for (int k = threadIdx.x; k < nz; k += NT) st->zr[k] = tot[1 + k];
    __syncthreads();
    if (threadIdx.x == 0) {
        st->res0 = sqrt(tot[0]);
        st->iters = 0;
        st->beta = 0.0;
        stop_logic(st, tot[0], true);
    }
}

// w += alpha p;  r -= alpha (q - C e);  then r.r, Z^T r and the stop test.
__global__ void __launch_bounds__(NT) k_cg_update(int n, double* __restrict__ w, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ C, const double* __restrict__ Z,
                                                  SolveState* st, double* part, unsigned* counter) {
    if (st->done) return;
    __shared__ double red[NWAVE];
    __shared__ double e[S_MAX];
    __shared__ double tot[1 + S_MAX];
    const int s = st->s;
    const double alpha = st->alpha;
    for (int k = threadIdx.x; k < s; k += NT) e[k] = st->e[k];
    __syncthreads();
    const int nz = st->hgerr_on ? s : 0;
    residual_reductions(Z, n, nz, part, red, [&](int i, bool write) {
        if (!write) return r[i];
        double ce = 0.0;
        for (int k = 0; k < s; ++k) ce += C[(size_t)k * n + i] * e[k];
        w[i] += alpha * p[i];
        const double ri = r[i] - alpha * (q[i] - ce);
        r[i] = ri;
        return ri;
    });
    if (!last_block(counter, gridDim.x)) return;
    reduce_partials(part, gridDim.x, 1 + nz, tot, red);
    for (int k = threadIdx.x; k < nz; k += NT) st->zr[k] = tot[1 + k];
    __syncthreads();
    if (threadIdx.x == 0) {
        st->iters += 1;
        stop_logic(st, tot[0], false);
    }
}

// Residual replacement: given t = g - H w (in r) and c = C^T t (in st->c0):
// z := c,  r := t - C c;  then r.r, Z^T r and the stop test (the iteration count is kept).
__global__ void __launch_bounds__(NT) k_cg_replace(int n, double* __restrict__ r, const double* __restrict__ C,
                                                   const double* __restrict__ Z, SolveState* st, double* part,
                                                   unsigned* counter) {
    __shared__ double red[NWAVE];
    __shared__ double c0[S_MAX];
    __shared__ double tot[1 + S_MAX];
    const int s = st->s;
    for (int k = threadIdx.x; k < s; k += NT) c0[k] = st->c0[k];
    __syncthreads();
    const int nz = st->hgerr_on ? s : 0;
    residual_reductions(Z, n, nz, part, red, [&](int i, bool write) {
        if (!write) return r[i];
        double cc = 0.0;
        for (int k = 0; k < s; ++k) cc += C[(size_t)k * n + i] * c0[k];
        const double ri = r[i] - cc;
        r[i] = ri;
        return ri;
    });
    if (!last_block(counter, gridDim.x)) return;
    reduce_partials(part, gridDim.x, 1 + nz, tot, red);
    for (int k = threadIdx.x; k < nz; k += NT) st->zr[k] = tot[1 + k];
    for (int k = threadIdx.x; k < s; k += NT) st->zacc[k] = c0[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        // re-test with the true residual at the current iteration count; beta is kept
        st->rho_true = tot[0];
        st->done = 0;
        st->status = BL_OK;
        const int saved_check = st->check_every;
        const double beta = st->beta;
        st->check_every = 1;
        stop_logic(st, tot[0], true);
        st->check_every = saved_check;
        st->beta = beta;
    }
}

// w += U z.
__global__ void __launch_bounds__(NT) k_cg_finish(int n, double* __restrict__ w, const double* __restrict__ U,
                                                  const SolveState* st) {
    __shared__ double z[S_MAX];
    const int s = st->s;
    for (int k = threadIdx.x; k < s; k += NT) z[k] = st->zacc[k];
    __syncthreads();
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        double acc = 0.0;
        for (int k = 0; k < s; ++k) acc += U[(size_t)k * n + i] * z[k];
        w[i] += acc;
    }
}

// ------------------------------------------------------------------ generic vector kernels
// out = sum_k coef[k] * vec[k]  (coefficients in device memory, sign-scaled by `scale`)
__global__ void __launch_bounds__(NT) k_lincomb(int n, int nvec, const double* const* __restrict__ vecs,
                                                const double* __restrict__ coef, double scale, double* out,
                                                int accumulate) {
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        double acc = accumulate ? out[i] : 0.0;
        for (int k = 0; k < nvec; ++k) acc += scale * coef[k] * vecs[k][i];
        out[i] = acc;
    }
}

// dots[k] = a_k . b_k for k < npair (vector pointers in device memory); deterministic.
__global__ void __launch_bounds__(NT) k_dots(int n, int npair, const double* const* __restrict__ a,
                                             const double* const* __restrict__ b, double* part, unsigned* counter,
                                             double* dots) {
    __shared__ double red[NWAVE];
    __shared__ double tot[NV_RED];
    for (int k = 0; k < npair; ++k) {
        double acc = 0.0;
        for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) acc += a[k][i] * b[k][i];
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * npair + k] = s;
    }
    if (!last_block(counter, gridDim.x)) return;
    reduce_partials(part, gridDim.x, npair, tot, red);
    for (int k = threadIdx.x; k < npair; k += NT) dots[k] = tot[k];
}

// y = x + alpha_dev[0] * scale * d  (line-search trial point, step on the device)
__global__ void __launch_bounds__(NT) k_axpy_dev(int n, const double* __restrict__ x, const double* __restrict__ d,
                                                 const double* __restrict__ alpha, double scale, double* y) {
    const double a = alpha[0] * scale;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) y[i] = x[i] + a * d[i];
}

// out[0] = a . b (deterministic), last block writes.
__global__ void __launch_bounds__(NT) k_dot_to(int n, const double* __restrict__ a, const double* __restrict__ b,
                                               double* part, unsigned* counter, double* out) {
    __shared__ double red[NWAVE];
    __shared__ double tot[1];
    double acc = 0.0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) acc += a[i] * b[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (!last_block(counter, gridDim.x)) return;
    reduce_partials(part, gridDim.x, 1, tot, red);
    if (threadIdx.x == 0) out[0] = tot[0];
}

// Three dots at once: out = [a.b, a.a, b.b].
__global__ void __launch_bounds__(NT) k_dots3(int n, const double* __restrict__ a, const double* __restrict__ b,
                                              double* part, unsigned* counter, double* out) {
    __shared__ double red[NWAVE];
    __shared__ double tot[3];
    double ab = 0.0, aa = 0.0, bb = 0.0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        ab += a[i] * b[i];
        aa += a[i] * a[i];
        bb += b[i] * b[i];
    }
    ab = block_sum(ab, red);
    aa = block_sum(aa, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3] = ab;
        part[blockIdx.x * 3 + 1] = aa;
        part[blockIdx.x * 3 + 2] = bb;
    }
    if (!last_block(counter, gridDim.x)) return;
    reduce_partials(part, gridDim.x, 3, tot, red);
    if (threadIdx.x < 3) out[threadIdx.x] = tot[threadIdx.x];
}

// y = beta y + (s1 c1[0] + s2 c2[0]) x   (c1/c2 device scalars, may be null: treated as 1 / 0)
__global__ void __launch_bounds__(NT) k_axpy2(int n, double beta, double* __restrict__ y, const double* __restrict__ x,
                                              const double* __restrict__ c1, double s1, const double* __restrict__ c2,
                                              double s2) {
    const double a = s1 * (c1 ? c1[0] : 1.0) + (c2 ? s2 * c2[0] : 0.0);
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + a * x[i];   // beta = 0 ignores y (may be uninitialised)
}

// out = a - b
__global__ void __launch_bounds__(NT) k_sub(int n, const double* __restrict__ a, const double* __restrict__ b,
                                            double* __restrict__ out) {
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) out[i] = a[i] - b[i];
}

int red_blocks(int n) {
    int b = (n + NT * 4 - 1) / (NT * 4);
    if (b > RED_BLOCKS) b = RED_BLOCKS;
    return b < 1 ? 1 : b;
}

hipError_t launch_cg_init(int n, double* w, double* r, const double* U, const double* C, const double* Z,
                          SolveState* st, double* part, unsigned* counter, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_init, dim3(red_blocks(n)), dim3(NT), 0, stream, n, w, r, U, C, Z, st, part, counter);
    return hipGetLastError();
}
hipError_t launch_cg_update(int n, double* w, double* r, const double* p, const double* q, const double* C,
                            const double* Z, SolveState* st, double* part, unsigned* counter, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_update, dim3(red_blocks(n)), dim3(NT), 0, stream, n, w, r, p, q, C, Z, st, part,
                       counter);
    return hipGetLastError();
}
hipError_t launch_cg_replace(int n, double* r, const double* C, const double* Z, SolveState* st, double* part,
                             unsigned* counter, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_replace, dim3(red_blocks(n)), dim3(NT), 0, stream, n, r, C, Z, st, part, counter);
    return hipGetLastError();
}
hipError_t launch_cg_finish(int n, double* w, const double* U, const SolveState* st, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_finish, dim3(red_blocks(n)), dim3(NT), 0, stream, n, w, U, st);
    return hipGetLastError();
}
hipError_t launch_lincomb(int n, int nvec, const double* const* vecs, const double* coef, double scale, double* out,
                          int accumulate, hipStream_t stream) {
    hipLaunchKernelGGL(k_lincomb, dim3(red_blocks(n)), dim3(NT), 0, stream, n, nvec, vecs, coef, scale, out,
                       accumulate);
    return hipGetLastError();
}
hipError_t launch_dots(int n, int npair, const double* const* a, const double* const* b, double* part,
                       unsigned* counter, double* dots, hipStream_t stream) {
    hipLaunchKernelGGL(k_dots, dim3(red_blocks(n)), dim3(NT), 0, stream, n, npair, a, b, part, counter, dots);
    return hipGetLastError();
}
hipError_t launch_dot_to(int n, const double* a, const double* b, double* part, unsigned* counter, double* out,
                         hipStream_t stream) {
    hipLaunchKernelGGL(k_dot_to, dim3(red_blocks(n)), dim3(NT), 0, stream, n, a, b, part, counter, out);
    return hipGetLastError();
}
hipError_t launch_dots3(int n, const double* a, const double* b, double* part, unsigned* counter, double* out,
                        hipStream_t stream) {
    hipLaunchKernelGGL(k_dots3, dim3(red_blocks(n)), dim3(NT), 0, stream, n, a, b, part, counter, out);
    return hipGetLastError();
}
hipError_t launch_axpy2(int n, double beta, double* y, const double* x, const double* c1, double s1, const double* c2,
                        double s2, hipStream_t stream) {
    hipLaunchKernelGGL(k_axpy2, dim3(red_blocks(n)), dim3(NT), 0, stream, n, beta, y, x, c1, s1, c2, s2);
    return hipGetLastError();
}
hipError_t launch_sub(int n, const double* a, const double* b, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_sub, dim3(red_blocks(n)), dim3(NT), 0, stream, n, a, b, out);
    return hipGetLastError();
}
hipError_t launch_axpy_dev(int n, const double* x, const double* d, const double* alpha, double scale, double* y,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_axpy_dev, dim3(red_blocks(n)), dim3(NT), 0, stream, n, x, d, alpha, scale, y);
    return hipGetLastError();
}

}  // namespace bl
