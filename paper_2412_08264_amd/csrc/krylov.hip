// Elementwise kernels of recycled CG and of the L-BFGS vector algebra.
//
// No kernel synchronises its blocks.  Reductions leave one partial record per block; the
// next kernel in the stream reduces those records in every block (fixed order, so every
// block obtains identical scalars and takes identical decisions) and block 0 stores the
// scalars for the host.  Records that only the host needs are summed by k_finish_sum.
#include "kernels.h"

namespace bl {

// Update this thread's pixel (one pixel per thread: the grid covers n exactly), then
// write the block record [r.r, Z^T r (nz values)].
template <typename Body>
__device__ __forceinline__ void residual_record(const double* __restrict__ Z, int n, int nz, double* part,
                                                Body body) {
    const int i = blockIdx.x * NT + threadIdx.x;
    const bool in = i < n;
    const double ri = in ? body(i) : 0.0;
    block_partials(part, 1 + nz, [&](int k) -> double {
        if (!in) return 0.0;
        return k == 0 ? ri * ri : Z[(size_t)(k - 1) * n + i] * ri;
    });
}

// Set-up after r = g - H w0 (record [g.g, C^T r]):  w += U c0;  r -= C c0.
__global__ void __launch_bounds__(NT) k_cg_init(int n, double* __restrict__ w, double* __restrict__ r,
                                                const double* __restrict__ U, const double* __restrict__ C,
                                                const double* __restrict__ Z, SolveState* st,
                                                const double* __restrict__ res_part, int res_nb,
                                                double* __restrict__ upd_part) {
    __shared__ double tot[NT];
    const int s = st->s;
    reduce_partials(res_part, res_nb, 1 + s, tot);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->gnorm = sqrt(tot[0]);
    const double* c0 = tot + 1;
    const int nz = st->hgerr_on ? s : 0;
    residual_record(Z, n, nz, upd_part, [&](int i) {
        w[i] += combo(U, n, i, c0, s);
        const double ri = r[i] - combo(C, n, i, c0, s);
        r[i] = ri;
        return ri;
    });
}

// Iteration j, second half: sigma = p.q and e = C^T q from the apply records;
// alpha = rho_j / sigma;  w += alpha p;  r -= alpha (q - C e);  z -= alpha e.
__global__ void __launch_bounds__(NT) k_cg_update(int n, int j, double* __restrict__ w, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ C, const double* __restrict__ Z,
                                                  SolveState* st, const double* __restrict__ app_part, int app_nb,
                                                  double* __restrict__ upd_part) {
    if (st->done) return;
    __shared__ double tot[NT];
    const int s = st->s;
    reduce_partials(app_part, app_nb, 1 + s, tot);
    const double sigma = tot[0];
    if (!(sigma > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->status = (sigma != sigma || fabs(sigma) == INFINITY) ? BL_E_NONFINITE : BL_E_INDEFINITE;
            st->iters = j;
            st->done = 1;
        }
        return;
    }
    const double alpha = st->rho2[j & 1] / sigma;
    const double* e = tot + 1;
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < s; k += NT) st->zacc[k] -= alpha * e[k];
        if (threadIdx.x == 0) st->alpha = alpha;
    }
    const int nz = st->hgerr_on ? s : 0;
    residual_record(Z, n, nz, upd_part, [&](int i) {
        const double ce = combo(C, n, i, e, s);
        w[i] += alpha * p[i];
        const double ri = r[i] - alpha * (q[i] - ce);
        r[i] = ri;
        return ri;
    });
}

// Residual replacement: r holds t = g - H w and the records [g.g, C^T t]:
// z := C^T t;  r := t - C z;  the solve resumes (the next apply step re-tests).
__global__ void __launch_bounds__(NT) k_cg_replace(int n, double* __restrict__ r, const double* __restrict__ C,
                                                   const double* __restrict__ Z, SolveState* st,
                                                   const double* __restrict__ res_part, int res_nb,
                                                   double* __restrict__ upd_part) {
    __shared__ double tot[NT];
    const int s = st->s;
    reduce_partials(res_part, res_nb, 1 + s, tot);
    const double* c = tot + 1;
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < s; k += NT) st->zacc[k] = c[k];
        if (threadIdx.x == 0) {
            st->done = 0;
            st->status = BL_OK;
        }
    }
    const int nz = st->hgerr_on ? s : 0;
    residual_record(Z, n, nz, upd_part, [&](int i) {
        const double ri = r[i] - combo(C, n, i, c, s);
        r[i] = ri;
        return ri;
    });
}

// w += U z.
__global__ void __launch_bounds__(NT) k_cg_finish(int n, double* __restrict__ w, const double* __restrict__ U,
                                                  const SolveState* st) {
    __shared__ double z[S_MAX];
    const int s = st->s;
    for (int k = threadIdx.x; k < s; k += NT) z[k] = st->zacc[k];
    __syncthreads();
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) w[i] += combo(U, n, i, z, s);
}

// out[k] = sum of the records (one block).
__global__ void __launch_bounds__(NT) k_finish_sum(const double* __restrict__ part, int nb, int nv,
                                                   double* __restrict__ out) {
    __shared__ double tot[NT];
    reduce_partials(part, nb, nv, tot);
    for (int k = threadIdx.x; k < nv; k += NT) out[k] = tot[k];
}

// ------------------------------------------------------------------ L-BFGS vector algebra
// Block records of up to three dots: [a.b, a.a, b.b] (first `nv` of them).
__global__ void __launch_bounds__(NT) k_dots_part(int n, int nv, const double* __restrict__ a,
                                                  const double* __restrict__ b, double* __restrict__ part) {
    double ab = 0.0, aa = 0.0, bb = 0.0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const double x = a[i], y = b[i];
        ab += x * y;
        aa += x * x;
        bb += y * y;
    }
    block_partials(part, nv, [&](int k) { return k == 0 ? ab : (k == 1 ? aa : bb); });
}

// y = beta y + (s1 sum(part1) + s2 sum(part2)) x; a null record stands for the value 1 / 0.
__global__ void __launch_bounds__(NT) k_axpy_red(int n, double beta, double* __restrict__ y,
                                                 const double* __restrict__ x, const double* __restrict__ part1,
                                                 double s1, const double* __restrict__ part2, double s2, int nb) {
    __shared__ double t1[NT], t2[NT];
    double c1 = 1.0, c2 = 0.0;
    if (part1) {
        reduce_partials(part1, nb, 1, t1);
        c1 = t1[0];
    }
    if (part2) {
        reduce_partials(part2, nb, 1, t2);
        c2 = t2[0];
    }
    const double a = s1 * c1 + s2 * c2;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + a * x[i];   // beta = 0 ignores y (may be uninitialised)
}

// out = a - b
__global__ void __launch_bounds__(NT) k_sub(int n, const double* __restrict__ a, const double* __restrict__ b,
                                            double* __restrict__ out) {
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) out[i] = a[i] - b[i];
}

// ------------------------------------------------------------------ launchers
// One pixel per thread (the residual-record kernels rely on it).
int red_blocks(int n) { return (n + NT - 1) / NT; }
// Blocks of the grid-stride vector kernels.
int vec_blocks(int n) {
    const int b = (n + NT * 4 - 1) / (NT * 4);
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

hipError_t launch_cg_init(int n, double* w, double* r, const double* U, const double* C, const double* Z,
                          SolveState* st, const double* res_part, int res_nb, double* upd_part, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_init, dim3(red_blocks(n)), dim3(NT), 0, stream, n, w, r, U, C, Z, st, res_part, res_nb,
                       upd_part);
    return hipGetLastError();
}
hipError_t launch_cg_update(int n, int j, double* w, double* r, const double* p, const double* q, const double* C,
                            const double* Z, SolveState* st, const double* app_part, int app_nb, double* upd_part,
                            hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_update, dim3(red_blocks(n)), dim3(NT), 0, stream, n, j, w, r, p, q, C, Z, st, app_part,
                       app_nb, upd_part);
    return hipGetLastError();
}
hipError_t launch_cg_replace(int n, double* r, const double* C, const double* Z, SolveState* st,
                             const double* res_part, int res_nb, double* upd_part, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_replace, dim3(red_blocks(n)), dim3(NT), 0, stream, n, r, C, Z, st, res_part, res_nb,
                       upd_part);
    return hipGetLastError();
}
hipError_t launch_cg_finish(int n, double* w, const double* U, const SolveState* st, hipStream_t stream) {
    hipLaunchKernelGGL(k_cg_finish, dim3(vec_blocks(n)), dim3(NT), 0, stream, n, w, U, st);
    return hipGetLastError();
}
hipError_t launch_finish_sum(const double* part, int nb, int nv, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(NT), 0, stream, part, nb, nv, out);
    return hipGetLastError();
}
hipError_t launch_dots_part(int n, int nv, const double* a, const double* b, double* part, hipStream_t stream) {
    hipLaunchKernelGGL(k_dots_part, dim3(vec_blocks(n)), dim3(NT), 0, stream, n, nv, a, b, part);
    return hipGetLastError();
}
hipError_t launch_axpy_red(int n, double beta, double* y, const double* x, const double* part1, double s1,
                           const double* part2, double s2, hipStream_t stream) {
    hipLaunchKernelGGL(k_axpy_red, dim3(vec_blocks(n)), dim3(NT), 0, stream, n, beta, y, x, part1, s1, part2, s2,
                       vec_blocks(n));
    return hipGetLastError();
}
hipError_t launch_sub(int n, const double* a, const double* b, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_sub, dim3(vec_blocks(n)), dim3(NT), 0, stream, n, a, b, out);
    return hipGetLastError();
}

}  // namespace bl
