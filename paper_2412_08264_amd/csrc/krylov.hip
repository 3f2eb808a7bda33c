// Record folding and the vector algebra of the lower-level L-BFGS solve.
//
// No kernel synchronises its blocks.  Reductions leave one partial record per block; the
// next kernel in the stream reduces those records in every block (fixed order, so every
// block obtains identical scalars).  Records that only the host needs are summed by
// k_finish_sum.
#include "kernels.h"

namespace bl {

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

// Dots a_i . b_i of up to VL_MAX vector pairs in one pass (records: one per block, k values).
__global__ void __launch_bounds__(NT) k_multidot(int n, VecPairs vp, double* __restrict__ part) {
    double acc[VL_MAX];
#pragma unroll
    for (int i = 0; i < VL_MAX; ++i) acc[i] = 0.0;
    for (int p = blockIdx.x * NT + threadIdx.x; p < n; p += gridDim.x * NT) {
#pragma unroll
        for (int i = 0; i < VL_MAX; ++i)
            if (i < vp.k) acc[i] += vp.a[i][p] * vp.b[i][p];
    }
    block_partials(part, vp.k, [&](int i) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < VL_MAX; ++u)
            if (u == i) v = acc[u];
        return v;
    });
}

// out = c0 x0 + sum_i c_i v_i (i < k).
__global__ void __launch_bounds__(NT) k_lincomb(int n, double c0, const double* __restrict__ x0, VecComb vc,
                                                double* __restrict__ out) {
    for (int p = blockIdx.x * NT + threadIdx.x; p < n; p += gridDim.x * NT) {
        double acc = c0 * x0[p];
#pragma unroll 8
        for (int i = 0; i < vc.k; ++i) acc += vc.c[i] * vc.v[i][p];
        out[p] = acc;
    }
}

// ------------------------------------------------------------------ launchers
// One pixel per thread (the residual-record kernels rely on it).
int red_blocks(int n) { return (n + NT - 1) / NT; }
// Blocks of the grid-stride vector kernels.
int vec_blocks(int n) {
    const int b = (n + NT * 4 - 1) / (NT * 4);
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

// Blocks of the many-vector kernels (multi-dot, linear combination): one pixel per thread up to
// 1024 blocks, so that a 256 x 256 image spreads over every compute unit.
int wide_blocks(int n) {
    const int b = red_blocks(n);
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
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
hipError_t launch_multidot(int n, const VecPairs& vp, double* part, hipStream_t stream) {
    hipLaunchKernelGGL(k_multidot, dim3(wide_blocks(n)), dim3(NT), 0, stream, n, vp, part);
    return hipGetLastError();
}
hipError_t launch_lincomb(int n, double c0, const double* x0, const VecComb& vc, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_lincomb, dim3(wide_blocks(n)), dim3(NT), 0, stream, n, c0, x0, vc, out);
    return hipGetLastError();
}
hipError_t launch_sub(int n, const double* a, const double* b, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_sub, dim3(vec_blocks(n)), dim3(NT), 0, stream, n, a, b, out);
    return hipGetLastError();
}

}  // namespace bl
