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

// ------------------------------------------------------------------ launchers
// One pixel per thread (the residual-record kernels rely on it).
int red_blocks(int n) { return (n + NT - 1) / NT; }
// Blocks of the grid-stride vector kernels.
int vec_blocks(int n) {
    const int b = (n + NT * 4 - 1) / (NT * 4);
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
hipError_t launch_sub(int n, const double* a, const double* b, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_sub, dim3(vec_blocks(n)), dim3(NT), 0, stream, n, a, b, out);
    return hipGetLastError();
}

}  // namespace bl
