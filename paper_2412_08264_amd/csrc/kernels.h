// Launchers of the HIP kernels (host side), shared by the translation units.
#pragma once

#include "common.h"

namespace bl {

// stencil.hip
int tiles_of(const Stencil& S);
// H v for ncols columns on tiles of `rows` (8, 16 or 32) rows; batch_q{1,2,4}.hip instantiate it.
hipError_t launch_hvp(const Stencil& S, bool fp32, const double* xhat, const double* v, double* out, int ncols,
                      int rows, hipStream_t st);
template <int Q>
hipError_t launch_hvp_q(const Stencil& S, bool fp32, const double* xhat, const double* v, double* out, int ncols,
                        hipStream_t st);
hipError_t launch_filter_state(const Stencil& S, const double* xhat, double* d1, double* d2, float* d2f,
                               hipStream_t stream);
int jac_blocks(const Stencil& S);
hipError_t launch_jac(const Stencil& S, const double* xhat, const double* w, int ncols, const double* d1,
                      const double* d2, double* part, double* G, int project, hipStream_t stream);
hipError_t launch_lower_grad(const Stencil& S, const double* x, const double* y, double* grad, double* part,
                             hipStream_t stream);
hipError_t launch_forward(const Stencil& S, const double* x, const double* e, double noise, double* y,
                          hipStream_t stream);

// krylov.hip
// Up to VL_MAX dot products in one pass, and a linear combination of up to VC_MAX vectors.
constexpr int VL_MAX = 24;
constexpr int VC_MAX = 40;
struct VecPairs {
    int k;
    const double* a[VL_MAX];
    const double* b[VL_MAX];
};
struct VecComb {
    int k;
    double c[VC_MAX];
    const double* v[VC_MAX];
};
hipError_t launch_multidot(int n, const VecPairs& vp, double* part, hipStream_t stream);
hipError_t launch_lincomb(int n, double c0, const double* x0, const VecComb& vc, double* out, hipStream_t stream);
int red_blocks(int n);
int vec_blocks(int n);
int wide_blocks(int n);   // blocks of launch_multidot / launch_lincomb (records: one per block)
hipError_t launch_finish_sum(const double* part, int nb, int nv, double* out, hipStream_t stream);
hipError_t launch_dots_part(int n, int nv, const double* a, const double* b, double* part, hipStream_t stream);
hipError_t launch_axpy_red(int n, double beta, double* y, const double* x, const double* part1, double s1,
                           const double* part2, double s2, hipStream_t stream);
hipError_t launch_sub(int n, const double* a, const double* b, double* out, hipStream_t stream);

// batch.hip: recycled CG over a batch of slots (one launch per half-iteration).  The tile-grid
// kernels take the tile height in rows (8, 16 or 32); batch_q{1,2,4}.hip instantiate them.
// `rec`: the slots of the launch have recycle spaces (all of them, or none).
hipError_t launch_b_residual(const Stencil& base, int rows, bool rec, const Slot* slots, const BatchMap& M,
                             int periodic, hipStream_t stream);
hipError_t launch_b_apply(const Stencil& base, int rows, bool rec, bool fp32, const Slot* slots, const BatchMap& M,
                          StepRef sr, hipStream_t stream);
// Fused FP64 step of the recycled CG (one launch per iteration), on tiles of `rows` rows.  `one`
// (host memory, may be null): the descriptor of the launch's only slot, passed by value with the
// kernel arguments when the map holds one slot; it must equal slots[M.slot[0]].
hipError_t launch_f_step(const Stencil& base, int rows, bool rec, const Slot* slots, const BatchMap& M, StepRef sr,
                         const Slot* one, hipStream_t stream);
template <int Q>
hipError_t launch_f_step_q(const Stencil& base, bool rec, const Slot* slots, const BatchMap& M, StepRef sr,
                           const Slot* one, hipStream_t stream);
template <int Q>
hipError_t launch_b_residual_q(const Stencil& base, bool rec, const Slot* slots, const BatchMap& M, int periodic,
                               hipStream_t stream);
template <int Q>
hipError_t launch_b_apply_q(const Stencil& base, bool rec, bool fp32, const Slot* slots, const BatchMap& M,
                            StepRef sr, hipStream_t stream);
#define BL_TILE_EXTERN(Q)                                                                                        \
    extern template hipError_t launch_b_residual_q<Q>(const Stencil&, bool, const Slot*, const BatchMap&, int,    \
                                                      hipStream_t);                                               \
    extern template hipError_t launch_b_apply_q<Q>(const Stencil&, bool, bool, const Slot*, const BatchMap&,      \
                                                   StepRef, hipStream_t);                                         \
    extern template hipError_t launch_f_step_q<Q>(const Stencil&, bool, const Slot*, const BatchMap&, StepRef,    \
                                                  const Slot*, hipStream_t);
#define BL_HVP_EXTERN(Q)                                                                                   \
    extern template hipError_t launch_hvp_q<Q>(const Stencil&, bool, const double*, const double*, double*, int, \
                                               hipStream_t);
BL_HVP_EXTERN(1)
BL_HVP_EXTERN(2)
BL_HVP_EXTERN(4)
#undef BL_HVP_EXTERN
BL_TILE_EXTERN(1)
BL_TILE_EXTERN(2)
BL_TILE_EXTERN(4)
#undef BL_TILE_EXTERN
hipError_t launch_b_init(const Slot* slots, const BatchMap& M, hipStream_t stream);
hipError_t launch_b_update(const Slot* slots, const BatchMap& M, StepRef sr, bool rec, hipStream_t stream);
hipError_t launch_b_replace(const Slot* slots, const BatchMap& M, int periodic, StepRef sr, hipStream_t stream);
hipError_t launch_b_finish(const Slot* slots, const BatchMap& M, hipStream_t stream);
hipError_t launch_b_fold(const Slot* slots, const BatchMap& list, int which, StepRef sr, hipStream_t stream);
hipError_t launch_b_admit(Slot* slots, int idx, const Slot& v, const StateInit& init, const double* mu,
                          hipStream_t stream);
hipError_t launch_b_set_j0(Slot* slots, int idx, int j0, hipStream_t stream);
hipError_t launch_b_headers(const Slot* slots, const BatchMap& list, int* out, int* ctr, int adv,
                            hipStream_t stream);

// rminres.hip: RMINRES (Algorithm 3) on 32 x 8 tiles, FP64, one solve.
// Scalars of the solve; slot k & 3 of a recurrence array holds step k's value.  Kernels read
// values of earlier steps and block 0 writes the current step's, so no block reads a slot
// that another block of the same launch writes.
struct MinresState {
    int done, status, iters, v_cur;     // header polled by the host
    double res, res0, est, gnorm;
    double tol, hg_tol;
    int max_iter, check_every, stop, s, nz, hgerr_on, store, v_cap;
    double beta[4], alpha[4], c[4], sn[4], zeta[4], gam[4], del[4], epst[4];
    double e[4][S_MAX];       // C^T H v_k
    double mh[4][S_MAX];      // b~_k in the coordinates of U (b~_k = U mh_k)
    double zacc[S_MAX];       // sum over steps of c_k zeta_{k-1} mh_k
    double mu[S_MAX];
};
struct MinresInit {
    double tol, hg_tol;
    int max_iter, check_every, stop, s, nz, hgerr_on, store, v_cap;
    const double* mu;         // device, s values (may be null when s = 0)
};
struct MinresArgs {
    const double* xhat;
    const double* g;
    double* w;
    double* r;
    double* q;
    double* u[3];             // unnormalised Lanczos vectors: u_k = beta_k v_k in u[k % 3]
    double* m[2];             // v~_k in m[k & 1]
    const double* U;
    const double* C;
    const double* Z;
    double* V;                // stored Lanczos vectors (store != 0)
    MinresState* st;
    double* rec_res;          // records of the residual launch (tiles x (1 + s))
    double* rec_app;          // records of the apply launch (tiles x (1 + s))
    double* rec_upd;          // records of the set-up and update launches (pixel blocks x (1 + nz))
    double* fold;             // FOLD_BLOCKS folded records of NV_RED values
    int n, ntiles, npix, s, nz;
};
hipError_t launch_m_residual(const Stencil& S, const MinresArgs& a, hipStream_t stream);
hipError_t launch_m_init(const MinresArgs& a, const MinresInit& in, bool fold, hipStream_t stream);
hipError_t launch_m_apply(const Stencil& S, const MinresArgs& a, int k, int nvb, bool fold, hipStream_t stream);
hipError_t launch_m_update(const MinresArgs& a, int k, int nvb, bool fold, hipStream_t stream);
hipError_t launch_m_finish(const MinresArgs& a, hipStream_t stream);
hipError_t launch_m_fold(const double* rec, int nb, int nv, double* out, hipStream_t stream);

// deflated.hip: deflated CG on 32 x 8 tiles, FP64, one solve (scalars in a SolveState).
struct DeflArgs {
    const double* xhat;
    const double* g;
    double* w;
    double* r;
    double* p[2];             // p_j in p[j & 1]
    double* q;
    const double* U;
    const double* C;
    const double* Z;
    const double* mu;         // selected generalized singular values (s, device; may be null)
    const double* Einv;       // (U^T C)^{-1}, s x s
    double* V;                // stored normalised residuals (store_basis)
    SolveState* st;
    double* rec_res;          // records: residual (tiles x (1 + s)), apply (tiles x 1),
    double* rec_app;          // set-up and update (pixel blocks x (1 + s + nz))
    double* rec_upd;
    double* fold;             // FOLD_BLOCKS folded records
    int n, ntiles, npix, s, nz;
};
hipError_t launch_d_residual(const Stencil& S, const DeflArgs& a, hipStream_t stream);
hipError_t launch_d_einv(int s, const double* UtC, double* Lscr, double* Einv, int* info, hipStream_t stream);
hipError_t launch_d_init(const DeflArgs& a, const StateInit& in, bool fold, hipStream_t stream);
hipError_t launch_d_apply(const Stencil& S, const DeflArgs& a, int j, int zw, bool fold, hipStream_t stream);
hipError_t launch_d_update(const DeflArgs& a, int j, int zw, bool fold, hipStream_t stream);

// dense.hip
int gram_chunks(int n);
hipError_t launch_gram(int n, int t1, int t2, const double* A, const double* B, double* part, double* out,
                       hipStream_t stream);
// The same over nch row chunks (part: nch x t1 x t2 doubles).
hipError_t launch_gram_n(int n, int t1, int t2, const double* A, const double* B, int nch, double* part,
                         double* out, hipStream_t stream);
// Row chunks of the C^T H C product a fused solve forms at admission: its partial sums take the
// place of four n-vectors of the solve, which are free until the set-up.
inline int mhc_chunks(int n, int s) {
    const long cap = s > 0 ? (4L * n) / ((long)s * s) : 1;
    const int g = gram_chunks(n);
    return cap < 1 ? 1 : (cap < g ? (int)cap : g);
}
hipError_t launch_gemm_tall(int n, int t, int k, const double* A, const double* X, int ldx, double* Out,
                            hipStream_t stream);
hipError_t launch_chol_drop(int t, const double* Gm, double tol, double* R, int* kept, int* tk, double* Xinv,
                            int ldx, hipStream_t stream);
size_t gsvd_scratch_doubles(int t, int p);
// size 0 / 1 / 2: the s largest / smallest / both ends of the generalized singular values
// (sizes 1 and 2 only with p >= t, checked by the caller).
hipError_t launch_gsvd_select(int t, int p, int s, int size, const double* M, const double* G, double* sc,
                              double* Xs, double* VHs, double* mu, int* info, hipStream_t stream);
// Ritz (kind 0) or harmonic Ritz (kind 1) selection, size 0 / 1 / 2 = S / L / M; scratch as
// gsvd_scratch_doubles.
hipError_t launch_ritz_select(int t, int s, int kind, int size, const double* M, const double* YtY, double* sc,
                              double* Xs, double* VHs, double* mu, int* info, hipStream_t stream);
// Inner refresh: C = op(A) B for small column-major matrices, and Y = M0 X with M0 the previous
// solve's projected Hessian in the basis [U, V] (blockdiag(sym(U^T C), T of the CG coefficients lz)).
hipError_t launch_small_gemm(int m, int k, int ncols, bool trans_a, const double* A, int lda, const double* B, int ldb,
                             double* C, int ldc, hipStream_t stream);
hipError_t launch_semiorth_prefix(int t0, int s0, const double* G, double tol, int* out, hipStream_t stream);
hipError_t launch_inner_y(int s0, int v, int t, const double* UtC, const double* lz, const double* X, double* Y,
                          hipStream_t stream);
// Left (side 1) or mixed (side 2) RGen vectors from the right ones in Xs.
hipError_t launch_rgen_side(int t, int side, const double* M, double* Xs, const int* info, hipStream_t stream);

}  // namespace bl
