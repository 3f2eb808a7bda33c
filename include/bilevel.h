/*
 * bilevel.h -- C ABI of libbilevel_hip.so: recycled-Krylov hypergradient solves on gfx950.
 *
 * Method: Ehrhardt, Gazzola, Scott, "Efficient gradient-based methods for bilevel
 * learning via recycling Krylov subspaces" (arXiv 2412.08264).
 *
 * Every call has C linkage, never throws and returns a bl_status.  All device arrays
 * are owned by the caller (allocated elsewhere, passed as raw device pointers); the
 * library never allocates device memory.  Scratch space is one caller-owned device
 * buffer of bl_workspace_bytes() bytes.  Hyperparameters theta and the hypergradient
 * live in host memory (p <= 512 doubles).
 *
 * Layout.  An image is h x w, row-major, n = h*w float64 values.  Tall matrices
 * (U, C, Z, V) are column-major with leading dimension n: column j starts at j*n.
 *
 * Streams.  A context is bound to one hipStream_t; all work is stream ordered.  Calls
 * that return host results (stats, gradients, status) synchronise that stream.
 *
 * Errors.  Argument and shape checks run on the host before any launch and return
 * BL_E_ARG / BL_E_SHAPE / BL_E_WORKSPACE.  Numerical outcomes are reported after the
 * work: BL_E_INDEFINITE when CG meets p^T H p <= 0, BL_E_NOT_CONVERGED at max_iter
 * (the iterate is still written), BL_E_NONFINITE on NaN/Inf.  HIP failures map to
 * BL_E_HIP (bl_last_error() gives the HIP message).
 */
#ifndef BILEVEL_H
#define BILEVEL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BL_OK = 0,
    BL_E_ARG = 1,            /* invalid argument (null pointer, bad enum, bad size)          */
    BL_E_SHAPE = 2,          /* inconsistent sizes (e.g. s > s_max, image too small)         */
    BL_E_WORKSPACE = 3,      /* workspace missing or smaller than bl_workspace_bytes()       */
    BL_E_NOT_CONVERGED = 4,  /* iteration limit reached                                      */
    BL_E_INDEFINITE = 5,     /* CG found p^T H p <= 0, or the projected matrix is not SPD    */
    BL_E_BREAKDOWN = 6,      /* a factorisation met a zero pivot                             */
    BL_E_RANK = 7,           /* refresh dropped dependent columns (non-fatal, s_cur reduced) */
    BL_E_NONFINITE = 8,      /* NaN or Inf met                                               */
    BL_E_HIP = 9             /* HIP runtime error                                            */
} bl_status;

typedef enum { BL_REG_TV = 0, BL_REG_FILTERS = 1 } bl_reg;
typedef enum { BL_PEN_LOG = 0, BL_PEN_QUAD = 1 } bl_penalty;     /* log(1+s^2) or s^2        */
typedef enum { BL_PREC_FP64 = 0, BL_PREC_MIXED = 1 } bl_prec;    /* mixed: FP32 HVP stencils  */
typedef enum { BL_STOP_RESID = 0, BL_STOP_HGERR = 1 } bl_stop;

/* Lower-level problem (Section 2.1 eq. bl2; Section 5 eq. ll2ex):
 *   TV:      Phi = ||A x - y||^2 + e^{t0} sum_i sqrt(|(D x)_i|^2 + e^{2 t1}),      p = 2
 *   filters: Phi = ||A x - y||^2 + eps/2 ||x||^2 + sum_j e^{w_j} sum_i phi((K_j x)_i),
 *            theta = [w_1, k_1 (f*f, row-major), ..., w_N, k_N],                   p = N(1+f^2)
 * A: same-size correlation with the normalised (2r+1)^2 Gaussian (zero outside the image);
 * D: forward differences, zero on the last column/row; K_j: same-size zero-padded
 * correlation with filter k_j.  Upper loss 1/2 ||x - x*||^2. */
typedef struct {
    int h, w;                /* image size, h, w >= 2                                         */
    int blur_radius;         /* r in [0, 8]                                                   */
    double blur_sigma;       /* > 0                                                           */
    int reg;                 /* bl_reg                                                        */
    int n_filters;           /* filters: 1..8                                                 */
    int filter_size;         /* filters: odd, 1..7                                            */
    double eps;              /* filters: coefficient of eps/2 ||x||^2                         */
    int penalty;             /* filters: bl_penalty                                           */
    int prec;                /* bl_prec                                                       */
} bl_problem;

/* Recycle state of one training sample (Section 2.2: U, C = H U with C^T C = I, and the
 * Krylov basis V of the last solve).  All pointers are caller-owned device memory.
 * U, C, Z: n x s_max; mu: s_max doubles; V: n x v_cap. */
typedef struct {
    double* U;
    double* C;
    double* Z;               /* Z = W V_H~ for the hypergradient-error estimate               */
    double* mu;              /* selected Ritz generalized singular values (0 for fill slots) */
    double* V;               /* first v_cap normalised CG residuals of the last solve         */
    int s_max, s_cur;        /* capacity / valid columns of U, C, Z, mu (s_cur = 0: none)     */
    int v_cap, v_cur;        /* capacity / valid columns of V                                 */
    double* lz;              /* 2 v_cap doubles or NULL: CG coefficients alpha_j (at 2j) and  */
                             /* rho_j = r_j.r_j (at 2j+1) of the stored residuals, written by */
                             /* CG solves with store_basis; read by the inner refresh          */
    int v_lz;                /* leading columns of V the coefficients describe (0: none)      */
} bl_recycle;

typedef struct {
    int stop;                /* bl_stop                                                       */
    double tol;              /* residual test ||r|| <= tol ||g||                              */
    double hg_tol;           /* error-estimate test ||mu . (Z^T r)|| <= hg_tol (absolute)     */
    int max_iter;
    int check_every;         /* the stop test runs at iterations j with j % check_every == 0; */
                             /* the estimate's Z^T r is formed on those iterations only      */
    int rr_every;            /* residual replacement period in mixed precision (0 = off)     */
    int store_basis;         /* store normalised residuals into rs->V                         */
} bl_solve_opts;

/* Recycle-space selections (Table 2) on the projected matrices of the refresh, W orthonormal:
 *   RGEN_L_R / _L / _M: the s largest Ritz generalized singular values of (J W, W^T H W)
 *     (Section 3.2), right vectors W X, left vectors W V_H, or their sum (each left vector taken
 *     as v = W^T H W x / ||W^T H W x||, x unit; side M is x + v), with Z and mu for the
 *     error-estimate test;
 *   RITZ_S / _L / _M: Ritz vectors (eq. ritz-matrix-decomp) of the smallest, the largest, or
 *     ceil(s/2) smallest and floor(s/2) largest Ritz values;
 *   HRITZ_S / _L / _M: harmonic Ritz vectors (eq. harmonic-ritz) chosen likewise by the harmonic
 *     Ritz values.
 *   RGEN_S_* / RGEN_M_*: the s smallest, or ceil(s/2) smallest and floor(s/2) largest, Ritz
 *     generalized singular values, sides as above; only where p >= t (J W of full column rank,
 *     so that no generalized singular value is zero), else BL_E_ARG.
 * Ritz and harmonic Ritz selections need no J and write mu = 0 and Z = 0: the error-estimate
 * test is then undefined (its estimate is 0), so solves after them use the residual test. */
typedef enum {
    BL_SEL_RGEN_L_R = 0, BL_SEL_RGEN_L_L = 1, BL_SEL_RGEN_L_M = 2,
    BL_SEL_RITZ_S = 3, BL_SEL_RITZ_L = 4, BL_SEL_RITZ_M = 5,
    BL_SEL_HRITZ_S = 6, BL_SEL_HRITZ_L = 7, BL_SEL_HRITZ_M = 8,
    BL_SEL_RGEN_S_R = 9, BL_SEL_RGEN_S_L = 10, BL_SEL_RGEN_S_M = 11,
    BL_SEL_RGEN_M_R = 12, BL_SEL_RGEN_M_L = 13, BL_SEL_RGEN_M_M = 14
} bl_select;

typedef struct {
    int s;                   /* requested recycle dimension (<= rs->s_max)                    */
    double rank_tol;         /* relative column-norm drop threshold for orthonormalising W   */
    int select;              /* bl_select (0: RGen-L(R))                                       */
    int inner;               /* 0: outer variant (eq. subtle-new), 1: inner (eq. subtle-old)  */
} bl_recycle_opts;

typedef struct {
    int iters;
    int status;              /* bl_status of the solve                                        */
    int t;                   /* refresh: columns of W kept; solve: unused                     */
    int s_cur;               /* refresh: recycle columns produced                             */
    double res_norm;         /* final recursive residual norm                                 */
    double res0_norm;        /* residual norm after the recycle-space projection             */
    double g_norm;
    double est;              /* estimate at the last tested iteration (NaN if unavailable)    */
    double ms[4];            /* wall-clock phases (ms), filled when timing is enabled         */
} bl_stats;

typedef struct bl_ctx bl_ctx;

/* Context bound to a HIP stream (hipStream_t passed as void*; NULL = default stream). */
bl_status bl_create(bl_ctx** ctx, void* hip_stream);
bl_status bl_destroy(bl_ctx* ctx);
const char* bl_status_string(int status);
const char* bl_last_error(const bl_ctx* ctx);
int bl_num_params(const bl_problem* P);
/* Device workspace for any call on problems of this shape with recycle capacity s_max and
 * stored-basis capacity v_cap (t_max = s_max + v_cap columns of refresh scratch). */
size_t bl_workspace_bytes(const bl_problem* P, int s_max, int v_cap);

/* Recycle storage of one training sample (the U, C = H U of Section 2.2.2 with Z, mu and the
 * stored basis V of Section 3.1) as one caller-owned device buffer: bl_recycle_bytes gives its
 * size for capacities s_max (0..64) and v_cap (s_max + v_cap <= 256), at least 256 bytes, and 0
 * for an invalid shape;
 * bl_recycle_init carves base (256-byte aligned, at least that many bytes) into U, C, Z
 * (n x s_max each), mu (s_max doubles), V (n x v_cap) and lz (2 v_cap doubles; V and lz NULL
 * when v_cap = 0), in that order, each array starting on a 256-byte boundary, and sets
 * s_cur = v_cur = v_lz = 0.  Host-only: no device
 * access, the buffer's contents are not touched.  BL_E_ARG (null pointer), BL_E_SHAPE (bad
 * capacities or problem), BL_E_WORKSPACE (buffer too small or misaligned). */
size_t bl_recycle_bytes(const bl_problem* P, int s_max, int v_cap);
bl_status bl_recycle_init(const bl_problem* P, int s_max, int v_cap, void* base, size_t bytes, bl_recycle* rs);

/* Measurement y = A x + noise * e (problem data; not on the timed path). */
bl_status bl_forward(bl_ctx* ctx, const bl_problem* P, const double* x, const double* e, double noise,
                     double* y, void* ws, size_t ws_bytes);

/* Lower-level solve (eq. ll2): L-BFGS with history m (Section 5), Armijo backtracking,
 * stop at ||grad Phi|| <= gtol.  x_inout: start point in, minimiser out.  out: iters in
 * stats->iters, final gradient norm in stats->res_norm. */
bl_status bl_lower_solve(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* y,
                         double* x_inout, double gtol, int max_iter, int m, void* ws, size_t ws_bytes,
                         bl_stats* out);

/* Ritz-GSV refresh, outer variant (Section 3.2, eqs. gsvd, partial-gsvd, RGen-L(R)): builds
 * W = orth([U, V]) from rs, projects M = W^T H W, G = J W at (xhat, theta), takes the s
 * largest Ritz generalized singular values (null(G) filled by Ritz-S when rank G < s),
 * and writes U, C = H U (C^T C = I), Z, mu and s_cur into rs.  rs->s_cur = 0 and
 * rs->v_cur = 0 leave rs empty.  opts->select picks another rule of bl_select on the same
 * projected matrices (Ritz and harmonic Ritz selections also work for indefinite H, where
 * RGen's Cholesky of W^T H W fails with BL_E_INDEFINITE). */
bl_status bl_recycle_update(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                            bl_recycle* rs, const bl_recycle_opts* opts, void* ws, size_t ws_bytes,
                            bl_stats* out);

/* Hessian solve H w = g (eq. hess_sys) by recycled CG (Galerkin counterpart of RMINRES,
 * Section 2.2.2) with the residual or hypergradient-error test (Section 4, eq.
 * hg-err-stop-lowrank).  rs == NULL or rs->s_cur == 0: plain CG.  w_inout: warm start in,
 * solution out.  With opts->store_basis the normalised residuals go to rs->V and the CG
 * coefficients (alpha_j, r_j.r_j) of those iterations to rs->lz (rs->v_lz of them), which the
 * inner refresh reads.  FP64 problems run one fused launch per iteration (Chronopoulos and
 * Gear's single-reduction form: beta from the recurrence of the projected residual's norm,
 * alpha and every test from the explicitly reduced r.r); mixed-precision problems run an apply
 * and an update launch per iteration with FP64 residual replacement every opts->rr_every. */
bl_status bl_hessian_solve(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                           const double* g, double* w_inout, bl_recycle* rs, const bl_solve_opts* opts,
                           void* ws, size_t ws_bytes, bl_stats* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): bl_hessian_solve with the same arguments and results
 * minus the workspace.  Its scratch is a static device array of BL_NOALLOC_SCRATCH_BYTES bytes,
 * one per GPU, held from the library's first use on that GPU until the process ends (its address
 * is looked up once per device, on the calling thread's current device, which must be the
 * device of the context's stream).  A problem whose solve needs more scratch (TV up to about
 * 1024 x 1024 fits; filters up to about 512 x 512) is refused with BL_E_WORKSPACE before any
 * launch.  The call allocates nothing and launches directly (no graph capture).  All calls on
 * one GPU share its array: calls that overlap on one GPU (other streams, other threads) race and
 * must be serialised by the caller; a call leaves the array holding its own data, and every
 * value a solve reads from it is written by that solve first. */
#define BL_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
bl_status bl_hessian_solve_noalloc(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                                   const double* g, double* w_inout, bl_recycle* rs, const bl_solve_opts* opts,
                                   bl_stats* out);

/* Hessian solve H w = g by RMINRES (Section 2.2.2, Algorithm 3): the correction V_k y + U z
 * minimising ||g - H w|| over w0 + range(U) + K_k((I - C C^T) H, r0) (eq. coupled), with the
 * Lanczos vectors kept orthogonal to C = H U (eq. arnoldi_aug_matrix).  H may be indefinite.
 * Same arguments as bl_hessian_solve; differences:
 *   * FP64 only (a problem with prec = BL_PREC_MIXED is refused with BL_E_ARG; rr_every is
 *     ignored);
 *   * the residual test is |zeta_j| <= tol ||g||, |zeta_j| the residual norm that MINRES's QR
 *     factors give; the error-estimate test forms Z^T r_j from the explicit residual kept by
 *     the recurrence of Appendix A's residual (in a one-vector form); both run on iterates j
 *     with j % check_every == 0;
 *   * with store_basis the normalised Lanczos vectors v_1, v_2, ... go to rs->V
 *     (rs->v_cur = min(iters, v_cap));
 *   * BL_E_BREAKDOWN if a Givens rotation meets a zero column (the iterate of the last test is
 *     kept); BL_E_INDEFINITE is never returned.
 * stats: res_norm = |zeta| at the returned iterate, res0_norm = ||r0|| after the projection.
 * Tiles of 32 x 8 pixels; no graph replay: two launches per step from the host, with a poll of
 * the stop flag every 8 steps (double-buffered: the device runs the next 8 steps while the host
 * reads the flag of the previous ones). */
bl_status bl_hessian_solve_rminres(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                                   const double* g, double* w_inout, bl_recycle* rs, const bl_solve_opts* opts,
                                   void* ws, size_t ws_bytes, bl_stats* out);

/* Hessian solve H w = g by deflated CG (Saad, Yeung, Erhel and Guyomarc'h 2000), the other
 * reading of a recycled CG beside bl_hessian_solve's Galerkin form (Section 2.2.2 defines only
 * RMINRES), with U and C = H U of the recycle state as the deflation space: with
 * E = U^T C (= U^T H U), the set-up w = w0 + U E^{-1} U^T r0, r0 -= C E^{-1} U^T r0 makes
 * U^T r = 0, and each direction p = r + beta p_prev - U E^{-1} C^T r is H-conjugate to U.  Same
 * arguments, stop tests and statistics as bl_hessian_solve; differences:
 *   * FP64 only (prec = BL_PREC_MIXED is refused with BL_E_ARG; rr_every is ignored);
 *   * BL_E_INDEFINITE before any iteration if U^T C is not positive definite;
 *   * with store_basis the normalised residuals go to rs->V (rs->v_lz = 0: no CG coefficients
 *     of the Galerkin form, so the inner refresh refuses this basis);
 *   * tiles of 32 x 8 pixels, no graph replay: two launches per step from the host with a
 *     double-buffered poll of the stop flag every 8 steps. */
bl_status bl_hessian_solve_deflated(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                                    const double* g, double* w_inout, bl_recycle* rs, const bl_solve_opts* opts,
                                    void* ws, size_t ws_bytes, bl_stats* out);

/* Hypergradient J w = -(D_theta grad_x Phi)^T w (eq. hypgrad) into grad_host (p doubles).
 * Filters: each filter's tap block is projected onto zero mean when project_zero_mean. */
bl_status bl_hypergradient(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                           const double* w, double* grad_host, int project_zero_mean, void* ws, size_t ws_bytes);

/* Matrix-free Hessian-vector products out[:, j] = H v[:, j], j < ncols (columns ld = n),
 * in the problem's precision (FP32 stencil arithmetic in mixed mode, FP64 output), on tiles
 * of bl_tile_rows(P) rows. */
bl_status bl_hvp(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat,
                 const double* v, double* out, int ncols, void* ws, size_t ws_bytes);

/* Gradient of the lower-level objective and its value (value to *phi_host if non-NULL). */
bl_status bl_lower_grad(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* y,
                        const double* x, double* grad, double* phi_host, void* ws, size_t ws_bytes);

/* Graph replay of the Krylov iterations, 1 (default) / 0.  The iterations of a solve run in
 * chunks of 16 for a lone solve and 8 for a batch (the step launches, scheduled residual
 * replacements, the header snapshot written into pinned host memory).  A chunk whose launch sequence has occurred before since the set of running
 * solves last changed is captured once (on a private stream of the context) and replayed with
 * hipGraphLaunch on the context's stream; the kernels take their iteration index from a device
 * counter, so the replays need no new arguments.  Results are bitwise those of direct launches.
 * If a capture fails, the batch falls back to direct launches. */
bl_status bl_set_graphs(bl_ctx* ctx, int enable);
/* Chunks captured into graphs and chunk replays on this context since it was created. */
bl_status bl_graph_counts(const bl_ctx* ctx, long long* captured, long long* replayed);

/* Time the phases of subsequent calls with HIP events (stats->ms), 0/1.  With 2, also record
 * HIP events around the step launches (FP64: the fused step; mixed: the apply) and the update
 * launch of every eighth Krylov step (see bl_kernel_times; with graph replay on, every step of
 * every eighth chunk, which then runs directly); sampling keeps the events' own cost out of the
 * run they measure. */
bl_status bl_set_timing(bl_ctx* ctx, int enable);

/* Per-kernel durations accumulated over solves since the last reset, iterations that ran
 * only, over the sampled steps: out4[0] = total ms of the step launches (the fused FP64 step,
 * or the mixed-precision apply: H p fused with p.q and C^T q), out4[1] = their count,
 * out4[2] / out4[3] = the same for the mixed-precision update launch (FP64 solves launch no
 * update: their pair of events brackets nothing and measures the events' own cost).  reset != 0
 * clears the totals after reading. */
bl_status bl_kernel_times(bl_ctx* ctx, double* out4, int reset);

/* ------------------------------------------------------------------------------------------
 * Batched and served Hessian solves.  An engine runs up to `cap` (<= 64) recycled-CG solves
 * side by side: each iteration is one launch per group of solves with the same operator class
 * (problems equal in every bl_problem field but h, w), tile height (bl_tile_rows) and recycling
 * (s_cur > 0 or not; at most 16 groups at a time): the fused step for FP64 groups, the apply
 * kernel (H p with p.q and C^T q) for mixed-precision groups, followed by one launch of the
 * update kernel over the running mixed-precision solves, whatever their sizes, recycle
 * dimensions and iteration indices.  Every solve reduces only its own records in a fixed
 * order, so its iterates, iteration count and status are bitwise those of the same solve
 * run alone (bl_hessian_solve, which is a one-solve engine) with the same tile height.  Solves are admitted and retired
 * between steps (continuous batching).  The engine's device memory is one caller-owned
 * workspace: fixed per-slot descriptors plus an arena from which each admitted solve takes
 * bl_engine_slot_bytes() and to which retirement returns it.  The engine holds pinned host
 * buffers of its own (released by bl_engine_destroy) and is used from one host thread.
 * ------------------------------------------------------------------------------------------ */
typedef struct bl_engine bl_engine;

/* Arena bytes one solve of problem P with s recycle columns (rs->s_cur) occupies. */
size_t bl_engine_slot_bytes(const bl_problem* P, int s);
/* Workspace for an engine of `cap` slots (1..64) with an arena of arena_bytes. */
size_t bl_engine_workspace_bytes(int cap, size_t arena_bytes);
/* Engine over the workspace ws (256-byte aligned); the arena is whatever ws_bytes leaves
 * after the fixed part. */
bl_status bl_engine_create(bl_ctx* ctx, int cap, void* ws, size_t ws_bytes, bl_engine** engine);
bl_status bl_engine_destroy(bl_engine* engine);
/* Admit the solve H(theta, xhat) w = g with recycle state rs (NULL or s_cur = 0: plain CG)
 * and options opts; same arguments and meaning as bl_hessian_solve.  theta and opts are
 * read during the call; xhat, g, w, rs and its arrays must stay valid until retirement.
 * Set-up work (FP64 residual, projection onto C) is enqueued at once.  Returns
 * BL_E_WORKSPACE (nothing enqueued) when no slot or no arena block of
 * bl_engine_slot_bytes() is free: retire a completed solve and try again; BL_E_ARG when the
 * problem would open a 17th (operator class, tile height, recycling) group among the admitted
 * solves. */
bl_status bl_engine_admit(bl_engine* engine, const bl_problem* P, const double* theta_host, const double* xhat,
                          const double* g, double* w_inout, bl_recycle* rs, const bl_solve_opts* opts, int* slot);
/* Advance all running solves by at most max_iters iterations; with return_on_done, return
 * as soon as one or more solves have completed.  The slots of completed solves go to
 * done[0 .. *n_done - 1] (done holds cap ints); their w is final when the call returns. */
bl_status bl_engine_step(bl_engine* engine, int max_iters, int return_on_done, int* done, int* n_done);
/* Statistics of a completed solve, and the slot and its arena block freed.  Returns the
 * solve's status (as bl_hessian_solve would); with store_basis rs->v_cur is set. */
bl_status bl_engine_retire(bl_engine* engine, int slot, bl_stats* out);
/* Running solves, free slots, free arena bytes and the largest free arena block. */
bl_status bl_engine_query(const bl_engine* engine, int* running, int* free_slots, size_t* free_bytes,
                          size_t* largest_free);

/* Workspace of bl_hessian_solve_batched for nprob problems P[k] with s[k] recycle columns
 * (s = NULL: none). */
size_t bl_batched_workspace_bytes(int nprob, const bl_problem* P, const int* s);
/* nprob independent solves (P[k], theta[k], xhat[k], g[k], w[k], rs[k]; rs = NULL: plain CG
 * for all; at most 16 (operator class, tile height, recycling) groups) with shared options,
 * advanced together (at most 64 at a time; later ones are admitted as earlier ones finish).
 * out[k] gets the statistics of solve k.  Returns BL_OK, or the first non-OK status of a
 * solve. */
bl_status bl_hessian_solve_batched(bl_ctx* ctx, int nprob, const bl_problem* P, const double* const* theta_host,
                                   const double* const* xhat, const double* const* g, double* const* w_inout,
                                   bl_recycle* rs, const bl_solve_opts* opts, void* ws, size_t ws_bytes,
                                   bl_stats* out);

/* ------------------------------------------------------------------------------------------
 * Tile shapes.  The fused apply and residual kernels of the Hessian solves work on tiles of
 * 32 columns and 8, 16 or 32 rows: tall tiles reuse more of each staged value, short tiles
 * give small images more blocks.  The height a solve uses is looked up in a process-wide
 * table keyed by the operator class (regulariser, blur radius, filter count and size,
 * precision) and the size class floor(log2(h*w)); without an entry it is the tallest tile
 * that still gives the image at least 256 tiles (one per compute unit), else 8 rows.  A
 * solve keeps the height it was admitted with; the table is read under a lock.
 * ------------------------------------------------------------------------------------------ */

/* Set (rows = 8, 16 or 32) or clear (rows = 0) the table entry of P's class and size class.
 * BL_E_ARG for another value. */
bl_status bl_tile_rows_set(const bl_problem* P, int rows);
/* The tile height solves of P use now (table entry or default); 0 for an invalid problem. */
int bl_tile_rows(const bl_problem* P);
/* Scratch of bl_autotune for P with s (0..64) recycle columns; 0 for an invalid shape. */
size_t bl_autotune_workspace_bytes(const bl_problem* P, int s);
/* Tile-height autotuner with a persistent cache.
 *   cache_path != NULL and the file holds an entry for P's operator class and size class: the
 *     stored height goes into the table and *best_rows; nothing is timed, no device work,
 *     theta_host, xhat, iters and ws may be NULL / 0; us_per_iter (may be NULL) gets zeros.
 *   otherwise: times recycled-CG solves of P at (theta_host, xhat) with s recycle columns at
 *     each height (8, 16, 32 rows): one of 16 iterations and one of 16 + 16 max(1, iters / 16)
 *     (iters in 1..100000), whose difference is the cost of the extra iterations without the
 *     per-solve set-up; stores the fastest height in the table, returns it in *best_rows and
 *     the microseconds per iteration in us_per_iter[0..2]; with cache_path the entry is then
 *     added to (or replaced in) the file, which is rewritten whole through a temporary file
 *     next to it and a rename.  The recycle columns are zero (the arithmetic of plain CG with
 *     every projection still read) and the stop test is off, so each solve runs exactly its
 *     iteration count.  Scratch: the caller's
 *     ws of bl_autotune_workspace_bytes(P, s) bytes (256-byte aligned); synchronous on the
 *     context's stream.
 * Cache file: text, one entry per line "reg radius n_filters filter_size prec log2n rows us8
 * us16 us32", '#' lines are comments.  A file that exists but does not parse, or cannot be
 * written, gives BL_E_ARG (bl_last_error names the line) and is left unchanged. */
bl_status bl_autotune(bl_ctx* ctx, const bl_problem* P, const double* theta_host, const double* xhat, int s,
                      int iters, const char* cache_path, void* ws, size_t ws_bytes, int* best_rows,
                      double* us_per_iter);
/* Load every entry of a tile cache file written by bl_autotune into the table (host only, no
 * context, no device work); *entries (may be NULL) gets their number.  BL_E_ARG when the file
 * is missing or does not parse; then the table is unchanged. */
bl_status bl_tile_cache_load(const char* cache_path, int* entries);

#ifdef __cplusplus
}
#endif
#endif /* BILEVEL_H */
