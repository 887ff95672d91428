/*
 * nrs.h -- C ABI of libnrs: the nearest-neighbour regularized stokeslet
 * (NEAREST) hot path on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Gallagher & Smith, "Passively parallel regularized
 * stokeslets" (arXiv:2001.06468); section and equation numbers below refer to
 * that paper.  Per time step the paper's cost is (1) the stokeslet matrix
 * multiplied by the nearest-neighbour matrix, (2) the full matrix with the
 * rigid-body unknowns, (3) the dense solve (Sec. 4).  This library performs
 * all three on the GPU, plus the geometry and nearest-neighbour map that feed
 * them and the time-stepping and warm-started iterative forms built on them.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is DEVICE memory unless stated otherwise, owned by
 *    the caller, and must stay valid until the work enqueued on the
 *    context's stream has completed.  The library never frees caller memory
 *    and keeps no pointer after a call returns.
 *  - Point coordinates are structure-of-arrays: x[c*N + i] is component c
 *    (0,1,2) of point i.  Body states are Y[b*12 + 0..2] = origin x0 and
 *    Y[b*12 + 3..11] = body frame B, row-major, column i = body axis i.
 *  - Unknowns are ordered component-major: sol[j*N + m] = f_j at force point m
 *    (j = 0,1,2), then sol[3N + 6b + 0..5] = (U, Omega) of free body b.
 *    n = 3N + 6M.  Matrices are column-major with leading dimension lda >= n.
 *  - f is the force density exerted ON THE FLUID by the body (the + sign of
 *    the nearest-neighbour form, Sec. 3 eq. 23), per unit quadrature weight;
 *    W_n = sum of w_q over the quadrature points whose nearest force point
 *    is n; the patch force is W_n f_n.
 *  - All work is enqueued on the context's stream (stream-ordered, no host
 *    synchronisation) unless the description says the call synchronises.
 *  - Errors: every function returns nrs_status.  Argument errors are detected
 *    on the host before anything is enqueued.  Numerical failures detected on
 *    the device are reported through nrs_info.  nrs_last_error() gives a
 *    human-readable detail of the last failure on a context.  No C++
 *    exception crosses this interface.
 */
#ifndef NRS_H
#define NRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nrs_status;
#define NRS_OK                0
#define NRS_E_ARG            -1  /* invalid argument (sizes, NULL, lda, precision)      */
#define NRS_E_HIP            -2  /* HIP runtime error                                    */
#define NRS_E_WORKSPACE      -3  /* workspace missing or smaller than nrs_workspace_size */
#define NRS_E_SINGULAR       -4  /* exact zero pivot in the FP64 factorisation           */
#define NRS_E_NOT_CONVERGED  -5  /* refinement / GMRES missed its tolerance              */
#define NRS_E_NONFINITE      -6  /* NaN or Inf in an input or in the solution            */
#define NRS_E_UNSUPPORTED    -7  /* size or option outside what this build implements    */

/* Solution methods (nrs_options.method). */
#define NRS_FP64_LU        0  /* FP64 assembly, FP64 LU with partial pivoting           */
#define NRS_FP32_IR        1  /* FP32 assembly + FP32 block-pivoted LU, FP64 refinement */
#define NRS_FP32_GEPP_IR   2  /* as NRS_FP32_IR but with full partial pivoting          */
#define NRS_GMRES          3  /* FP64 GMRES(m) on the stored FP64 matrix, from x_init   */
#define NRS_FP32_GMRES_IR  4  /* FP32 assembly + FP32 tile LU (static block pivoting),
                                 then flexible GMRES(m) in FP64 on the matrix-free
                                 operator with the LU as right preconditioner        */
#define NRS_BF16_GMRES_IR  5  /* as NRS_FP32_GMRES_IR, but the tile LU's trailing
                                 updates take BF16 copies of the finished tiles on
                                 the matrix cores (FP32 accumulation, FP32 pivots and
                                 tile solves); the workspace also holds those copies */
#define NRS_GMRES_BLOCK    6  /* flexible GMRES(m) in FP64 on the matrix-free operator,
                                 from x_init, with a block-diagonal right
                                 preconditioner: one dense block per free body
                                 (its force and (U, Omega) unknowns; rows of
                                 fixed points unpreconditioned), the exact
                                 inverse of the body's diagonal block
                                 (NRS_PRECOND_EXACT) or a learned prediction of
                                 it (NRS_PRECOND_MODEL, nrs_block_model_fit)    */

/* Body blocks of NRS_GMRES_BLOCK (nrs_options.precond). */
#define NRS_PRECOND_EXACT  0  /* FP64 assembly, then the inverse of every body's
                                 diagonal block (Gauss-Jordan, one workgroup
                                 per body)                                     */
#define NRS_PRECOND_MODEL  1  /* no assembly: each body's block inverse is
                                 R_b K(psi_b) R_b^T from the Fourier model K of
                                 nrs_block_model_fit at the body's beat phase  */
#define NRS_BLOCK_MAX_HARMONICS 16

typedef struct nrs_ctx nrs_ctx;

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t, borrowed; NULL = the null stream).  The context's own device
 * memory is 64 bytes of status words (allocated on first use by the network
 * calls); every larger buffer is a caller workspace.
 * Returns NRS_E_HIP if the device cannot be selected. */
nrs_status  nrs_create(nrs_ctx** out, int device, void* stream);
nrs_status  nrs_destroy(nrs_ctx* ctx);
nrs_status  nrs_set_stream(nrs_ctx* ctx, void* stream);
const char* nrs_status_string(nrs_status s);
const char* nrs_last_error(const nrs_ctx* ctx);
/* Version string "nrs <major>.<minor> gfx950". */
const char* nrs_version(void);

/* ------------------------------------------------------------------------ */
/* Scene description and geometry at time t (Sec. 4: the state Y = [X0; B]
 * of the swimmers and their body-frame shapes).                             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t N, Q;          /* force (coarse) points, quadrature (fine) points      */
  int32_t M, P;          /* free bodies, travelling-wave parts                   */
  const double*  xi;     /* [3][N] body-frame offset, or lab position if body<0 */
  const int32_t* body;   /* [N] -1 = fixed point, else 0..M-1                    */
  const int32_t* part;   /* [N] wave part index or -1                            */
  const double*  s;      /* [N] arc parameter of wave points                     */
  const double*  ufix;   /* [3][N] prescribed lab velocity of fixed points       */
  const double*  Xi;     /* [3][Q] as xi, for quadrature points                  */
  const int32_t* bodyX;  /* [Q]                                                  */
  const int32_t* partX;  /* [Q]                                                  */
  const double*  sX;     /* [Q]                                                  */
  const double*  w0;     /* [Q] base quadrature weight                           */
  const double*  wave;   /* [P][6] beta, A0, A1, k, omega, phi                   */
} nrs_scene;

/* Geometry of all points at time t for body states Y [M][12]:
 *   wave displacement d(s,t) = (beta s, (A0 + A1 s) sin(k s - omega t + phi), 0)
 *   free-body point: x = x0 + B (xi + d),  u = B dd/dt  (deformation velocity)
 *   fixed point:     x = xi,               u = ufix
 *   quadrature weight w = w0 * |d(xi + d)/ds| on wave parts, w0 elsewhere.
 * Outputs x [3][N], X [3][Q], w [Q], u [3][N] (any may be NULL to skip). */
nrs_status nrs_geometry(nrs_ctx* ctx, const nrs_scene* sc, double t, const double* Y,
                        double* x, double* X, double* w, double* u);

/* ------------------------------------------------------------------------ */
/* Nearest-neighbour map (Sec. 3 eq. 20): nu[q] = argmin_n |x_n - X_q| over
 * the force points n of q's group (force points of group g are
 * group_off[g] .. group_off[g+1]-1; group_off is a HOST array of G+1
 * entries).  Squared distances are (dx*dx + dy*dy) + dz*dz in FP64 without
 * fused multiply-add; the lowest index wins a tie, so the result is
 * bit-for-bit the brute-force map.  nu_out: [Q] int32.
 * NRS_E_ARG if a group with quadrature points has no force points.          */
/* ------------------------------------------------------------------------ */
nrs_status nrs_nearest(nrs_ctx* ctx, int64_t N, const double* x, int32_t G,
                       const int32_t* group_off_host, int64_t Q, const double* X,
                       const int32_t* groupX, int32_t* nu_out);

/* ------------------------------------------------------------------------ */
/* One resistance / swimming problem at fixed geometry.                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t N, Q;
  int32_t M;
  const double*  x;      /* [3][N] force points                                  */
  const double*  X;      /* [3][Q] quadrature points                             */
  const double*  w;      /* [Q] quadrature weights (NULL = all 1, the paper's
                            unweighted sum of Sec. 3 eq. 23)                     */
  const int32_t* nu;     /* [Q] nearest force point of each quadrature point     */
  const int32_t* body;   /* [N] -1 = prescribed velocity, else free body 0..M-1  */
  const double*  Y;      /* [M][12] body states; x0 = moment centre (NULL iff M=0)*/
  double eps, mu;        /* regularisation parameter, viscosity                  */
} nrs_problem;

typedef struct {
  int32_t method;        /* NRS_FP64_LU, NRS_FP32_IR, NRS_FP32_GEPP_IR, NRS_GMRES,
                            NRS_FP32_GMRES_IR, NRS_BF16_GMRES_IR                 */
  int32_t max_refine;    /* refinement sweeps (IR) before falling back; <=0: 4   */
  double  tol;           /* IR: stop when |d|_inf <= tol |x|_inf, <=0: 1e-9.
                            GMRES: relative residual |b - A x|_2 <= tol |b|_2,
                            <=0: 1e-11 (NRS_GMRES), 1e-12 (the GMRES-IR forms) */
  int32_t gmres_restart; /* GMRES(m) restart length 1..63, <=0: 50 (NRS_GMRES),
                            60 (the GMRES-IR forms)                             */
  int32_t gmres_max_iter;/* total GMRES iterations before LU fallback, <=0: 1000
                            (NRS_GMRES), 300 (the GMRES-IR forms)              */
  int32_t no_fallback;   /* 1 = report failure instead of falling back to FP64 LU */
  const double* x_init;  /* [n] device initial guess for NRS_GMRES (NULL = zero); may
                            equal sol (start from sol's current content)       */
  /* Warm start of the GMRES solves inside nrs_rk4_step:
     NRS_WARM_NONE, NRS_WARM_PREVIOUS (the previous solve of the same time
     stepping workspace on this context) or NRS_WARM_MODEL (the network of the
     learned warm start, below). */
  int32_t warm_start;
  const float* model_theta;     /* device [nrs_mlp_param_count()] (NRS_WARM_MODEL)  */
  double model_scales[3];       /* force, U and Omega scales of the model outputs   */
  const int32_t* body_off;      /* device [M+1] from nrs_mlp_body_offsets           */
  /* NRS_GMRES with x_init and free bodies: before iterating, project the
     initial forces onto each body's force and torque balance (the constraint
     rows hold exactly) and refit each body's (U, Omega) to the velocity
     residual by least squares.  Always applied to NRS_WARM_MODEL starts. */
  int32_t x_init_complete;
  /* nrs_solve_batched, asynchronous form only (infos = NULL) on a non-default
     stream: capture every launch and copy of the batch into a HIP graph on
     the first call and replay it on later calls with the same arguments
     (same sizes, pointers, eps, mu, workspace and refinement settings; the
     array contents may change).  Up to 8 graphs are kept per context. */
  int32_t graph;
  /* nrs_rk4_step / nrs_rk4_step_tracers with NRS_FP32_IR, non-zero: only the
     first stage of a step assembles and factors; stages 2-4 refine against
     those FP32 factors (x0 from them, then FP64 matrix-free residuals and
     correction sweeps, at most max_refine sweeps, <= 0: 12), since the
     stage matrices differ from the first one by the motion over dt/2 or dt.
     The stopping rule and the accuracy are those of NRS_FP32_IR; a stage
     that does not converge sends the step to the FP64 fallback like any
     failed stage.  Ignored by every other call. */
  int32_t reuse_stage_factors;
  /* Non-zero: the FP32 tile-LU forms (NRS_FP32_IR, NRS_FP32_GMRES_IR,
     NRS_BF16_GMRES_IR) of nrs_solve, nrs_rk4_step and nrs_dopri5_integrate
     factor the equilibrated matrix D_r A D_c: D_r, D_c powers of two, row
     scaling r_i = max_j |a_ij|, dr_i = 2^-floor(log2 r_i), then column
     scaling of the row-scaled matrix likewise, so every row's and column's
     largest entry has magnitude in [1, 2) and the scaling adds no rounding.
     Refinement keeps the unscaled FP64 residual: correction = D_c (LU)^-1
     D_r r.  Zero (default): factor A itself.  (NRS_FP32_GEPP_IR, whose
     partial pivoting needs no scaling, and nrs_solve_batched never scale.) */
  int32_t equilibrate;
  /* NRS_GMRES_BLOCK: which body blocks precondition the GMRES (NRS_PRECOND_
     EXACT or NRS_PRECOND_MODEL).  With NRS_PRECOND_MODEL: precond_model is
     the device model [2H+1][nb][nb] of nrs_block_model_fit (H =
     precond_harmonics, nb = precond_nb = 3 N_b + 6 for bodies of N_b force
     points), precond_phase the device beat phases psi_b = omega t - phi [M]
     of the bodies (nrs_solve only; the time stepping entry points take each
     body's phase from its first wave point of the scene at the stage time).
     Every free body's points must form one contiguous run, bodies in order;
     a body whose block order exceeds nrs_block_limit() or differs from
     precond_nb is left unpreconditioned (nrs_solve with info then returns
     NRS_E_UNSUPPORTED after writing the solution).  x_init and tol,
     gmres_restart, gmres_max_iter as for the GMRES-IR forms (defaults
     1e-12, 60, 300); warm_start (NRS_WARM_PREVIOUS, NRS_WARM_MODEL) applies
     inside the time stepping entry points as for NRS_GMRES. */
  int32_t precond;
  int32_t precond_harmonics;
  int32_t precond_nb;
  const double* precond_model;
  const double* precond_phase;
  /* nrs_rk4_step / nrs_rk4_step_tracers with NRS_FP32_IR or NRS_FP32_GEPP_IR
     (stages that factor): correction sweeps queued per stage before the
     step's one host check.  0 (default): adaptive, the largest number of
     sweeps a stage needed in the previous step on the same workspace plus
     one (max_refine while unknown); k > 0: k.  Never more than max_refine
     (<= 0: 4).  A step whose stages miss the tolerance with fewer than
     max_refine sweeps queued is redone with max_refine before the FP64
     fallback, so the result is that of max_refine queued sweeps; sweeps
     queued after convergence skip their work but still cost their launches.
     Ignored by every other call and with reuse_stage_factors. */
  int32_t ir_queue;
} nrs_options;

typedef struct {
  int32_t method_used;   /* method whose result is in sol                        */
  int32_t fell_back;     /* 1 if the requested method failed and FP64 LU ran     */
  int32_t iterations;    /* refinement sweeps or GMRES iterations performed      */
  int32_t singular;      /* 1 if a zero pivot was met                            */
  double  backward_error;/* |b - A x|_inf / (|A|_inf |x|_inf + |b|_inf), FP64 A  */
  double  correction;    /* last |d|_inf / |x|_inf of the refinement             */
} nrs_info;
/* backward_error: the synchronous forms (info / infos != NULL) evaluate it
 * at the returned sol.  The asynchronous forms (nrs_query_info, the RK4
 * stages) report the last residual the refinement took, i.e. at the iterate
 * before its last correction; after that correction the error is about
 * correction times smaller. */

/* Bytes of device workspace that nrs_solve / nrs_assemble / nrs_apply need
 * for this size and method. */
nrs_status nrs_workspace_size(nrs_ctx* ctx, int64_t N, int64_t Q, int32_t M,
                              int32_t method, size_t* bytes);

/* Assemble the full matrix A (order n = 3N + 6M, column-major, leading
 * dimension lda) in FP64 (precision = 64) or FP32 (precision = 32):
 *   A_s[jN+m, kN+n] = (8 pi mu)^-1 sum_{q: nu(q)=n} w_q S^eps_jk(x_m - X_q)
 * (Sec. 3 eqs. 18 and 21-23, the stokeslet matrix times the nearest-neighbour
 * matrix, fused so the 3N x 3Q matrix never exists), then the rigid-body
 * blocks of the swimming problem (Sec. 2 and Sec. 4): columns -1 (U) and
 * -(e_i x r_m) (Omega), force rows W_m, moment rows W_m (r_m x .), zero
 * 6M x 6M block, r_m = x_m - x0.  A: device, n x lda elements of the chosen
 * precision.  Writes every entry of the leading n x n block.  Quadrature
 * points whose nu is outside [0, N) contribute nothing (no error is
 * reported; nrs_solve reports them as NRS_E_ARG). */
nrs_status nrs_assemble(nrs_ctx* ctx, const nrs_problem* pb, int32_t precision,
                        void* A, int64_t lda, void* ws, size_t ws_bytes);

/* Matrix-free FP64 product y = A v with A as in nrs_assemble (the NEAREST
 * operator of Sec. 3 eq. 23 evaluated on the fly plus the rigid-body rows).
 * v, y: [n] device.  Out-of-range nu as in nrs_assemble. */
nrs_status nrs_apply(nrs_ctx* ctx, const nrs_problem* pb, const double* v, double* y,
                     void* ws, size_t ws_bytes);

/* Solve A sol = b, b = [u_x; u_y; u_z; (F_ext, T_ext) per body], for the
 * force densities and rigid-body velocities (Sec. 4, step 3).
 * NRS_FP32_IR refines the FP32 solution with FP64 residuals; in the
 * synchronous form (info != NULL), if the refinement stalls (the static
 * block pivots can leave the FP32 factors too inexact for plain refinement
 * on large wall-bounded systems), it continues from its iterate with the
 * flexible GMRES of NRS_FP32_GMRES_IR on the same factors (relative residual
 * 1e-12) before any FP64 fallback; info->iterations then counts both.
 * The GMRES-IR forms synchronise with the host once every few GMRES steps
 * even in the asynchronous form.
 * u: [3][N] prescribed velocities; ftext: [M][6] external force and torque
 * (NULL = force- and torque-free); sol: [n] output.
 * With info == NULL the call is fully asynchronous; numerical status then
 * stays in the workspace and nrs_query_info() reads it.  With info != NULL
 * the call synchronises the stream, fills *info, and may run the FP64 LU
 * fallback.  Returns NRS_E_SINGULAR / NRS_E_NOT_CONVERGED in that case when
 * no method succeeded. */
nrs_status nrs_solve(nrs_ctx* ctx, const nrs_problem* pb, const double* u, const double* ftext,
                     const nrs_options* opt, void* ws, size_t ws_bytes, double* sol,
                     nrs_info* info);

/* Synchronise and read the numerical status of the last asynchronous solve
 * that used workspace ws. */
nrs_status nrs_query_info(nrs_ctx* ctx, void* ws, nrs_info* info);

/* Many independent problems of different orders solved together (the
 * resistance problems of Sec. 4 for several bodies / parameter values at
 * once), method NRS_FP32_IR only.  problems, u, ftext, sol and infos are
 * HOST arrays of B entries; the arrays they point to are on the device as
 * in nrs_solve (ftext may be NULL, or hold NULL entries).  The FP32
 * factorisations of all B systems run in one launch of the tile LU, and each
 * triangular sweep of the refinement in one launch over the batch; the
 * remaining per-system steps are spread over the context's stream and three
 * side streams the context owns (default priority), forked from and joined
 * back into the context's stream with events, so the call as a whole is
 * ordered on the context's stream like every other call.
 * Workspace: nrs_solve_batched_workspace_size() bytes for the same problem
 * list (holds every system's FP32 matrix side by side).  The descriptors are
 * staged through a pinned host buffer owned by the context.
 * Refinement runs at most options.max_refine sweeps (<= 0: 3 for batches).
 * With infos == NULL the call is asynchronous.  With infos != NULL it
 * synchronises, fills infos[B], and solves any system whose refinement
 * failed again alone with FP64 partial pivoting (fell_back = 1) unless
 * options.no_fallback is set, in which case NRS_E_NOT_CONVERGED is returned.
 * Errors: NRS_E_ARG (bad sizes, NULL arrays, bad nu/body values),
 * NRS_E_UNSUPPORTED (method other than NRS_FP32_IR, n > 262144),
 * NRS_E_WORKSPACE, NRS_E_HIP. */
nrs_status nrs_solve_batched_workspace_size(nrs_ctx* ctx, int32_t B, const nrs_problem* problems,
                                            int32_t method, size_t* bytes);
nrs_status nrs_solve_batched(nrs_ctx* ctx, int32_t B, const nrs_problem* problems,
                             const double* const* u, const double* const* ftext,
                             const nrs_options* opt, void* ws, size_t ws_bytes,
                             double* const* sol, nrs_info* infos);

/* ------------------------------------------------------------------------ */
/* Dense LU and triangular solves on their own (the linear-algebra part of
 * Sec. 4 step 3), for tests and reuse.                                      */
/* ------------------------------------------------------------------------ */
/* In-place LU factorisation of the n x n column-major matrix A (precision 32
 * or 64; 16 = FP32 matrix and factors whose trailing updates take BF16
 * copies of the finished tiles on the matrix cores with FP32 accumulation,
 * pivot_scope 1 only), n <= 262144.
 * pivot_scope = 0: partial pivoting over the whole column, P A = L U.
 * pivot_scope = 1: static block pivoting for use with iterative refinement:
 *   pivots are searched only inside each 64 x 64 diagonal tile, and those
 *   interchanges are not applied to the L tiles left of the diagonal; block
 *   row m (rows 64m .. 64m+63) then satisfies
 *     P_m (A_m - sum_{k<m} L_mk U_k) = L_mm U_m   on the columns >= 64m.
 * Outputs (device):
 *   ipiv [n] int32: ipiv[j] = row interchanged with row j at step j (0-based,
 *        LAPACK order; for scope 1 the interchanges stay inside a tile);
 *   perm [n] int32: scope 0: the composite permutation, (P b)[i] = b[perm[i]];
 *        scope 1: logical row i of its tile came from original row perm[i];
 *   singular_flag [1] int32: bit 0 set if an exact zero pivot is met, bit 1
 *        if a bounded wait between the workgroups of a partial-pivoting
 *        panel timed out (left untouched otherwise; the caller clears it).
 * ws: device workspace of at least nrs_lu_factor_workspace_size(n, precision)
 * bytes, owned by the caller (the tile LU's ticket, flag and timeout words,
 * cleared by the call itself, and for precision 16 the BF16 tile copies,
 * 2 n^2 bytes rounded up to whole tiles).  The same workspace must not be in
 * use by another call that has not completed.  nrs_lu_query() reports
 * whether a bounded wait of the call timed out (the factors are then not
 * valid).  Asynchronous.
 * Errors: NRS_E_ARG (sizes, NULL pointers, lda < n, precision, scope),
 * NRS_E_UNSUPPORTED (n > 262144), NRS_E_WORKSPACE, NRS_E_HIP. */
nrs_status nrs_lu_factor_workspace_size(nrs_ctx* ctx, int64_t n, int32_t precision,
                                        size_t* bytes);
nrs_status nrs_lu_factor(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                         void* A, int64_t lda, int32_t* ipiv, int32_t* perm,
                         int32_t* singular_flag, void* ws, size_t ws_bytes);

/* Solve with the factors of nrs_lu_factor (same pivot_scope and perm):
 * x = A^-1 b, b and x [n] device vectors of the same precision (32 or 64;
 * x may not alias b).  ws: device workspace of at least
 * nrs_lu_solve_workspace_size(n) bytes, owned by the caller (the
 * triangular solves' ticket, flag and solution-word buffers, cleared by the
 * call itself).  Asynchronous; nrs_lu_query() reports a timed-out wait.
 * Errors as nrs_lu_factor. */
nrs_status nrs_lu_solve_workspace_size(nrs_ctx* ctx, int64_t n, size_t* bytes);
nrs_status nrs_lu_solve(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                        const void* LU, int64_t lda, const int32_t* perm, const void* b, void* x,
                        void* ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * nrs_lu_solve without a workspace, same arguments, kernels and results.
 * Its synchronisation words live in a static device array of the library,
 * sized for n <= NRS_NOALLOC_MAX_N (about 517 KiB), one copy per GPU, held
 * until the process ends.  Every call on a GPU uses that GPU's copy: calls
 * that overlap in time on one GPU race (issue them on one stream or
 * otherwise serialise them).  The call clears the words it uses before the
 * solve (with a fill kernel, no memset).  Never calls hipMalloc, hipFree or
 * an allocating routine.  Asynchronous; nrs_lu_query(ctx, NULL, flags)
 * reports its wait-timeout word.  Errors as nrs_lu_solve, and
 * NRS_E_UNSUPPORTED for n > NRS_NOALLOC_MAX_N. */
#define NRS_NOALLOC_MAX_N 65536
nrs_status nrs_lu_solve_noalloc(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                                const void* LU, int64_t lda, const int32_t* perm, const void* b,
                                void* x);

/* Equilibration of an FP32 matrix in place, as nrs_solve applies it before
 * the FP32 factorisation: A <- D_r A D_c with dr_i = 2^-floor(log2 max_j
 * |a_ij|) and dc_j = 2^-floor(log2 max_i dr_i |a_ij|) (1 for an all-zero row
 * or column).  A: n x n column-major, leading dimension lda >= n; dr, dc:
 * [n] FP32 device outputs.  ws: device workspace of at least 4 n bytes
 * (row maxima).  Asynchronous.  Errors: NRS_E_ARG, NRS_E_WORKSPACE. */
nrs_status nrs_equilibrate(nrs_ctx* ctx, int64_t n, float* A, int64_t lda, float* dr, float* dc,
                           void* ws, size_t ws_bytes);

/* Synchronise the context's stream and report the status of the last
 * nrs_lu_factor or nrs_lu_solve that used workspace ws (ws = NULL: the last
 * nrs_lu_solve_noalloc on the context's device): *flags = 1 if one of its
 * bounded waits between workgroups timed out (its output is then not
 * valid), else 0.  Each such call clears the word when it starts. */
nrs_status nrs_lu_query(nrs_ctx* ctx, const void* ws, int32_t* flags);

/* Autotuning of launch shapes.  Times every candidate launch shape of the
 * FP32 and FP64 assembly kernels (rows per workgroup 64 / 128 / 256 x force
 * points per strip 4 / 8 / 16) on this problem (one warm-up launch, then the
 * best of three runs of eight back-to-back launches each, HIP events on the
 * context's stream), and records the fastest
 * for the problem's size class (floor(log2 N), floor(log2(Q / N))) in the
 * context; every later assembly of a problem of that class, in any entry
 * point, uses it.  Every shape computes each matrix entry with the same
 * operations, so tuning never changes a result.  Synchronises.  ws: at least
 * nrs_workspace_size(N, Q, M, NRS_FP32_IR) bytes.  out (host, may be NULL):
 * the choice and its timings. */
typedef struct {
  int32_t size_class;
  int32_t block32, strip32, block64, strip64;
  float ms32, ms64;                 /* tuned average per assembly, ms        */
  float default_ms32, default_ms64; /* default shape (128 rows, 8 points)    */
} nrs_tune_result;
nrs_status nrs_autotune(nrs_ctx* ctx, const nrs_problem* pb, void* ws, size_t ws_bytes,
                        nrs_tune_result* out);
/* Forget every tuned shape of the context (defaults again). */
nrs_status nrs_autotune_clear(nrs_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* Learned block preconditioner for GMRES (not part of the paper's method:  */
/* a preconditioner for the same linear system; the GMRES residual decides).*/
/* ------------------------------------------------------------------------ */
/* A free body's diagonal block of the swimming problem (Sec. 2 and Sec. 4:
 * its rows of the NEAREST operator, Sec. 3 eq. 23, restricted to its own
 * force points, with its rigid-body columns and force and moment rows) is,
 * in the body's own frame, the same for every identical swimmer at the same
 * beat phase psi = omega t - phi: the regularized stokeslet, the nearest map
 * within the body's group and the patch weights do not change when the body
 * is rotated and translated.  The model stores the inverse of that block as
 * a Fourier series in psi, K(psi) = C_0 + sum_{h<=H} (C_ch cos h psi +
 * C_sh sin h psi); NRS_GMRES_BLOCK with NRS_PRECOND_MODEL applies R_b
 * K(psi_b) R_b^T to body b's unknowns (R_b = its frame B on every 3-vector).
 * Blocks here are column-major nb x nb, unknowns ordered as in the system
 * of a single body at the origin with B = I: (f_x of its points, f_y, f_z,
 * U, Omega), nb = 3 N_b + 6. */

/* *nb_max = largest block order the library inverts and applies (192: one
 * workgroup holds the block in registers, FP64); larger bodies are not
 * preconditioned. */
nrs_status nrs_block_limit(nrs_ctx* ctx, int32_t* nb_max);

/* In-place inverses of `count` blocks of order nb (1 <= nb <= nb_max):
 * blocks [count][nb][nb] column-major, each replaced by its inverse (Gauss-
 * Jordan elimination with partial pivoting, FP64).  singular: device int32,
 * |= 1 if a block had a zero or non-finite pivot (that block's output is
 * then not an inverse).  Asynchronous.  Errors: NRS_E_ARG, NRS_E_UNSUPPORTED
 * (nb > nb_max). */
nrs_status nrs_block_invert(nrs_ctx* ctx, int32_t count, int32_t nb, double* blocks,
                            int32_t* singular);

/* Fit of the model to the inverses K_s at the S phases psi_s = 2 pi s / S
 * (s = 0..S-1; inverses [S][nb][nb], e.g. nrs_assemble of a one-body problem
 * in its own frame at each phase followed by nrs_block_invert):
 *   C_0 = (1/S) sum_s K_s,  C_ch = (2/S) sum_s cos(h psi_s) K_s,
 *   C_sh = (2/S) sum_s sin(h psi_s) K_s,   h = 1..H,
 * the least-squares trigonometric fit of degree H since S >= 2H + 1.
 * model: device [2H+1][nb][nb] (C_0, C_c1, C_s1, C_c2, ...).  Asynchronous.
 * Errors: NRS_E_ARG (S < 2H + 1, H outside 0..NRS_BLOCK_MAX_HARMONICS, NULL). */
nrs_status nrs_block_model_fit(nrs_ctx* ctx, int32_t S, int32_t nb, int32_t H,
                               const double* inverses, double* model);

/* The model's K(psi_i) for `count` phases psi [count] (device): blocks
 * [count][nb][nb] column-major.  Asynchronous.  Errors: NRS_E_ARG. */
nrs_status nrs_block_model_eval(nrs_ctx* ctx, int32_t nb, int32_t H, const double* model,
                                int32_t count, const double* psi, double* blocks);

/* ------------------------------------------------------------------------ */
/* Learned warm start for GMRES (not part of the paper's method: an initial */
/* guess for the same linear system; the GMRES residual decides).           */
/* ------------------------------------------------------------------------ */
/* Network: for each free body b with points m (one contiguous run per body,
 * bodies in order), features phi_m = (B^T (x_m - x0), B^T u_m, s_m) in the
 * body frame (x, u lab frame; s the point's arclength parameter), then
 *   h1 = tanh(W1 phi + b1), c = mean h1, h2 = tanh(W2 h1 + V2 c + b2),
 *   y_m = W3 h2 + b3 (3 outputs per point), z_b = W4 mean h2 + b4 (6 per body),
 * hidden width NRS_MLP_HIDDEN.  theta: FP32 [nrs_mlp_param_count()] holding
 * W1 (64 x 7 row-major), b1, W2 (64 x 64), V2 (64 x 64), b2, W3 (3 x 64), b3,
 * W4 (6 x 64), b4.  The model predicts y = B^T f / scales[0] and
 * z = (B^T U / scales[1], B^T Omega / scales[2]). */
#define NRS_MLP_HIDDEN      64
#define NRS_MLP_MAX_POINTS  256   /* force points per body */
#define NRS_WARM_NONE       0
#define NRS_WARM_PREVIOUS   1
#define NRS_WARM_MODEL      2
int64_t nrs_mlp_param_count(void);

/* body_off [M+1] (device) of the point-to-body map body [N]; synchronises and
 * returns NRS_E_ARG unless every body's points form one contiguous run, the
 * runs are in body order and adjacent, and no body has more than
 * NRS_MLP_MAX_POINTS points. */
nrs_status nrs_mlp_body_offsets(nrs_ctx* ctx, int64_t N, const int32_t* body, int32_t M,
                                int32_t* body_off);
/* phi [N][7] FP32; points with body < 0 get zeros.  x, u: [3][N]; s: [N];
 * Y: [M][12]. */
nrs_status nrs_mlp_features(nrs_ctx* ctx, int64_t N, const double* x, const double* u,
                            const double* s, const int32_t* body, int32_t M, const double* Y,
                            float* phi);
/* Forward pass over N points in M bodies (phi [N][7]).  sel: device [nsel]
 * body ids, or NULL for all M bodies.  y: [N][3] written at the points of the
 * evaluated bodies; z: [M][6].  A body id outside [0, M) or a range outside
 * [0, N) or longer than NRS_MLP_MAX_POINTS is skipped and raises bit 1 of
 * nrs_mlp_status. */
nrs_status nrs_mlp_forward(nrs_ctx* ctx, const float* theta, int64_t N, int32_t M,
                           const int32_t* body_off, const int32_t* sel, int32_t nsel,
                           const float* phi, float* y, float* z);
/* Loss L = mean over the selected bodies of (mean over the body's points and
 * components of (y - t_pt)^2 + mean over the 6 components of (z - t_body)^2)
 * and its gradient: grad [nrs_mlp_param_count() + 1], last entry L.  The
 * per-body contributions are summed in a fixed order (deterministic).
 * t_pt: [N][3]; t_body: [M][6]; ws: nrs_mlp_grad_workspace_size bytes. */
nrs_status nrs_mlp_grad_workspace_size(int32_t nsel, size_t* bytes);
nrs_status nrs_mlp_grad(nrs_ctx* ctx, const float* theta, int64_t N, int32_t M,
                        const int32_t* body_off, const int32_t* sel, int32_t nsel,
                        const float* phi, const float* t_pt, const float* t_body, float* grad,
                        void* ws, size_t ws_bytes);
/* Adam (Kingma and Ba 2015) step number `step` >= 1 on count parameters:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
nrs_status nrs_adam_step(nrs_ctx* ctx, int64_t count, float* theta, const float* grad, float* m,
                         float* v, int32_t step, float lr, float beta1, float beta2, float eps);
/* Training targets from a solution sol [3N + 6M]: t_pt = B^T f / scales[0],
 * t_body = (B^T U / scales[1], B^T Omega / scales[2]); scales: HOST [3]. */
nrs_status nrs_mlp_targets(nrs_ctx* ctx, int64_t N, int32_t M, const int32_t* body,
                           const double* Y, const double* sol, const double* scales,
                           float* t_pt, float* t_body);
/* Initial guess x0 [3N + 6M] (FP64) from the network: features, forward pass
 * and the map back to the lab frame (zero force density at points outside
 * the bodies).  scales: HOST [3]; ws: nrs_mlp_warm_start_workspace_size. */
nrs_status nrs_mlp_warm_start_workspace_size(int64_t N, int32_t M, size_t* bytes);
nrs_status nrs_mlp_warm_start(nrs_ctx* ctx, const float* theta, const double* scales, int64_t N,
                              int32_t M, const int32_t* body, const int32_t* body_off,
                              const double* x, const double* u, const double* s,
                              const double* Y, double* x0, void* ws, size_t ws_bytes);
/* Synchronise, return and clear the sticky error bits of the network kernels
 * (1: a body id or point range was invalid and the body was skipped). */
nrs_status nrs_mlp_status(nrs_ctx* ctx, int32_t* flags);

/* ------------------------------------------------------------------------ */
/* Time stepping (Sec. 4: Y' = F(Y, t), F from the solve).                   */
/* ------------------------------------------------------------------------ */
/* One classical RK4 step of the body states Y [M][12] (in place) from t to
 * t + dt.  Each of the four stages evaluates the geometry, the nearest map
 * (group_off_host / groupX as in nrs_nearest), the solve (method in opt) and
 * the rates dx0/dt = U, dB/dt = [Omega]x B; after the step each body frame
 * is re-orthonormalised by modified Gram-Schmidt.  ftext: [M][6] or NULL.
 * Asynchronous; the numerical status of the four solves accumulates in the
 * workspace (nrs_query_info: fell_back/iterations report the worst stage).
 * ws must hold nrs_rk4_workspace_size bytes. */
nrs_status nrs_rk4_workspace_size(nrs_ctx* ctx, const nrs_scene* sc, int32_t method, size_t* bytes);
nrs_status nrs_rk4_step(nrs_ctx* ctx, const nrs_scene* sc, int32_t G, const int32_t* group_off_host,
                        const int32_t* groupX, double eps, double mu, const double* ftext,
                        double* Y, double t, double dt, const nrs_options* opt,
                        void* ws, size_t ws_bytes);

/* Adaptive time stepping with the Dormand-Prince 5(4) pair (Dormand and
 * Prince, 1980; the kind of integrator the paper's MATLAB ode45 is): Y [M][12]
 * (in place) from t0 to t1.  Every attempt evaluates six new stages (the
 * geometry, nearest map, solve with opt->method and rates of nrs_rk4_step);
 * its first stage is the last stage of the previous accepted step.  Error
 * estimate e = h sum_i (b5_i - b4_i) k_i, norm ||e / (atol + rtol max(|y|,
 * |y_new|))||_rms; accepted when <= 1; next step h * min(10, 0.9 norm^-1/5)
 * after an acceptance (at most h right after a rejection), h * max(0.2,
 * 0.9 norm^-1/5) after a rejection; the last step is cut to end at t1.  Body
 * frames are not re-orthonormalised between steps.  *h_io: first step in,
 * proposed next step out.  At most max_steps attempts.  Synchronises with
 * the host once per attempt (one scalar and the solve status); if a stage
 * solve misses its tolerance the attempt is redone with NRS_FP64_LU (unless
 * opt->no_fallback).  stats (host, may be NULL): attempts and solves. */
typedef struct {
  int32_t accepted, rejected, solves, fell_back;
  double t;   /* time reached */
  double h;   /* proposed next step */
} nrs_dopri5_stats;
nrs_status nrs_dopri5_workspace_size(nrs_ctx* ctx, const nrs_scene* sc, int32_t method,
                                     size_t* bytes);
nrs_status nrs_dopri5_integrate(nrs_ctx* ctx, const nrs_scene* sc, int32_t G,
                                const int32_t* group_off_host, const int32_t* groupX, double eps,
                                double mu, const double* ftext, double* Y, double t0, double t1,
                                double* h_io, double rtol, double atol, const nrs_options* opt,
                                int32_t max_steps, nrs_dopri5_stats* stats, void* ws,
                                size_t ws_bytes);

/* ------------------------------------------------------------------------ */
/* Flow at field points and passive tracers.  The regularized single-layer  */
/* equation (Sec. 3, eq. 19) holds anywhere in the fluid, so the nearest-   */
/* neighbour sum of eq. 23 evaluated at a field point y gives the velocity  */
/* there; the particle-tracking experiments (Sec. 4.3, Sec. 5.2) carry      */
/* tracers with it.  Tracers do not act on the fluid.                       */
/* ------------------------------------------------------------------------ */
/* Bytes of device workspace nrs_field_velocity and nrs_tracer_rk4_step need
 * for P field points and up to Q quadrature points (0 <= P <= 2^28). */
nrs_status nrs_field_workspace_size(nrs_ctx* ctx, int64_t P, int64_t Q, size_t* bytes);

/* u_j(y_p) = (8 pi mu)^-1 sum_q S^eps_jk(y_p - X_q) w_q f_k[nu(q)]
 * for P field points y [3][P] (component-major, device, FP64).  Reads
 * pb->N, Q, X, w (NULL = all 1), nu, eps and mu only; f [3][N] (device) are
 * the force densities, i.e. the first 3N entries of a solution of
 * nrs_solve.  Quadrature points whose nu is outside [0, N) contribute
 * nothing.  u [3][P] (device) may alias y.  P = 0 does nothing.  The result
 * does not depend on the order of the quadrature points beyond rounding, and
 * repeated calls with the same sizes give identical bits.  Asynchronous.
 * Errors: NRS_E_ARG (NULL arrays, sizes, eps or mu), NRS_E_UNSUPPORTED
 * (N > 2^20 or Q > 2^30), NRS_E_WORKSPACE, NRS_E_HIP. */
nrs_status nrs_field_velocity(nrs_ctx* ctx, const nrs_problem* pb, const double* f, int64_t P,
                              const double* y, double* u, void* ws, size_t ws_bytes);

/* One classical RK4 step of P tracers y [3][P] (device, in place) through
 * flows known in advance (forces precomputed, as in the node experiment):
 * flows[0..2] (HOST array of three problems, fields as in nrs_field_velocity)
 * with force densities f[0..2] (HOST array of three device pointers) are the
 * flow at t, t + dt/2 and t + dt; both middle stages use flows[1]:
 *   k1 = u0(y), k2 = u1(y + dt/2 k1), k3 = u1(y + dt/2 k2), k4 = u2(y + dt k3),
 *   y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * ws: nrs_field_workspace_size(P, largest Q of the three) bytes.
 * Asynchronous; errors as nrs_field_velocity. */
nrs_status nrs_tracer_rk4_step(nrs_ctx* ctx, const nrs_problem* flows, const double* const* f,
                               int64_t P, double* y, double dt, void* ws, size_t ws_bytes);

/* nrs_rk4_step with P passive tracers ytr [3][P] (device, in place) carried
 * by the same step: every stage evaluates its own flow (that stage's
 * geometry and solved forces) at the tracers' stage positions, and the
 * tracers take the RK4 combination of the four rates (not orthonormalised).
 * If the step is redone with FP64 LU, the tracers are redone with it.
 * P = 0 is nrs_rk4_step.  ws: nrs_rk4_tracers_workspace_size bytes
 * (P = 0 gives nrs_rk4_workspace_size). */
nrs_status nrs_rk4_tracers_workspace_size(nrs_ctx* ctx, const nrs_scene* sc, int32_t method,
                                          int64_t P, size_t* bytes);
nrs_status nrs_rk4_step_tracers(nrs_ctx* ctx, const nrs_scene* sc, int32_t G,
                                const int32_t* group_off_host, const int32_t* groupX, double eps,
                                double mu, const double* ftext, double* Y, double t, double dt,
                                const nrs_options* opt, int64_t P, double* ytr, void* ws,
                                size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* NRS_H */
