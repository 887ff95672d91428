// Internal declarations shared by the libnrs translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nrs.h"

namespace nrs {
constexpr int32_t kBlockMax = 192;   // largest body block order of the block preconditioner (62 points)
}

// A captured batched solve (nrs_solve_batched with options.graph): the
// executable graph, the argument hash it was captured for, and the pinned
// host copy of the batch descriptors its copy nodes read.
struct nrs_graph_entry {
  uint64_t key;
  hipGraphExec_t exec;
  void* host_desc;
};

// Autotuned assembly launch shape of one size class (see nrs_autotune).
struct nrs_tune_entry {
  int32_t cls;       // size class: 64 * floor(log2 N) + floor(log2(Q / N))
  int32_t shape32;   // assembly shape index, FP32 (-1: not tuned)
  int32_t shape64;   // FP64
};

struct nrs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // device address of the library's static scratch array on this device
  // (the no-allocation triangular solve), from hipGetSymbolAddress
  int32_t* scratch = nullptr;
  // largest body block order of the block preconditioner
  int32_t block_lim = nrs::kBlockMax;
  // Arnoldi steps queued ahead of the first host check of a block-preconditioned
  // GMRES solve (the previous solve's iteration count plus one)
  int32_t bg_chunk = 6;
  // pinned host staging of batch descriptors; the event marks the last copy
  void* staging = nullptr;
  size_t staging_cap = 0;
  hipEvent_t staging_event = nullptr;
  // zero-initialised device words for sticky kernel error bits ([0]: network)
  int32_t* dflags = nullptr;
  // workspace of the last completed nrs_rk4_step (its solution seeds the next
  // step's first GMRES solve under NRS_WARM_PREVIOUS)
  const void* rk_prev_ws = nullptr;
  // correction sweeps the stages of that step needed at most (0: unknown);
  // sizes the adaptive refinement queue of the next step
  int32_t rk_sweeps = 0;
  // captured batched solves, oldest first (at most kMaxGraphs)
  std::vector<nrs_graph_entry> graphs;
  // autotuned assembly shapes by size class
  std::vector<nrs_tune_entry> tune;
  // side streams of the batched solve (default priority): the per-system
  // kernels of a batch are spread over the context's stream and these, forked
  // from and joined back into the context's stream with events, so that the
  // short kernels of different systems overlap
  static constexpr int kAux = 3;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kAux] = {};
};

namespace nrs {
// Tuned assembly shape for a problem of N force and Q quadrature points in
// precision bits (32 / 64), or -1 (default shape) if its class is not tuned.
int32_t asm_shape_for(const nrs_ctx* ctx, int64_t N, int64_t Q, int bits);
int32_t size_class(int64_t N, int64_t Q);
}  // namespace nrs

nrs_status ctx_dev_flags(nrs_ctx* ctx);   // allocates ctx->dflags (zeroed) on first use

inline nrs_status set_error(nrs_ctx* ctx, nrs_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

namespace nrs {

constexpr int kMaxGroups = 512;
constexpr double kPi = 3.14159265358979323846;

struct GroupTable {
  int32_t G;
  int32_t off[kMaxGroups + 1];
};

// Solve status words kept in the workspace (device) so that an asynchronous
// solve can be inspected later.
struct SolveState {
  int32_t converged;    // refinement / GMRES reached its tolerance
  int32_t failed;       // refinement diverged or stagnated
  int32_t iterations;
  int32_t singular;     // zero pivot met
  int32_t method_used;
  int32_t fell_back;
  int32_t nonfinite;
  int32_t stop;
  int32_t sync_err;     // a bounded wait in the triangular solves timed out
  int32_t prec_err;     // block preconditioner set-up: 2 bodies not runs, 4 block too large,
                        // 8 block order differs from the model's
  int32_t lu_ctl[4];    // tile LU: ticket, exit count, wait-timeout flag         // converged || failed: refinement kernels become no-ops
  double bwd;           // normwise backward error of the last residual
  double corr;          // last |d|/|x|
  double prev_corr;
  double anorm;         // |A|_inf of the FP64 operator (estimated from the FP32 copy)
};

// Bump allocator over a caller-provided workspace.
struct Arena {
  char* base;
  size_t cap;
  size_t used = 0;
  bool overflow = false;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    used = off + bytes;
    if (base == nullptr || used > cap) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T*>(base + off);
  }
};

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline int64_t lda_for(int64_t n) { return round_up(n < 1 ? 1 : n, 64); }
// doubles of scratch the |A|_inf kernels need
inline int64_t rowsum_chunks(int64_t n) { return n <= 4096 ? (n + 255) / 256 : 16; }
inline int64_t rowsum_scratch(int64_t n) { return rowsum_chunks(n) * n + 1024; }

// One quadrature point as a source of the field sum: position and
// g = w_q f[nu(q)] (zero when nu(q) is outside [0, N)); 64 bytes so that a
// wave reads a record with one scalar load.
struct alignas(64) FieldSrc {
  double X, Y, Z, gx, gy, gz, pad0, pad1;
};

// Sorted quadrature data, produced by build_csr.
struct Sorted {
  int32_t* seg;      // [N+1] segment offsets into the sorted order
  int32_t* perm;     // [Q] original index of sorted point p
  int32_t* nus;      // [Q] nearest force point of sorted point p
  double4* X64;      // [Q] (x, y, z, w) in FP64
  float4* X32hi;     // [Q] (x_hi, y_hi, z_hi, w) in FP32
  float4* X32lo;     // [Q] (x_lo, y_lo, z_lo, 0): x = x_hi + x_lo to FP32 x FP32 precision
  double* W;         // [N] patch weights
  int32_t* cnt;      // [N+2] scratch; cnt[N+1] counts quadrature points with nu out of range
  FieldSrc* fsrc;    // [Q] source records of the matrix-free product (original order)
};

// All device buffers of one solve, carved from the workspace.
struct SolveBuffers {
  Sorted srt;
  float* A32;        // lda x n (FP32 path)
  double* A64;       // lda x n (FP64 path / fallback)
  int64_t lda;
  int32_t* ipiv;     // [n]
  int32_t* perm;     // [n] composite row permutation of the factorisation
  int32_t* perm64;   // [n] same for the FP64 fallback factors
  int32_t* ipiv64;
  double* b;         // [n]
  double* x;         // [n] current solution
  double* r;         // [n] residual
  float* d32;        // [n]
  double* d64;       // [n]
  double* part;      // [chunks][3N] partial products of the matrix-free apply
  double* red;       // reduction scratch
  int32_t* tsync;    // triangular-solve synchronisation words (zero between calls)
  int32_t* lu_done;  // [nt*nt] tile flags of the tile LU
  SolveState* st;
  int32_t chunks;
  // GMRES (method NRS_GMRES only)
  double* AT;        // lda x n row-major copy of A64
  double* V;         // [n][kGmresLd]
  double* gw0;
  double* gw1;
  double* gpart;
  struct GmresState* gst;
  double* Z;         // flexible GMRES: preconditioned basis [n][kGmresLd]
  double* fzv;       // [n] z_k, the operator's input
  double* fax;       // [n] A x for the true residual
  uint16_t* sh;      // BF16 tile copies of the tile LU (NRS_BF16_GMRES_IR)
  void* gepp;        // scratch of the partial-pivoting panel (gepp_scratch_bytes)
  float* eqr;        // [n] row scale factors of the equilibrated FP32 matrix
  float* eqc;        // [n] column scale factors
  uint32_t* eqmax;   // [n] row maxima (scratch of the equilibration)
  bool equil;        // the FP32 factors are of D_r A D_c (eqr, eqc valid)
  // block preconditioner (NRS_GMRES_BLOCK)
  int32_t* boff;     // [M+1] body point offsets
  int32_t* bstarts;  // [1] counter of the body-run check
  double* bpsi;      // [M] beat phase of every body
  double* blocks;    // [M][kBlockStride] body blocks / their inverses
  const nrs_scene* phase_scene;   // time stepping: the scene whose wave parts give
  double phase_t;                 // every body's phase at time phase_t (else NULL)
};

size_t solve_workspace_bytes(int64_t N, int64_t Q, int32_t M, int32_t method);
// with64 = false leaves out the FP64 matrix and the tile LU's row-tile
// hand-over area (batched FP32 solves)
bool carve_solve(Arena& ar, int64_t N, int64_t Q, int32_t M, int32_t method, SolveBuffers& sb,
                 bool with64 = true);

// One system of the persistent tile LU (64 x 64 tiles, static block pivoting).
template <class T>
struct LuSys {
  T* A;             // column-major, leading dimension lda
  int64_t lda;
  int64_t n;
  int64_t nt;       // tiles per dimension, ceil(n / 64)
  int32_t* lperm;   // [n] block-local permutation: logical row r <- original row lperm[r]
  int32_t* ipiv;    // [n] LAPACK-style interchanges (may be NULL)
  int32_t* done;    // [nt * nt] tile completion flags, zero before the launch
  int32_t* sing;    // set to 1 on an exact zero pivot
  // BF16 copies of the finished off-diagonal tiles, 64 x 64 each at
  // (i nt + j) * 4096, k index contiguous (L tiles [row][k], U tiles
  // [column][k]); when set (FP32 only), the trailing updates take these as
  // matrix-core inputs (BF16 in, FP32 accumulate).  NULL: FP32 updates.
  uint16_t* sh = nullptr;
  // Single FP32 system run one workgroup per CU (NULL otherwise): the row
  // tile (m + 1, m) before its solve, 64 x 64 column-major at m * 4096, and
  // its flag, so that the diagonal task of band m + 1 solves it itself.
  T* pre = nullptr;
  int32_t* preflag = nullptr;
};
template <class T>
struct LuBatch {
  LuSys<T> one;            // used when sys == NULL (single system)
  const LuSys<T>* sys;     // device array of B systems, or NULL
  const int32_t* pref;     // device ticket prefix over (band, system), or NULL
  int32_t B;
  int32_t nbands;
  int32_t total;           // number of tasks
};
// ctl: [0] ticket, [1] exit count (both zero before launch, cleared by the
// kernel), [2] sticky wait-timeout flag
template <class T>
hipError_t launch_lu_tiles(const LuBatch<T>& bt, int32_t* ctl, hipStream_t s);
void lu_task_prefix(const int32_t* nts, int32_t B, std::vector<int32_t>& pref, int32_t& nbands);

// One system of the multi-workgroup triangular solves.
template <class T>
struct TrsvSys {
  const T* LU;
  int64_t lda;
  int64_t n;
  T* x;                 // solution (upper pass in place)
  const T* rhs;         // right-hand side of the lower pass
  const int32_t* perm;  // scope 0: composite permutation; scope 1: tile-local
  int32_t* flags;       // [ceil(n/64)] block flags, zero before the launch (FP64)
  const int32_t* stop;  // nonzero: skip this system (may be NULL)
  int32_t* epoch;       // launch counter of this system's sweeps (FP32)
  uint64_t* xp;         // [n] tagged solution words (epoch tag, value bits) (FP32)
};
template <class T>
struct TrsvBatch {
  TrsvSys<T> one;           // used when sys == NULL (single system)
  const TrsvSys<T>* sys;    // device array of B systems, or NULL
  const int32_t* pref;      // device ticket prefix over (step, system), or NULL
  int32_t B;
  int32_t nsteps;           // max blocks over systems
  int32_t total;            // number of tickets (sum of blocks)
};
// Lower then upper pass over a batch; ctl[0..1] zero before, kept zero.
template <class T>
hipError_t launch_trsv_batch(const TrsvBatch<T>& bt, int32_t scope, int32_t* ctl, int32_t* err,
                             hipStream_t s);

// ---- learned warm start (learn.hip) ----
constexpr int kMlpHidden = 64;     // hidden width: one wavefront
constexpr int kMlpMaxPts = 256;    // force points per body
constexpr int kMlpParams = kMlpHidden * 7 + kMlpHidden + 2 * kMlpHidden * kMlpHidden +
                           kMlpHidden + 3 * kMlpHidden + 3 + 6 * kMlpHidden + 6;
// nb workgroups (bodies sel[0..nb) or 0..nb); nbodies / npts bound the body ids
// and point ranges (invalid ones are skipped with err bit 1)
hipError_t launch_mlp_forward(const float* th, int32_t nb, int32_t nbodies, int64_t npts,
                              const int32_t* body_off, const int32_t* sel, const float* phi,
                              float* y, float* z, int32_t* err, hipStream_t s);
// rows: [nsel][kMlpParams + 1] scratch; grad: [kMlpParams + 1], last = loss
hipError_t launch_mlp_grad(const float* th, int32_t nbodies, int64_t npts,
                           const int32_t* body_off, const int32_t* sel, int32_t nsel,
                           const float* phi, const float* t_pt, const float* t_body, float* rows,
                           float* grad, int32_t* err, hipStream_t s);
hipError_t launch_adam(int64_t count, float* th, const float* g, float* m, float* v, int32_t t,
                       float lr, float beta1, float beta2, float eps, hipStream_t s);
// off: [M+1] body point offsets; starts: one counter word; err |= 2 if a
// body's points are not one contiguous run in body order or exceed kMlpMaxPts
hipError_t launch_body_off(int64_t N, int32_t M, const int32_t* body, int32_t* off,
                           int32_t* starts, int32_t* err, hipStream_t s);
hipError_t launch_features(int64_t N, const double* x, const double* u, const double* sarc,
                           const int32_t* body, int32_t M, const double* Y, float* phi,
                           hipStream_t s);
hipError_t launch_targets(int64_t N, int32_t M, const int32_t* body, const double* Y,
                          const double* sol, const double* sc, float* t_pt, float* t_body,
                          hipStream_t s);
hipError_t launch_to_lab(int64_t N, int32_t M, const int32_t* body, const double* Y,
                         const float* y, const float* z, const double* sc, double* x0,
                         hipStream_t s);

// ---- block preconditioner (precond.hip) ----
constexpr int64_t kBlockStride = (int64_t)kBlockMax * kBlockMax;
constexpr int32_t kBlockHarmonicsMax = 16;    // harmonics of the learned block model
// err |= 4 for a body block above nb_lim, 8 for one whose order is not nb_model (> 0)
hipError_t launch_block_check(int32_t M, int64_t N, const int32_t* off, int32_t nb_lim,
                              int32_t nb_model, int32_t* err, hipStream_t s);
// psi[b] = omega t - phi of body b's first wave point (scene arrays part, wave)
hipError_t launch_body_phase(int32_t M, int64_t N, const int32_t* off, const int32_t* part,
                             const double* wave, int32_t P, double t, double* psi, hipStream_t s);
// the diagonal body blocks of the stored FP64 matrix, column-major, stride kBlockStride
hipError_t launch_block_extract(int32_t M, int64_t N, const int32_t* off, int32_t nb_lim,
                                const double* A, int64_t lda, double* blocks, hipStream_t s);
// in-place inverses of `count` blocks: off == NULL -> all of order nb_uniform
// at the given stride; else the bodies' blocks (orders from off, <= nb_lim)
hipError_t launch_block_inverse(int32_t count, int32_t nb_uniform, int64_t stride, int64_t N,
                                const int32_t* off, int32_t nb_lim, double* blocks, int32_t* sing,
                                hipStream_t s);
// Fourier coefficients [2H+1][nb*nb] of S inverses at phases 2 pi s / S
hipError_t launch_block_fit(int32_t S, int32_t nb, int32_t H, const double* inv, double* model,
                            hipStream_t s);
// blocks[b] = K(psi[b]) of the model; off != NULL: only bodies of order nb
hipError_t launch_block_model(int32_t count, int64_t N, const int32_t* off, int32_t nb_lim,
                              int32_t nb, int32_t H, const double* model, const double* psi,
                              int64_t stride, double* blocks, hipStream_t s);
struct GmresArgs;
// z_k = M^-1 v_k of the flexible GMRES in a (Y != NULL: body-frame blocks).
// begin = true: first normalise the new basis vector into V[:, k] and copy
// it to Z[:, k] and zv (the multi-workgroup Arnoldi kernels leave it
// unnormalised); false: V[:, k], Z[:, k] and zv already hold it (the
// one-workgroup kernels below write it).
hipError_t launch_prec_block(const GmresArgs& a, int32_t M, int64_t N, const int32_t* off,
                             int32_t nb_lim, int32_t nb_model, const double* Y,
                             const double* blocks, double* zv, bool begin, hipStream_t s);
// One-workgroup flexible GMRES kernels for n <= kGmresSmallN (rows held in
// registers, no inter-workgroup reductions): the residual (only_if_stopped:
// skips unless the current cycle has stopped), the Arnoldi orthogonalisation
// of A z_k (CGS2, Givens rotations, stop rules as the multi-workgroup
// kernels) and the end-of-cycle update x += Z y (skips unless stopped).  The
// residual and the orthogonalisation also write the next basis vector into
// V, Z (identity outside the bodies) and zv.
constexpr int64_t kGmresSmallN = 8192;
hipError_t launch_bg_residual(const GmresArgs& a, const double* Ax, bool only_if_stopped,
                              double* zv, hipStream_t s);
hipError_t launch_bg_orth(const GmresArgs& a, const double* Aw, double* zv, hipStream_t s);
hipError_t launch_bg_update(const GmresArgs& a, hipStream_t s);

// ---- GMRES (gmres.hip) ----
constexpr int kGmresLd = 64;       // basis row length; restart m <= kGmresLd - 1
struct GmresState {
  int32_t done;       // true residual <= tol |b|
  int32_t stop;       // current cycle finished (estimate converged, breakdown, m or max_iter)
  int32_t fail;       // non-finite values
  int32_t k;          // Arnoldi steps in the current cycle
  int32_t iters;      // total Arnoldi steps
  int32_t cur;        // which w buffer holds the next (unnormalised) basis vector
  int32_t counter;    // last-workgroup ticket (zero between launches)
  int32_t m, max_iter;
  int32_t halt;       // done | stop | fail: launches queued behind a finished cycle skip
  int32_t skip_true;  // !stop | done | fail: the end-of-cycle launches queued ahead skip
  double tol, bnorm, beta, nrm;
  double g[kGmresLd + 1], cs[kGmresLd], sn[kGmresLd], h1[kGmresLd], h2[kGmresLd];
  double H[(kGmresLd + 1) * kGmresLd];   // column-major, leading dimension kGmresLd + 1
};
struct GmresArgs {
  int64_t n, ld;
  const double* AT;   // row-major operator, row r at AT + r * ld
  const double* b;
  double* x;
  double* V;          // [n][kGmresLd]
  double* Z = nullptr;  // [n][kGmresLd] preconditioned basis (flexible GMRES), else NULL
  double* w0;
  double* w1;
  double* part;       // [gmres_blocks(n)][kGmresLd]
  GmresState* st;
  const float* eqr = nullptr;  // flexible GMRES on equilibrated factors: the
  const float* eqc = nullptr;  // preconditioner is D_c (LU)^-1 D_r
};
int64_t gmres_blocks(int64_t n);
hipError_t launch_transpose64(int64_t n, const double* A, int64_t lda, double* AT, int64_t ld,
                              hipStream_t s);
hipError_t launch_gmres_init(GmresState* st, double tol, int32_t m, int32_t max_iter,
                             hipStream_t s);
hipError_t launch_gmres_residual(const GmresArgs& a, hipStream_t s);
hipError_t launch_gmres_steps(const GmresArgs& a, int32_t count, hipStream_t s);
hipError_t launch_gmres_update(const GmresArgs& a, hipStream_t s);
// Flexible GMRES with a preconditioner between the Arnoldi steps (GMRES-IR):
// the operator products are computed outside (Ax, Aw given), the preconditioner
// input is v32 (FP32 copy of the new basis vector) and its output d32.
hipError_t launch_fgmres_residual(const GmresArgs& a, const double* Ax, hipStream_t s);
hipError_t launch_fgmres_begin(const GmresArgs& a, float* v32, hipStream_t s);
hipError_t launch_fgmres_zstore(const GmresArgs& a, const float* d32, double* zv, hipStream_t s);
// Aw = A z_k: into the next basis buffer, dots with V, then the two CGS passes
hipError_t launch_fgmres_orth(const GmresArgs& a, const double* Aw, hipStream_t s);
// adds the GMRES iterations to the solve state and reports convergence
hipError_t launch_fgmres_report(SolveState* st, const GmresState* g, hipStream_t s);
// Initial-guess completion for swimming problems: project the forces of x0
// onto the force / torque balance (weights W, targets ftext or zero), then
// refit every body's (U, Omega) to the velocity residual by least squares.
// res: [n] scratch, small: [6M] scratch.
hipError_t launch_rigid_completion(int64_t N, int32_t M, const double* x, const double* Y,
                                   const int32_t* body, const double* W, const double* ftext,
                                   const double* AT, int64_t ld, const double* b, double* x0,
                                   double* res, double* small, hipStream_t s);
// converged / failed / iterations of the GMRES state into the solve state
hipError_t launch_gmres_report(SolveState* st, const GmresState* g, hipStream_t s);

// ---- kernels / launchers (each returns hipError_t of the launch) ----
hipError_t launch_geometry(const nrs_scene& sc, double t, const double* Y, double* x, double* X,
                           double* w, double* u, hipStream_t s);
hipError_t launch_nearest(int64_t N, const double* x, const GroupTable& gt, int64_t Q,
                          const double* X, const int32_t* groupX, int32_t* nu, hipStream_t s);
// nu-sorted layout (counting sort, deterministic order inside segments),
// packed coordinates and patch weights; st (may be NULL) gets the argument
// error of a nu outside [0, N)
hipError_t launch_build_csr(int64_t N, int64_t Q, const double* X, const double* w,
                            const int32_t* nu, Sorted& srt, SolveState* st, hipStream_t s);
// Assembly launch shapes: shape index -> (rows per workgroup, force points
// per strip); -1 = default.  Results do not depend on the shape.
constexpr int kAsmShapes = 9;
constexpr int kAsmDefaultShape = 4;   // 128 rows, 8 force points
void asm_shape_dims(int32_t shape, int32_t* blk, int32_t* tn);
template <class T>
hipError_t launch_assemble(const nrs_problem& pb, const Sorted& srt, T* A, int64_t lda,
                           hipStream_t s, int32_t shape = -1);
hipError_t launch_rhs(int64_t N, int32_t M, const double* u, const double* ftext, double* b,
                      hipStream_t s, float* b32 = nullptr, const int32_t* body = nullptr,
                      SolveState* st = nullptr);
hipError_t launch_apply(const nrs_problem& pb, const Sorted& srt, const double* v, double* y,
                        double* part, int32_t chunks, const int32_t* stop, hipStream_t s);
template <class T>
hipError_t launch_lu_factor(int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* perm,
                            int32_t* sing, hipStream_t s, void* scratch = nullptr);
// bytes of the GEPP panel scratch (candidate rows, barrier counters) for order n
size_t gepp_scratch_bytes(int64_t n);
// Factor with scope 0 (GEPP, lu.hip) or 1 (tile LU with static block
// pivoting, lu_tiles.hip; done [nt*nt] and ctl [4] zero before the call).
// gepp: NULL or gepp_scratch_bytes(n) bytes for scope 0 (multi-workgroup panel).
template <class T>
hipError_t lu_factor_any(int64_t n, int32_t scope, T* A, int64_t lda, int32_t* ipiv,
                         int32_t* perm, int32_t* sing, int32_t* done, int32_t* ctl,
                         hipStream_t s, uint16_t* sh = nullptr, void* gepp = nullptr);
// elements of the BF16 tile copies of an order-n tile LU
inline int64_t lu_shadow_elems(int64_t n) {
  const int64_t nt = (n + 63) / 64;
  return nt * nt * 4096;
}
inline int64_t lu_tiles_nt(int64_t n) { return (n + 63) / 64; }
// Caller workspace of nrs_lu_factor / nrs_lu_solve: a head of kLuHeadInts
// words (factor: [0] ticket, [1] exit count, [2] wait-timeout flag; solve:
// [2] wait-timeout flag), then the call's synchronisation words, then (factor
// with BF16 update inputs) the BF16 tile copies, 256-byte aligned.
constexpr int64_t kLuHeadInts = 64;
constexpr int64_t kLuTimeoutWord = 2;
// A single FP32 system of at most kLuSoloTiles tile rows runs the tile LU one
// workgroup per CU; up to kLuHandoverTiles tile rows its diagonal tasks also
// solve the preceding row tile themselves (LuSys::pre).  Measured, FP32 LU
// without -> with the hand-over: n = 2048 0.99 -> 0.97 ms, n = 3150 1.52 ->
// 1.48 ms, n = 4096 1.97 -> 1.93 ms, n = 5000 2.46 -> 2.45 ms, but n = 6300
// 3.39 -> 3.60 ms (the hand-over store then delays the row tile's own solve,
// which later tasks of the band wait for).
constexpr int64_t kLuSoloTiles = 112;
constexpr int64_t kLuHandoverTiles = 80;
// Tile-LU synchronisation words: nt * nt tile flags, then (nt <=
// kLuHandoverTiles) nt hand-over flags, all zero before a launch; then the
// hand-over tiles, nt x 4096 FP32 words from a 64-word boundary.
inline int64_t lu_done_flag_ints(int64_t n) {
  const int64_t nt = lu_tiles_nt(n);
  return nt * nt + (nt <= kLuHandoverTiles ? nt : 0);
}
inline int64_t lu_done_ints(int64_t n) {
  const int64_t nt = lu_tiles_nt(n);
  return (lu_done_flag_ints(n) + 63) / 64 * 64 + (nt <= kLuHandoverTiles ? nt * 4096 : 0);
}
inline int64_t lu_factor_sync_ints(int64_t n) { return kLuHeadInts + lu_done_ints(n); }
template <class T>
hipError_t launch_lu_solve(int64_t n, int32_t scope, const T* LU, int64_t lda,
                           const int32_t* perm, const T* b, T* x, int32_t* sync, int32_t* err,
                           const int32_t* stop, hipStream_t s);
// ints of the zero-initialised synchronisation buffer launch_lu_solve needs.
// Layout (int32 units): [0] ticket, [1] exit count, [2, 2 + nblk) block flags,
// [2 + nblk] epoch, then n 64-bit tagged solution words (8-byte aligned).
inline int64_t trsv_sync_ints(int64_t n) { return 2 + (n + 63) / 64 + 2 + 2 * n; }
inline int32_t* trsv_epoch(int32_t* sync, int64_t n) { return sync + 2 + (n + 63) / 64; }
inline uint64_t* trsv_xp(int32_t* sync, int64_t n) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(trsv_epoch(sync, n) + 1);
  return reinterpret_cast<uint64_t*>((a + 7) & ~uintptr_t(7));
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_ipiv_to_perm(int64_t n, const int32_t* ipiv, int32_t* perm, hipStream_t s);

// refinement helpers
hipError_t launch_state_init(SolveState* st, int32_t method, hipStream_t s);
hipError_t launch_anorm32(int64_t n, const float* A, int64_t lda, SolveState* st, double* red,
                          hipStream_t s);
hipError_t launch_anorm64(int64_t n, const double* A, int64_t lda, SolveState* st, double* red,
                          hipStream_t s);
// eqr / eqc (may be NULL): the row / column scale factors of an equilibrated
// FP32 factorisation (residual rows scaled by eqr before the correction
// solve, the correction's entries by eqc after it)
hipError_t launch_ir_residual2(int64_t n, const double* b, const double* Ax, const double* x,
                               double* r, float* r32, double* r64, SolveState* st, int force,
                               hipStream_t s, const float* eqr = nullptr);
hipError_t launch_ir_update32(int64_t n, double* x, const float* d, double tol, int32_t first,
                              SolveState* st, hipStream_t s, const float* eqc = nullptr);
hipError_t launch_convert_f32(int64_t n, const double* a, float* b, hipStream_t s,
                              const float* scale = nullptr);
// A <- D_r A D_c in place (FP32, powers of two, the largest entry of every row
// and column then in [1, 2)); dr [n], dc [n] out; rmax [n] scratch.
hipError_t launch_equilibrate(int64_t n, float* A, int64_t lda, float* dr, float* dc,
                              uint32_t* rmax, hipStream_t s);
// a solve's status record and its two synchronisation-word arrays in one launch
hipError_t launch_solve_begin(SolveState* st, int32_t method, int32_t* a, int64_t na, int32_t* b,
                              int64_t nb, hipStream_t s);
// the end of an RK stage: report, body rates, and (Y != NULL) Ys = Y + a K
hipError_t launch_stage_end(SolveState* total, const SolveState* stage, int32_t M, int64_t N,
                            double* Ys, const double* sol, double* K, const double* Y, double a,
                            hipStream_t s);

// time stepping
hipError_t launch_rk_stage_state(int32_t M, const double* Y, const double* K, double a,
                                 double* Ys, hipStream_t s);
hipError_t launch_rk_combine(int32_t M, double* Y, const double* K1, const double* K2,
                             const double* K3, const double* K4, double dt, hipStream_t s);
// Y + h sum_j c[j] K[j] (j < count <= 7), passed by value to the kernels
struct RkComb {
  const double* K[7];
  double c[7];
  int32_t count;
};
hipError_t launch_rk_lincomb(int64_t n, const double* Y, const RkComb& cb, double h, double* out,
                             hipStream_t s);
// out[0] = || h sum_j c[j] K[j] / (atol + rtol max(|Y|, |Yn|)) ||_rms
hipError_t launch_dp_error(int64_t n, const double* Y, const double* Yn, const RkComb& cb, double h,
                           double rtol, double atol, double* out, hipStream_t s);

// flow at field points and tracers

// Field points in blocks of 64 (one per lane), sources cut into `chunks`
// ranges of `chunk` records; partial sums need chunks * 3P doubles.
// cap >= chunks never decreases with Q, so a buffer of cap * 3P doubles
// planned for some Q serves every smaller Q.
struct FieldPlan {
  int64_t pblocks, chunk;
  int32_t chunks, cap;
};
FieldPlan field_plan(int64_t P, int64_t Q);
hipError_t launch_field_sources(int64_t N, int64_t Q, const double* X, const double* w,
                                const int32_t* nu, const double* f, FieldSrc* src, hipStream_t s,
                                const int32_t* stop = nullptr);
// chunk partial sums part[chunk][3][P] of the flow at y + c K (unscaled)
hipError_t launch_field_part(const FieldPlan& fp, int64_t P, int64_t Q, const double* y,
                             const double* K, double c, const FieldSrc* src, double eps,
                             double* part, hipStream_t s, const int32_t* stop);
// u [3][P] = flow of the sources at y + c K (K may be NULL: at y)
hipError_t launch_field(const FieldPlan& fp, int64_t P, int64_t Q, const double* y,
                        const double* K, double c, const FieldSrc* src, double eps, double mu,
                        double* part, double* u, hipStream_t s);
hipError_t launch_tracer_combine(int64_t P, double* y, const double* K1, const double* K2,
                                 const double* K3, const double* K4, double dt, hipStream_t s);

}  // namespace nrs
