// The exported C ABI (include/nrs.h): argument validation, workspace layout
// and the host-side sequencing of the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "nrs_internal.h"

using namespace nrs;

namespace {

nrs_status fail(nrs_ctx* ctx, nrs_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

#define NRS_HIP(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, NRS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

nrs_status use_device(nrs_ctx* ctx) {
  if (!ctx) return NRS_E_ARG;
  NRS_HIP(ctx, hipSetDevice(ctx->device));
  return NRS_OK;
}

// chunk partial sums the matrix-free product may need: it runs the field
// pair sum at the N force points
int32_t apply_chunks(int64_t N, int64_t Q) { return field_plan(N, Q).cap; }

bool uses_fp32(int32_t method) {
  return method == NRS_FP32_IR || method == NRS_FP32_GEPP_IR || method == NRS_FP32_GMRES_IR ||
         method == NRS_BF16_GMRES_IR;
}
// the GMRES-IR forms (flexible GMRES straight after the tile LU)
bool gmres_ir(int32_t method) { return method == NRS_FP32_GMRES_IR || method == NRS_BF16_GMRES_IR; }
// methods whose single-system solves can run the flexible GMRES on the FP32 factors
bool uses_fgmres(int32_t method) { return method == NRS_FP32_IR || gmres_ir(method); }
// methods that iterate from an initial guess (x_init, warm starts)
bool krylov_warm(int32_t method) { return method == NRS_GMRES || method == NRS_GMRES_BLOCK; }
constexpr double kFgmresTol = 1e-12;

// Bytes of the caller workspace of nrs_lu_factor / nrs_lu_solve.
size_t lu_factor_ws_bytes(int64_t n, int32_t precision) {
  size_t b = (size_t)lu_factor_sync_ints(n) * sizeof(int32_t);
  if (precision == 16) b += (size_t)lu_shadow_elems(n) * sizeof(uint16_t);
  else b += gepp_scratch_bytes(n);
  return b + 256;
}
size_t lu_solve_ws_bytes(int64_t n) {
  return (size_t)(kLuHeadInts + round_up(trsv_sync_ints(n), 64)) * sizeof(int32_t) + 256;
}
int32_t* align256(void* p) {
  return reinterpret_cast<int32_t*>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255));
}

}  // namespace

// Scratch of nrs_lu_solve_noalloc: the head words and the triangular-solve
// words of one solve of order up to NRS_NOALLOC_MAX_N (the layout of
// kLuHeadInts + trsv_sync_ints(n)).  Each GPU holds one copy for the life of
// the process.  Host code never uses this name as an address: it uses the
// per-device address from hipGetSymbolAddress (nrs_ctx::scratch).
constexpr int64_t kNoAllocInts =
    kLuHeadInts +
    (2 + (NRS_NOALLOC_MAX_N + 63) / 64 + 2 + 2 * (int64_t)NRS_NOALLOC_MAX_N + 63) / 64 * 64;
static __device__ __align__(256) int32_t scratch[kNoAllocInts];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_at[kMaxScratchDevices] = {};

// Device address of the scratch array on ctx's device (current), looked up
// once per device.
nrs_status setup_scratch(nrs_ctx* ctx) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (ctx->device < 0 || ctx->device >= kMaxScratchDevices)
    return fail(ctx, NRS_E_UNSUPPORTED, "device index too large");
  if (!g_scratch_at[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ctx, NRS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_at[ctx->device] = static_cast<int32_t*>(p);
  }
  ctx->scratch = g_scratch_at[ctx->device];
  return NRS_OK;
}

}  // namespace

// The context's zeroed device flag words (allocated on first use).
nrs_status ctx_dev_flags(nrs_ctx* ctx) {
  if (ctx->dflags) return NRS_OK;
  NRS_HIP(ctx, hipMalloc(&ctx->dflags, 16 * sizeof(int32_t)));
  NRS_HIP(ctx, hipMemset(ctx->dflags, 0, 16 * sizeof(int32_t)));
  return NRS_OK;
}

namespace {

nrs_status check_problem(nrs_ctx* ctx, const nrs_problem* pb) {
  if (!pb) return fail(ctx, NRS_E_ARG, "problem is NULL");
  if (pb->N <= 0 || pb->Q <= 0 || pb->M < 0) return fail(ctx, NRS_E_ARG, "need N > 0, Q > 0, M >= 0");
  if (pb->N > (int64_t)1 << 20 || pb->Q > (int64_t)1 << 30 || pb->M > (1 << 16))
    return fail(ctx, NRS_E_UNSUPPORTED, "N, Q or M too large");
  if (!pb->x || !pb->X || !pb->nu || !pb->body) return fail(ctx, NRS_E_ARG, "x, X, nu, body required");
  if (pb->M > 0 && !pb->Y) return fail(ctx, NRS_E_ARG, "Y required when M > 0");
  if (3 * pb->N + 6 * (int64_t)pb->M > 262144)
    return fail(ctx, NRS_E_UNSUPPORTED, "more than 262144 unknowns");
  if (!(pb->eps > 0.0) || !(pb->mu > 0.0) || !std::isfinite(pb->eps) || !std::isfinite(pb->mu))
    return fail(ctx, NRS_E_ARG, "eps and mu must be positive and finite");
  return NRS_OK;
}

}  // namespace

namespace nrs {

// Workspace layout: [SolveState][Sorted][A32?][A64][vectors][apply partials]
bool carve_solve(Arena& ar, int64_t N, int64_t Q, int32_t M, int32_t method, SolveBuffers& sb,
                 bool with64) {
  const int64_t n = 3 * N + 6 * (int64_t)M;
  sb.st = ar.take<SolveState>(1);
  sb.srt.seg = ar.take<int32_t>(N + 1);
  sb.srt.cnt = ar.take<int32_t>(N + 2);
  sb.srt.perm = ar.take<int32_t>(Q);
  sb.srt.nus = ar.take<int32_t>(Q);
  sb.srt.X64 = ar.take<double4>(Q);
  sb.srt.X32hi = ar.take<float4>(Q);
  sb.srt.X32lo = ar.take<float4>(Q);
  sb.srt.W = ar.take<double>(N);
  sb.srt.fsrc = ar.take<FieldSrc>(Q);
  sb.lda = lda_for(n);
  sb.A32 = uses_fp32(method) ? ar.take<float>((size_t)sb.lda * n) : nullptr;
  sb.A64 = with64 ? ar.take<double>((size_t)sb.lda * n) : nullptr;
  sb.ipiv = ar.take<int32_t>(n);
  sb.perm = ar.take<int32_t>(n);
  sb.ipiv64 = ar.take<int32_t>(n);
  sb.perm64 = ar.take<int32_t>(n);
  sb.b = ar.take<double>(n);
  sb.x = ar.take<double>(n);
  sb.r = ar.take<double>(n);
  sb.d64 = ar.take<double>(n);
  sb.d32 = ar.take<float>(n);
  sb.chunks = apply_chunks(N, Q);
  sb.part = ar.take<double>((size_t)sb.chunks * 3 * N);
  sb.red = ar.take<double>(rowsum_scratch(n));
  sb.tsync = ar.take<int32_t>(trsv_sync_ints(n));
  sb.gepp = ar.take<char>(gepp_scratch_bytes(n));
  const bool f32 = uses_fp32(method);
  sb.eqr = f32 ? ar.take<float>(n) : nullptr;
  sb.eqc = f32 ? ar.take<float>(n) : nullptr;
  sb.eqmax = f32 ? ar.take<uint32_t>(n) : nullptr;
  sb.equil = false;
  sb.lu_done = ar.take<int32_t>(with64 ? lu_done_ints(n) : lu_done_flag_ints(n));
  sb.AT = sb.V = sb.gw0 = sb.gw1 = sb.gpart = nullptr;
  sb.gst = nullptr;
  sb.Z = sb.fzv = sb.fax = nullptr;
  sb.sh = (with64 && method == NRS_BF16_GMRES_IR) ? ar.take<uint16_t>(lu_shadow_elems(n)) : nullptr;
  const bool blk = method == NRS_GMRES_BLOCK;
  sb.boff = blk ? ar.take<int32_t>((size_t)M + 1) : nullptr;
  sb.bstarts = blk ? ar.take<int32_t>(1) : nullptr;
  sb.bpsi = blk ? ar.take<double>((size_t)M + 1) : nullptr;
  sb.blocks = blk ? ar.take<double>((size_t)M * kBlockStride) : nullptr;
  sb.phase_scene = nullptr;
  sb.phase_t = 0.0;
  const bool fg = (with64 && uses_fgmres(method)) || blk;
  if (fg) {
    sb.Z = ar.take<double>((size_t)n * kGmresLd);
    sb.fzv = ar.take<double>(n);
    sb.fax = ar.take<double>(n);
  }
  if (method == NRS_GMRES || fg) {
    if (method == NRS_GMRES) sb.AT = ar.take<double>((size_t)sb.lda * n);
    sb.V = ar.take<double>((size_t)n * kGmresLd);
    sb.gw0 = ar.take<double>(n);
    sb.gw1 = ar.take<double>(n);
    sb.gpart = ar.take<double>((size_t)gmres_blocks(n) * kGmresLd);
    sb.gst = ar.take<GmresState>(1);
  }
  return !ar.overflow;
}

size_t solve_workspace_bytes(int64_t N, int64_t Q, int32_t M, int32_t method) {
  Arena ar(nullptr, 0);
  SolveBuffers sb;
  carve_solve(ar, N, Q, M, method, sb);
  return ar.used + 256;
}

}  // namespace nrs

namespace {

// FP64 LU path: assemble, factor with partial pivoting, solve into x.
nrs_status run_fp64_lu(nrs_ctx* ctx, const nrs_problem& pb, SolveBuffers& sb, double* x,
                       bool norm, hipStream_t s) {
  const int64_t n = 3 * pb.N + 6 * (int64_t)pb.M;
  NRS_HIP(ctx, launch_assemble<double>(pb, sb.srt, sb.A64, sb.lda, s,
                                       asm_shape_for(ctx, pb.N, pb.Q, 64)));
  if (norm) NRS_HIP(ctx, launch_anorm64(n, sb.A64, sb.lda, sb.st, sb.red, s));
  NRS_HIP(ctx, lu_factor_any<double>(n, 0, sb.A64, sb.lda, sb.ipiv64, sb.perm64,
                                      &sb.st->singular, sb.lu_done, sb.st->lu_ctl, s, nullptr,
                                      sb.gepp));
  NRS_HIP(ctx, launch_lu_solve<double>(n, 0, sb.A64, sb.lda, sb.perm64, sb.b, x, sb.tsync,
                                       &sb.st->sync_err, nullptr, s));
  return NRS_OK;
}

// FP32 factors + FP64 refinement.  Correction solves use the FP32 factors;
// residuals use the matrix-free FP64 operator.
nrs_status run_fp32_ir(nrs_ctx* ctx, const nrs_problem& pb, SolveBuffers& sb, double* x,
                       int32_t scope, int32_t max_refine, double tol, bool norm, bool equil,
                       hipStream_t s, bool b32_ready = false) {
  const int64_t n = 3 * pb.N + 6 * (int64_t)pb.M;
  NRS_HIP(ctx, launch_assemble<float>(pb, sb.srt, sb.A32, sb.lda, s,
                                      asm_shape_for(ctx, pb.N, pb.Q, 32)));
  if (norm) NRS_HIP(ctx, launch_anorm32(n, sb.A32, sb.lda, sb.st, sb.red, s));
  sb.equil = equil;
  if (equil) NRS_HIP(ctx, launch_equilibrate(n, sb.A32, sb.lda, sb.eqr, sb.eqc, sb.eqmax, s));
  const float* er = equil ? sb.eqr : nullptr;
  const float* ec = equil ? sb.eqc : nullptr;
  NRS_HIP(ctx, lu_factor_any<float>(n, scope, sb.A32, sb.lda, sb.ipiv, sb.perm,
                                     &sb.st->singular, sb.lu_done, sb.st->lu_ctl, s,
                                     scope == 1 ? sb.sh : nullptr, sb.gepp));
  // x0 = D_c (LU)^-1 D_r b (b32_ready: the right-hand side kernel wrote the
  // unscaled FP32 copy already)
  float* b32 = reinterpret_cast<float*>(sb.r);  // r is free until the first residual
  if (!b32_ready || equil) NRS_HIP(ctx, launch_convert_f32(n, sb.b, b32, s, er));
  NRS_HIP(ctx, launch_lu_solve<float>(n, scope, sb.A32, sb.lda, sb.perm, b32, sb.d32, sb.tsync,
                                      &sb.st->sync_err, &sb.st->stop, s));
  NRS_HIP(ctx, launch_ir_update32(n, x, sb.d32, tol, 1, sb.st, s, ec));
  for (int it = 0; it < max_refine; ++it) {
    NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.d64, sb.part, sb.chunks, &sb.st->stop, s));
    NRS_HIP(ctx, launch_ir_residual2(n, sb.b, sb.d64, x, nullptr, b32, nullptr, sb.st, 0, s, er));
    NRS_HIP(ctx, launch_lu_solve<float>(n, scope, sb.A32, sb.lda, sb.perm, b32, sb.d32,
                                        sb.tsync, &sb.st->sync_err, &sb.st->stop, s));
    NRS_HIP(ctx, launch_ir_update32(n, x, sb.d32, tol, 0, sb.st, s, ec));
  }
  return NRS_OK;
}

// Refinement against factors already in sb.A32 / sb.perm (the tile LU of an
// earlier, nearby system): x0 from them, then FP64 matrix-free residuals of
// this system and correction sweeps; queued sweeps after convergence skip.
nrs_status run_fp32_reuse(nrs_ctx* ctx, const nrs_problem& pb, SolveBuffers& sb, double* x,
                          int32_t max_refine, double tol, hipStream_t s, bool b32_ready = false) {
  const int64_t n = 3 * pb.N + 6 * (int64_t)pb.M;
  // the factors (and their scale factors, if equilibrated) of the earlier system
  const float* er = sb.equil ? sb.eqr : nullptr;
  const float* ec = sb.equil ? sb.eqc : nullptr;
  float* b32 = reinterpret_cast<float*>(sb.r);
  if (!b32_ready || sb.equil) NRS_HIP(ctx, launch_convert_f32(n, sb.b, b32, s, er));
  NRS_HIP(ctx, launch_lu_solve<float>(n, 1, sb.A32, sb.lda, sb.perm, b32, sb.d32, sb.tsync,
                                      &sb.st->sync_err, &sb.st->stop, s));
  NRS_HIP(ctx, launch_ir_update32(n, x, sb.d32, tol, 1, sb.st, s, ec));
  for (int it = 0; it < max_refine; ++it) {
    NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.d64, sb.part, sb.chunks, &sb.st->stop, s));
    NRS_HIP(ctx, launch_ir_residual2(n, sb.b, sb.d64, x, nullptr, b32, nullptr, sb.st, 0, s, er));
    NRS_HIP(ctx, launch_lu_solve<float>(n, 1, sb.A32, sb.lda, sb.perm, b32, sb.d32, sb.tsync,
                                        &sb.st->sync_err, &sb.st->stop, s));
    NRS_HIP(ctx, launch_ir_update32(n, x, sb.d32, tol, 0, sb.st, s, ec));
  }
  return NRS_OK;
}

// FP64 GMRES on the stored FP64 matrix from x's initial content (x_init
// copied in by the caller, else zero).  Synchronises once per chunk of
// Arnoldi steps to decide whether to queue more.
nrs_status run_gmres(nrs_ctx* ctx, const nrs_problem& pb, SolveBuffers& sb, double* x,
                     const nrs_options& o, bool norm, hipStream_t s) {
  const int64_t n = 3 * pb.N + 6 * (int64_t)pb.M;
  const int32_t m = o.gmres_restart > 0 ? o.gmres_restart : 50;
  const int32_t max_iter = o.gmres_max_iter > 0 ? o.gmres_max_iter : 1000;
  const double tol = o.tol > 0 ? o.tol : 1e-11;
  NRS_HIP(ctx, launch_assemble<double>(pb, sb.srt, sb.A64, sb.lda, s,
                                       asm_shape_for(ctx, pb.N, pb.Q, 64)));
  if (norm) NRS_HIP(ctx, launch_anorm64(n, sb.A64, sb.lda, sb.st, sb.red, s));
  NRS_HIP(ctx, launch_transpose64(n, sb.A64, sb.lda, sb.AT, sb.lda, s));
  if (o.x_init && o.x_init != x)
    NRS_HIP(ctx, hipMemcpyAsync(x, o.x_init, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  else if (!o.x_init)
    NRS_HIP(ctx, launch_fill_f64(x, 0.0, n, s));
  if (o.x_init && o.x_init_complete && pb.M > 0)
    NRS_HIP(ctx, launch_rigid_completion(pb.N, pb.M, pb.x, pb.Y, pb.body, sb.srt.W, sb.b + 3 * pb.N,
                                         sb.AT, sb.lda, sb.b, x, sb.gw1, sb.gpart, s));
  GmresArgs a;
  a.n = n;
  a.ld = sb.lda;
  a.AT = sb.AT;
  a.b = sb.b;
  a.x = x;
  a.V = sb.V;
  a.w0 = sb.gw0;
  a.w1 = sb.gw1;
  a.part = sb.gpart;
  a.st = sb.gst;
  NRS_HIP(ctx, launch_gmres_init(sb.gst, tol, m, max_iter, s));
  NRS_HIP(ctx, launch_gmres_residual(a, s));
  struct Hdr {
    int32_t done, stop, fail, k, iters;
  } h;
  constexpr int kChunk = 8;
  for (;;) {
    NRS_HIP(ctx, launch_gmres_steps(a, kChunk, s));
    NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
    NRS_HIP(ctx, hipStreamSynchronize(s));
    if (h.fail || h.done) break;
    if (!h.stop) continue;
    NRS_HIP(ctx, launch_gmres_update(a, s));
    NRS_HIP(ctx, launch_gmres_residual(a, s));
    NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
    NRS_HIP(ctx, hipStreamSynchronize(s));
    if (h.fail || h.done || h.iters >= max_iter) break;
  }
  NRS_HIP(ctx, launch_gmres_report(sb.st, sb.gst, s));
  return NRS_OK;
}

// Flexible GMRES(m) in FP64 from the iterate in x (GMRES-IR): the operator is
// the matrix-free FP64 product, the right preconditioner the FP32 tile-LU
// factors in sb.A32 (two triangular passes per step).  Queues kChunk steps
// between host checks; every launch queued behind a finished cycle skips
// (the state's halt word).  Reports into sb.st (iterations are added).
nrs_status run_fgmres(nrs_ctx* ctx, const nrs_problem& pb, SolveBuffers& sb, double* x,
                      const nrs_options& o, hipStream_t s) {
  const int64_t n = 3 * pb.N + 6 * (int64_t)pb.M;
  const int32_t m = (o.gmres_restart > 0 && o.gmres_restart < kGmresLd) ? o.gmres_restart : 60;
  const int32_t max_iter = o.gmres_max_iter > 0 ? o.gmres_max_iter : 300;
  const double tol = (gmres_ir(o.method) && o.tol > 0) ? o.tol : kFgmresTol;
  float* v32 = reinterpret_cast<float*>(sb.r);
  GmresArgs a;
  a.n = n;
  a.ld = kGmresLd;
  a.AT = nullptr;
  a.b = sb.b;
  a.x = x;
  a.V = sb.V;
  a.Z = sb.Z;
  a.w0 = sb.gw0;
  a.w1 = sb.gw1;
  a.part = sb.gpart;
  a.st = sb.gst;
  if (sb.equil) {
    a.eqr = sb.eqr;
    a.eqc = sb.eqc;
  }
  const int32_t* halt = &sb.gst->halt;
  NRS_HIP(ctx, launch_gmres_init(sb.gst, tol, m, max_iter, s));
  NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.fax, sb.part, sb.chunks, nullptr, s));
  NRS_HIP(ctx, launch_fgmres_residual(a, sb.fax, s));
  struct Hdr {
    int32_t done, stop, fail, k, iters;
  } h;
  constexpr int kChunk = 4;
  for (;;) {
    for (int i = 0; i < kChunk; ++i) {
      NRS_HIP(ctx, launch_fgmres_begin(a, v32, s));
      NRS_HIP(ctx, launch_lu_solve<float>(n, 1, sb.A32, sb.lda, sb.perm, v32, sb.d32, sb.tsync,
                                          &sb.st->sync_err, halt, s));
      NRS_HIP(ctx, launch_fgmres_zstore(a, sb.d32, sb.fzv, s));
      NRS_HIP(ctx, launch_apply(pb, sb.srt, sb.fzv, sb.d64, sb.part, sb.chunks, halt, s));
      NRS_HIP(ctx, launch_fgmres_orth(a, sb.d64, s));
    }
    NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
    NRS_HIP(ctx, hipStreamSynchronize(s));
    if (h.fail || h.done) break;
    if (!h.stop) continue;
    NRS_HIP(ctx, launch_gmres_update(a, s));
    NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.fax, sb.part, sb.chunks, nullptr, s));
    NRS_HIP(ctx, launch_fgmres_residual(a, sb.fax, s));
    NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
    NRS_HIP(ctx, hipStreamSynchronize(s));
    if (h.fail || h.done || h.iters >= max_iter) break;
  }
  NRS_HIP(ctx, launch_fgmres_report(sb.st, sb.gst, s));
  return NRS_OK;
}

// Flexible GMRES(m) in FP64 on the matrix-free operator from x's initial
// content (x_init, else zero), right-preconditioned by one dense block per
// free body: the inverses of the bodies' diagonal blocks of the assembled
// FP64 matrix (NRS_PRECOND_EXACT) or the learned model's blocks at the
// bodies' phases (NRS_PRECOND_MODEL, psi: [M] device).  Host checks every
// kChunk steps as in run_fgmres.
nrs_status run_gmres_block(nrs_ctx* ctx, const nrs_problem& pb, SolveBuffers& sb, double* x,
                           const nrs_options& o, const double* psi, bool norm, hipStream_t s) {
  const int64_t N = pb.N, n = 3 * N + 6 * (int64_t)pb.M;
  const int32_t M = pb.M;
  const int32_t m = (o.gmres_restart > 0 && o.gmres_restart < kGmresLd) ? o.gmres_restart : 60;
  const int32_t max_iter = o.gmres_max_iter > 0 ? o.gmres_max_iter : 300;
  const double tol = o.tol > 0 ? o.tol : kFgmresTol;
  const bool model = o.precond == NRS_PRECOND_MODEL;
  const int32_t lim = ctx->block_lim;
  if (o.x_init && o.x_init != x)
    NRS_HIP(ctx, hipMemcpyAsync(x, o.x_init, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  else if (!o.x_init)
    NRS_HIP(ctx, launch_fill_f64(x, 0.0, n, s));
  if (M > 0) {
    NRS_HIP(ctx, launch_body_off(N, M, pb.body, sb.boff, sb.bstarts, &sb.st->prec_err, s));
    NRS_HIP(ctx, launch_block_check(M, N, sb.boff, lim, model ? o.precond_nb : 0,
                                    &sb.st->prec_err, s));
  }
  if (model && sb.phase_scene && M > 0) {
    NRS_HIP(ctx, launch_body_phase(M, N, sb.boff, sb.phase_scene->part, sb.phase_scene->wave,
                                   sb.phase_scene->P, sb.phase_t, sb.bpsi, s));
    psi = sb.bpsi;
  }
  if (model) {
    NRS_HIP(ctx, launch_block_model(M, N, sb.boff, lim, o.precond_nb, o.precond_harmonics,
                                    o.precond_model, psi, kBlockStride, sb.blocks, s));
  } else {
    NRS_HIP(ctx, launch_assemble<double>(pb, sb.srt, sb.A64, sb.lda, s,
                                         asm_shape_for(ctx, pb.N, pb.Q, 64)));
    if (norm) NRS_HIP(ctx, launch_anorm64(n, sb.A64, sb.lda, sb.st, sb.red, s));
    NRS_HIP(ctx, launch_block_extract(M, N, sb.boff, lim, sb.A64, sb.lda, sb.blocks, s));
    NRS_HIP(ctx, launch_block_inverse(M, 0, kBlockStride, N, sb.boff, lim, sb.blocks,
                                      &sb.st->singular, s));
  }
  GmresArgs a;
  a.n = n;
  a.ld = kGmresLd;
  a.AT = nullptr;
  a.b = sb.b;
  a.x = x;
  a.V = sb.V;
  a.Z = sb.Z;
  a.w0 = sb.gw0;
  a.w1 = sb.gw1;
  a.part = sb.gpart;
  a.st = sb.gst;
  const int32_t* halt = &sb.gst->halt;
  const double* Yrot = model ? pb.Y : nullptr;
  const int32_t nbm = model ? o.precond_nb : 0;
  NRS_HIP(ctx, launch_gmres_init(sb.gst, tol, m, max_iter, s));
  NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.fax, sb.part, sb.chunks, nullptr, s));
  struct Hdr {
    int32_t done, stop, fail, k, iters;
  } h;
  if (n <= kGmresSmallN) {
    // one workgroup per Arnoldi step; the end of a cycle (update, true
    // residual, restart) is queued behind every batch of steps and skips
    // unless the cycle stopped, so a solve that converges within its first
    // batch synchronises with the host once.  The batch length follows the
    // previous solve's iteration count.
    NRS_HIP(ctx, launch_bg_residual(a, sb.fax, false, sb.fzv, s));
    int32_t chunk = std::min(16, std::max(2, ctx->bg_chunk));
    for (;;) {
      for (int i = 0; i < chunk; ++i) {
        NRS_HIP(ctx, launch_prec_block(a, M, N, sb.boff, lim, nbm, Yrot, sb.blocks, sb.fzv, false,
                                       s));
        NRS_HIP(ctx, launch_apply(pb, sb.srt, sb.fzv, sb.d64, sb.part, sb.chunks, halt, s));
        NRS_HIP(ctx, launch_bg_orth(a, sb.d64, sb.fzv, s));
      }
      NRS_HIP(ctx, launch_bg_update(a, s));
      NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.fax, sb.part, sb.chunks, &sb.gst->skip_true, s));
      NRS_HIP(ctx, launch_bg_residual(a, sb.fax, true, sb.fzv, s));
      NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
      NRS_HIP(ctx, hipStreamSynchronize(s));
      if (h.fail || h.done || h.iters >= max_iter) break;
      chunk = 4;
    }
    ctx->bg_chunk = h.iters + 1;
    NRS_HIP(ctx, launch_fgmres_report(sb.st, sb.gst, s));
    return NRS_OK;
  }
  NRS_HIP(ctx, launch_fgmres_residual(a, sb.fax, s));
  constexpr int kChunk = 4;
  for (;;) {
    for (int i = 0; i < kChunk; ++i) {
      NRS_HIP(ctx, launch_prec_block(a, M, N, sb.boff, lim, nbm, Yrot, sb.blocks, sb.fzv, true, s));
      NRS_HIP(ctx, launch_apply(pb, sb.srt, sb.fzv, sb.d64, sb.part, sb.chunks, halt, s));
      NRS_HIP(ctx, launch_fgmres_orth(a, sb.d64, s));
    }
    NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
    NRS_HIP(ctx, hipStreamSynchronize(s));
    if (h.fail || h.done) break;
    if (!h.stop) continue;
    NRS_HIP(ctx, launch_gmres_update(a, s));
    NRS_HIP(ctx, launch_apply(pb, sb.srt, x, sb.fax, sb.part, sb.chunks, nullptr, s));
    NRS_HIP(ctx, launch_fgmres_residual(a, sb.fax, s));
    NRS_HIP(ctx, hipMemcpyAsync(&h, sb.gst, sizeof(h), hipMemcpyDeviceToHost, s));
    NRS_HIP(ctx, hipStreamSynchronize(s));
    if (h.fail || h.done || h.iters >= max_iter) break;
  }
  NRS_HIP(ctx, launch_fgmres_report(sb.st, sb.gst, s));
  return NRS_OK;
}

// Options of NRS_GMRES_BLOCK; need_phase: the caller supplies precond_phase.
nrs_status check_block_options(nrs_ctx* ctx, const nrs_options& o, int32_t M, bool need_phase) {
  if (o.method != NRS_GMRES_BLOCK) return NRS_OK;
  if (o.precond != NRS_PRECOND_EXACT && o.precond != NRS_PRECOND_MODEL)
    return fail(ctx, NRS_E_ARG, "precond must be NRS_PRECOND_EXACT or NRS_PRECOND_MODEL");
  if (o.precond == NRS_PRECOND_MODEL) {
    if (!o.precond_model) return fail(ctx, NRS_E_ARG, "precond_model required");
    if (o.precond_harmonics < 0 || o.precond_harmonics > kBlockHarmonicsMax)
      return fail(ctx, NRS_E_ARG, "precond_harmonics outside 0..NRS_BLOCK_MAX_HARMONICS");
    if (o.precond_nb < 9 || (o.precond_nb - 6) % 3 != 0)
      return fail(ctx, NRS_E_ARG, "precond_nb must be 3 N_b + 6 with N_b >= 1");
    if (o.precond_nb > ctx->block_lim)
      return fail(ctx, NRS_E_UNSUPPORTED, "precond_nb exceeds nrs_block_limit()");
    if (need_phase && M > 0 && !o.precond_phase)
      return fail(ctx, NRS_E_ARG, "precond_phase required");
  }
  return NRS_OK;
}

nrs_status read_state(nrs_ctx* ctx, const SolveState* dst, SolveState& hst) {
  NRS_HIP(ctx, hipMemcpyAsync(&hst, dst, sizeof(SolveState), hipMemcpyDeviceToHost, ctx->stream));
  NRS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return NRS_OK;
}

void fill_info(const SolveState& h, nrs_info* info) {
  info->method_used = h.method_used;
  info->fell_back = h.fell_back;
  info->iterations = h.iterations;
  info->singular = h.singular;
  info->backward_error = h.bwd;
  info->correction = h.corr;
}

// Core of nrs_solve on already-carved buffers.  When `sync` is set the
// state is read back and the FP64 fallback may run.
nrs_status solve_core(nrs_ctx* ctx, const nrs_problem& pb, const double* u, const double* ftext,
                      const nrs_options& o, SolveBuffers& sb, double* sol, bool sync,
                      SolveState* hst_out, bool reuse = false) {
  hipStream_t s = ctx->stream;
  const int64_t N = pb.N, Q = pb.Q, n = 3 * N + 6 * (int64_t)pb.M;
  const int32_t method = o.method;
  const int32_t max_refine = o.max_refine > 0 ? o.max_refine : 4;
  const double tol = o.tol > 0 ? o.tol : 1e-9;
  // the status record and (factorisation paths) the synchronisation words
  const bool fact = method != NRS_GMRES_BLOCK;
  NRS_HIP(ctx, launch_solve_begin(sb.st, method, fact ? sb.tsync : nullptr,
                                  fact ? trsv_sync_ints(n) : 0, fact ? sb.lu_done : nullptr,
                                  fact ? lu_done_flag_ints(n) : 0, s));
  NRS_HIP(ctx, launch_build_csr(N, Q, pb.X, pb.w, pb.nu, sb.srt, sb.st, s));
  // the right-hand side with the body check; the FP32 forms that factor the
  // unscaled matrix also get its FP32 copy here
  const bool b32_ready =
      uses_fp32(method) &&
      !(reuse ? sb.equil : (method != NRS_FP32_GEPP_IR && o.equilibrate != 0));
  NRS_HIP(ctx, launch_rhs(N, pb.M, u, ftext, sb.b, s,
                          b32_ready ? reinterpret_cast<float*>(sb.r) : nullptr, pb.body, sb.st));
  nrs_status st = NRS_OK;
  if (reuse) {
    st = run_fp32_reuse(ctx, pb, sb, sol, o.max_refine > 0 ? o.max_refine : 12, tol, s, b32_ready);
  } else if (method == NRS_FP64_LU) {
    st = run_fp64_lu(ctx, pb, sb, sol, sync, s);
  } else if (uses_fp32(method)) {
    const bool fgm = gmres_ir(method);
    // equilibration serves the static block pivots of the tile LU; the fully
    // pivoted form factors A itself
    const bool gepp = method == NRS_FP32_GEPP_IR;
    st = run_fp32_ir(ctx, pb, sb, sol, gepp ? 0 : 1, fgm ? 0 : max_refine, tol, sync,
                     !gepp && o.equilibrate != 0, s, b32_ready);
    if (st == NRS_OK && fgm) st = run_fgmres(ctx, pb, sb, sol, o, s);
  } else if (method == NRS_GMRES) {
    st = run_gmres(ctx, pb, sb, sol, o, sync, s);
  } else if (method == NRS_GMRES_BLOCK) {
    st = run_gmres_block(ctx, pb, sb, sol, o, o.precond_phase, sync, s);
  } else {
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  }
  if (st != NRS_OK) return st;
  if (!sync) return NRS_OK;
  SolveState h;
  if ((st = read_state(ctx, sb.st, h)) != NRS_OK) return st;
  if (h.nonfinite == 2)
    return fail(ctx, NRS_E_ARG, "nu outside [0, N) or body outside [-1, M)");
  const int32_t prec_err = method == NRS_GMRES_BLOCK ? h.prec_err : 0;
  bool ok = method == NRS_FP64_LU ? true : (h.converged && !h.failed);
  if (!ok && method == NRS_FP32_IR && sb.Z && !h.nonfinite && !h.sync_err && !h.lu_ctl[2]) {
    // the refinement stalled: GMRES-IR from its iterate on the same factors
    if ((st = run_fgmres(ctx, pb, sb, sol, o, s)) != NRS_OK) return st;
    if ((st = read_state(ctx, sb.st, h)) != NRS_OK) return st;
    ok = h.converged && !h.failed;
  }
  if (!ok && !o.no_fallback) {
    NRS_HIP(ctx, launch_state_init(sb.st, NRS_FP64_LU, s));
    if (method == NRS_GMRES_BLOCK) {
      NRS_HIP(ctx, launch_fill_i32(sb.tsync, 0, trsv_sync_ints(n), s));
      NRS_HIP(ctx, launch_fill_i32(sb.lu_done, 0, lu_done_flag_ints(n), s));
    }
    if ((st = run_fp64_lu(ctx, pb, sb, sol, true, s)) != NRS_OK) return st;
    if ((st = read_state(ctx, sb.st, h)) != NRS_OK) return st;
    h.fell_back = 1;
    ok = true;
  }
  // final backward error of the returned solution (FP64 operator)
  NRS_HIP(ctx, launch_apply(pb, sb.srt, sol, sb.d64, sb.part, sb.chunks, nullptr, s));
  NRS_HIP(ctx, launch_ir_residual2(n, sb.b, sb.d64, sol, sb.r, nullptr, nullptr, sb.st, 1, s));
  SolveState h2;
  if ((st = read_state(ctx, sb.st, h2)) != NRS_OK) return st;
  h.bwd = h2.bwd;
  h.nonfinite |= h2.nonfinite;
  h.sync_err |= h2.sync_err | h.lu_ctl[2] | h2.lu_ctl[2];
  if (hst_out) *hst_out = h;
  if (h.sync_err) return fail(ctx, NRS_E_HIP, "LU / triangular solve: a bounded wait timed out");
  if (h.nonfinite) return fail(ctx, NRS_E_NONFINITE, "non-finite values in the solution");
  if (h.singular && h.method_used == NRS_FP64_LU)
    return fail(ctx, NRS_E_SINGULAR, "zero pivot in the FP64 factorisation");
  if (!ok) return fail(ctx, NRS_E_NOT_CONVERGED, "refinement did not converge");
  if (prec_err)
    return fail(ctx, NRS_E_UNSUPPORTED,
                std::string("block preconditioner: ") +
                    ((prec_err & 2) ? "body points are not one contiguous run per body; " : "") +
                    ((prec_err & 4) ? "a body block exceeds nrs_block_limit(); " : "") +
                    ((prec_err & 8) ? "a body block differs from precond_nb; " : "") +
                    "those bodies were left unpreconditioned");
  return NRS_OK;
}

}  // namespace

extern "C" {

const char* nrs_version(void) { return "nrs 0.1 gfx950"; }

const char* nrs_status_string(nrs_status s) {
  switch (s) {
    case NRS_OK: return "ok";
    case NRS_E_ARG: return "invalid argument";
    case NRS_E_HIP: return "HIP runtime error";
    case NRS_E_WORKSPACE: return "workspace too small";
    case NRS_E_SINGULAR: return "singular matrix";
    case NRS_E_NOT_CONVERGED: return "not converged";
    case NRS_E_NONFINITE: return "non-finite values";
    case NRS_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

nrs_status nrs_create(nrs_ctx** out, int device, void* stream) {
  if (!out) return NRS_E_ARG;
  *out = nullptr;
  nrs_ctx* c = new (std::nothrow) nrs_ctx();
  if (!c) return NRS_E_HIP;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipSetDevice(device) != hipSuccess || setup_scratch(c) != NRS_OK) {
    delete c;
    return NRS_E_HIP;
  }
  *out = c;
  return NRS_OK;
}

nrs_status nrs_destroy(nrs_ctx* ctx) {
  if (ctx) {
    hipSetDevice(ctx->device);
    if (ctx->staging_event) {
      hipEventSynchronize(ctx->staging_event);
      hipEventDestroy(ctx->staging_event);
    }
    if (ctx->staging) hipHostFree(ctx->staging);
    if (ctx->dflags) hipFree(ctx->dflags);
    for (int j = 0; j < nrs_ctx::kAux; ++j) {
      if (ctx->aux[j]) {
        hipStreamSynchronize(ctx->aux[j]);
        hipStreamDestroy(ctx->aux[j]);
      }
      if (ctx->join_ev[j]) hipEventDestroy(ctx->join_ev[j]);
    }
    if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
    if (!ctx->graphs.empty()) {
      if (ctx->stream) hipStreamSynchronize(ctx->stream);
      for (auto& g : ctx->graphs) {
        hipGraphExecDestroy(g.exec);
        hipHostFree(g.host_desc);
      }
    }
  }
  delete ctx;
  return NRS_OK;
}

nrs_status nrs_set_stream(nrs_ctx* ctx, void* stream) {
  if (!ctx) return NRS_E_ARG;
  ctx->stream = static_cast<hipStream_t>(stream);
  return NRS_OK;
}

const char* nrs_last_error(const nrs_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

nrs_status nrs_geometry(nrs_ctx* ctx, const nrs_scene* sc, double t, const double* Y, double* x,
                        double* X, double* w, double* u) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (!sc || sc->N < 0 || sc->Q < 0 || sc->M < 0 || sc->P < 0)
    return fail(ctx, NRS_E_ARG, "bad scene sizes");
  if ((sc->N > 0 && (!sc->xi || !sc->body || !sc->part || !sc->s || !sc->ufix)) ||
      (sc->Q > 0 && (!sc->Xi || !sc->bodyX || !sc->partX || !sc->sX || !sc->w0)))
    return fail(ctx, NRS_E_ARG, "scene arrays missing");
  if (sc->P > 0 && !sc->wave) return fail(ctx, NRS_E_ARG, "wave table missing");
  if (sc->M > 0 && !Y) return fail(ctx, NRS_E_ARG, "Y required when M > 0");
  if (!std::isfinite(t)) return fail(ctx, NRS_E_ARG, "t must be finite");
  NRS_HIP(ctx, launch_geometry(*sc, t, Y, x, X, w, u, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_nearest(nrs_ctx* ctx, int64_t N, const double* x, int32_t G,
                       const int32_t* group_off_host, int64_t Q, const double* X,
                       const int32_t* groupX, int32_t* nu_out) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (N <= 0 || Q < 0 || G <= 0 || !x || !group_off_host || (Q > 0 && (!X || !groupX || !nu_out)))
    return fail(ctx, NRS_E_ARG, "bad nearest-neighbour arguments");
  if (G > kMaxGroups) return fail(ctx, NRS_E_UNSUPPORTED, "too many groups");
  GroupTable gt;
  gt.G = G;
  for (int g = 0; g <= G; ++g) gt.off[g] = group_off_host[g];
  if (gt.off[0] != 0 || gt.off[G] != N) return fail(ctx, NRS_E_ARG, "group_off must span [0, N]");
  for (int g = 0; g < G; ++g)
    if (gt.off[g + 1] <= gt.off[g]) return fail(ctx, NRS_E_ARG, "every group needs a force point");
  NRS_HIP(ctx, launch_nearest(N, x, gt, Q, X, groupX, nu_out, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_workspace_size(nrs_ctx* ctx, int64_t N, int64_t Q, int32_t M, int32_t method,
                              size_t* bytes) {
  if (!bytes || N <= 0 || Q <= 0 || M < 0) return fail(ctx, NRS_E_ARG, "bad sizes");
  if (method < NRS_FP64_LU || method > NRS_GMRES_BLOCK)
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  *bytes = solve_workspace_bytes(N, Q, M, method);
  return NRS_OK;
}

nrs_status nrs_assemble(nrs_ctx* ctx, const nrs_problem* pb, int32_t precision, void* A,
                        int64_t lda, void* ws, size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_problem(ctx, pb))) return st;
  const int64_t n = 3 * pb->N + 6 * (int64_t)pb->M;
  if (!A || lda < n) return fail(ctx, NRS_E_ARG, "A NULL or lda < n");
  if (precision != 32 && precision != 64) return fail(ctx, NRS_E_ARG, "precision must be 32 or 64");
  Arena ar(ws, ws_bytes);
  SolveBuffers sb;
  if (!carve_solve(ar, pb->N, pb->Q, pb->M, precision == 32 ? NRS_FP32_IR : NRS_FP64_LU, sb))
    return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  // no status record: the call reports nothing from the device, and
  // quadrature points whose nu is out of range are left out of the layout
  NRS_HIP(ctx, launch_build_csr(pb->N, pb->Q, pb->X, pb->w, pb->nu, sb.srt, nullptr, s));
  if (precision == 32)
    NRS_HIP(ctx, launch_assemble<float>(*pb, sb.srt, static_cast<float*>(A), lda, s,
                                        asm_shape_for(ctx, pb->N, pb->Q, 32)));
  else
    NRS_HIP(ctx, launch_assemble<double>(*pb, sb.srt, static_cast<double*>(A), lda, s,
                                         asm_shape_for(ctx, pb->N, pb->Q, 64)));
  return NRS_OK;
}

nrs_status nrs_apply(nrs_ctx* ctx, const nrs_problem* pb, const double* v, double* y, void* ws,
                     size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_problem(ctx, pb))) return st;
  if (!v || !y) return fail(ctx, NRS_E_ARG, "v and y required");
  Arena ar(ws, ws_bytes);
  SolveBuffers sb;
  if (!carve_solve(ar, pb->N, pb->Q, pb->M, NRS_FP64_LU, sb))
    return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  NRS_HIP(ctx, launch_build_csr(pb->N, pb->Q, pb->X, pb->w, pb->nu, sb.srt, nullptr, s));
  NRS_HIP(ctx, launch_apply(*pb, sb.srt, v, y, sb.part, sb.chunks, nullptr, s));
  return NRS_OK;
}

nrs_status nrs_solve(nrs_ctx* ctx, const nrs_problem* pb, const double* u, const double* ftext,
                     const nrs_options* opt, void* ws, size_t ws_bytes, double* sol,
                     nrs_info* info) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_problem(ctx, pb))) return st;
  if (!u || !sol) return fail(ctx, NRS_E_ARG, "u and sol required");
  nrs_options o = {};
  o.method = NRS_FP64_LU;
  if (opt) o = *opt;
  if (o.method < NRS_FP64_LU || o.method > NRS_GMRES_BLOCK)
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  if ((o.method == NRS_GMRES || gmres_ir(o.method) || o.method == NRS_GMRES_BLOCK) &&
      o.gmres_restart >= kGmresLd)
    return fail(ctx, NRS_E_UNSUPPORTED, "GMRES restart length must be below 64");
  if ((st = check_block_options(ctx, o, pb->M, true)) != NRS_OK) return st;
  Arena ar(ws, ws_bytes);
  SolveBuffers sb;
  if (!carve_solve(ar, pb->N, pb->Q, pb->M, o.method, sb))
    return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  SolveState h = {};
  st = solve_core(ctx, *pb, u, ftext, o, sb, sol, info != nullptr, &h);
  if (info) fill_info(h, info);
  return st;
}

nrs_status nrs_query_info(nrs_ctx* ctx, void* ws, nrs_info* info) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (!ws || !info) return fail(ctx, NRS_E_ARG, "ws and info required");
  SolveState h;
  if ((st = read_state(ctx, static_cast<const SolveState*>(ws), h))) return st;
  fill_info(h, info);
  return NRS_OK;
}

nrs_status nrs_lu_factor_workspace_size(nrs_ctx* ctx, int64_t n, int32_t precision,
                                        size_t* bytes) {
  if (!bytes || n <= 0) return fail(ctx, NRS_E_ARG, "bad LU workspace arguments");
  if (precision != 16 && precision != 32 && precision != 64)
    return fail(ctx, NRS_E_ARG, "precision must be 16, 32 or 64");
  if (n > 262144) return fail(ctx, NRS_E_UNSUPPORTED, "n too large");
  *bytes = lu_factor_ws_bytes(n, precision);
  return NRS_OK;
}

nrs_status nrs_lu_solve_workspace_size(nrs_ctx* ctx, int64_t n, size_t* bytes) {
  if (!bytes || n <= 0) return fail(ctx, NRS_E_ARG, "bad LU workspace arguments");
  if (n > 262144) return fail(ctx, NRS_E_UNSUPPORTED, "n too large");
  *bytes = lu_solve_ws_bytes(n);
  return NRS_OK;
}

nrs_status nrs_lu_factor(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope, void* A,
                         int64_t lda, int32_t* ipiv, int32_t* perm, int32_t* singular_flag,
                         void* ws, size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (n <= 0 || !A || lda < n || !ipiv || !perm || !singular_flag)
    return fail(ctx, NRS_E_ARG, "bad LU arguments");
  if (pivot_scope != 0 && pivot_scope != 1) return fail(ctx, NRS_E_ARG, "pivot_scope is 0 or 1");
  if (precision != 16 && precision != 32 && precision != 64)
    return fail(ctx, NRS_E_ARG, "precision must be 16, 32 or 64");
  if (precision == 16 && pivot_scope != 1)
    return fail(ctx, NRS_E_ARG, "precision 16 needs pivot_scope 1");
  if (n > 262144) return fail(ctx, NRS_E_UNSUPPORTED, "n too large");
  if (!ws || ws_bytes < lu_factor_ws_bytes(n, precision))
    return fail(ctx, NRS_E_WORKSPACE, "LU workspace missing or too small");
  // head and tile flags start at zero on every call (this also clears the
  // previous call's timeout flag)
  int32_t* ctl = align256(ws);
  int32_t* done = ctl + kLuHeadInts;
  const int64_t words = lu_factor_sync_ints(n);
  NRS_HIP(ctx, launch_fill_i32(ctl, 0, words, ctx->stream));
  if (precision == 16) {
    uint16_t* sh = reinterpret_cast<uint16_t*>(ctl + words);
    NRS_HIP(ctx, lu_factor_any<float>(n, 1, static_cast<float*>(A), lda, ipiv, perm, singular_flag,
                                      done, ctl, ctx->stream, sh));
  } else if (precision == 32) {
    NRS_HIP(ctx, lu_factor_any<float>(n, pivot_scope, static_cast<float*>(A), lda, ipiv, perm,
                                      singular_flag, done, ctl, ctx->stream, nullptr,
                                      ctl + words));
  } else {
    NRS_HIP(ctx, lu_factor_any<double>(n, pivot_scope, static_cast<double*>(A), lda, ipiv, perm,
                                       singular_flag, done, ctl, ctx->stream, nullptr,
                                       ctl + words));
  }
  return NRS_OK;
}

}  // extern "C"

namespace {

// Triangular solves of nrs_lu_solve on the synchronisation words at sync
// (kLuHeadInts head words, then trsv_sync_ints(n) words), all cleared first.
nrs_status lu_solve_on(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                       const void* LU, int64_t lda, const int32_t* perm, const void* b, void* x,
                       int32_t* sync) {
  NRS_HIP(ctx, launch_fill_i32(sync, 0, kLuHeadInts + trsv_sync_ints(n), ctx->stream));
  int32_t* err = sync + kLuTimeoutWord;
  int32_t* words = sync + kLuHeadInts;
  if (precision == 32)
    NRS_HIP(ctx, launch_lu_solve<float>(n, pivot_scope, static_cast<const float*>(LU), lda, perm,
                                        static_cast<const float*>(b), static_cast<float*>(x),
                                        words, err, nullptr, ctx->stream));
  else
    NRS_HIP(ctx, launch_lu_solve<double>(n, pivot_scope, static_cast<const double*>(LU), lda,
                                         perm, static_cast<const double*>(b),
                                         static_cast<double*>(x), words, err, nullptr,
                                         ctx->stream));
  return NRS_OK;
}

nrs_status check_lu_solve(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                          const void* LU, int64_t lda, const int32_t* perm, const void* b,
                          const void* x) {
  if (n <= 0 || !LU || lda < n || !perm || !b || !x || b == x)
    return fail(ctx, NRS_E_ARG, "bad LU solve arguments");
  if (pivot_scope != 0 && pivot_scope != 1) return fail(ctx, NRS_E_ARG, "pivot_scope is 0 or 1");
  if (precision != 32 && precision != 64) return fail(ctx, NRS_E_ARG, "precision must be 32 or 64");
  if (n > 262144) return fail(ctx, NRS_E_UNSUPPORTED, "n too large");
  return NRS_OK;
}

}  // namespace

extern "C" {

nrs_status nrs_lu_solve(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                        const void* LU, int64_t lda, const int32_t* perm, const void* b, void* x,
                        void* ws, size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_lu_solve(ctx, n, precision, pivot_scope, LU, lda, perm, b, x))) return st;
  if (!ws || ws_bytes < lu_solve_ws_bytes(n))
    return fail(ctx, NRS_E_WORKSPACE, "LU solve workspace missing or too small");
  return lu_solve_on(ctx, n, precision, pivot_scope, LU, lda, perm, b, x, align256(ws));
}

nrs_status nrs_lu_solve_noalloc(nrs_ctx* ctx, int64_t n, int32_t precision, int32_t pivot_scope,
                                const void* LU, int64_t lda, const int32_t* perm, const void* b,
                                void* x) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_lu_solve(ctx, n, precision, pivot_scope, LU, lda, perm, b, x))) return st;
  if (n > NRS_NOALLOC_MAX_N)
    return fail(ctx, NRS_E_UNSUPPORTED,
                "nrs_lu_solve_noalloc: n above NRS_NOALLOC_MAX_N (use nrs_lu_solve)");
  if (!ctx->scratch) return fail(ctx, NRS_E_HIP, "scratch address not set up");
  return lu_solve_on(ctx, n, precision, pivot_scope, LU, lda, perm, b, x, ctx->scratch);
}

nrs_status nrs_equilibrate(nrs_ctx* ctx, int64_t n, float* A, int64_t lda, float* dr, float* dc,
                           void* ws, size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (n <= 0 || !A || lda < n || !dr || !dc) return fail(ctx, NRS_E_ARG, "bad equilibration arguments");
  if (!ws || ws_bytes < (size_t)n * sizeof(uint32_t))
    return fail(ctx, NRS_E_WORKSPACE, "equilibration workspace missing or too small");
  NRS_HIP(ctx, launch_equilibrate(n, A, lda, dr, dc, static_cast<uint32_t*>(ws), ctx->stream));
  return NRS_OK;
}

nrs_status nrs_lu_query(nrs_ctx* ctx, const void* ws, int32_t* flags) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (!flags) return fail(ctx, NRS_E_ARG, "flags required");
  if (!ws && !ctx->scratch) return fail(ctx, NRS_E_HIP, "scratch address not set up");
  const int32_t* head = ws ? align256(const_cast<void*>(ws)) : ctx->scratch;
  int32_t h = 0;
  NRS_HIP(ctx, hipMemcpyAsync(&h, head + kLuTimeoutWord, sizeof(h), hipMemcpyDeviceToHost,
                              ctx->stream));
  NRS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *flags = h ? 1 : 0;
  return NRS_OK;
}

}  // extern "C"

namespace nrs {

int32_t size_class(int64_t N, int64_t Q) {
  auto lg = [](int64_t v) {
    int r = 0;
    while (v > 1) {
      v >>= 1;
      ++r;
    }
    return r;
  };
  return 64 * lg(N) + lg(Q / (N > 0 ? N : 1));
}

int32_t asm_shape_for(const nrs_ctx* ctx, int64_t N, int64_t Q, int bits) {
  if (!ctx) return -1;
  const int32_t c = size_class(N, Q);
  for (const auto& e : ctx->tune)
    if (e.cls == c) return bits == 32 ? e.shape32 : e.shape64;
  return -1;
}

}  // namespace nrs

extern "C" {

nrs_status nrs_autotune(nrs_ctx* ctx, const nrs_problem* pb, void* ws, size_t ws_bytes,
                        nrs_tune_result* out) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_problem(ctx, pb))) return st;
  Arena ar(ws, ws_bytes);
  SolveBuffers sb;
  if (!carve_solve(ar, pb->N, pb->Q, pb->M, NRS_FP32_IR, sb))
    return fail(ctx, NRS_E_WORKSPACE, "workspace too small (size it for NRS_FP32_IR)");
  hipStream_t s = ctx->stream;
  NRS_HIP(ctx, launch_state_init(sb.st, NRS_FP64_LU, s));
  NRS_HIP(ctx, launch_build_csr(pb->N, pb->Q, pb->X, pb->w, pb->nu, sb.srt, sb.st, s));
  hipEvent_t e0, e1;
  NRS_HIP(ctx, hipEventCreate(&e0));
  NRS_HIP(ctx, hipEventCreate(&e1));
  int32_t best[2] = {kAsmDefaultShape, kAsmDefaultShape};
  float best_ms[2] = {0.f, 0.f}, def_ms[2] = {0.f, 0.f};
  hipError_t err = hipSuccess;
  // per shape: one warm-up launch, then the best of three timed runs of
  // kLaunches back-to-back launches (one event pair around each run, so that
  // launch latency is not counted once per launch)
  constexpr int kLaunches = 8;
  auto launch = [&](int prec, int shape) {
    return prec == 0 ? launch_assemble<float>(*pb, sb.srt, sb.A32, sb.lda, s, shape)
                     : launch_assemble<double>(*pb, sb.srt, sb.A64, sb.lda, s, shape);
  };
  for (int prec = 0; prec < 2 && err == hipSuccess; ++prec) {
    for (int shape = 0; shape < kAsmShapes && err == hipSuccess; ++shape) {
      err = launch(prec, shape);
      float avg = 0.f;
      for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
        err = hipEventRecord(e0, s);
        for (int k = 0; k < kLaunches && err == hipSuccess; ++k) err = launch(prec, shape);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        const float per = ms / kLaunches;
        if (rep == 0 || per < avg) avg = per;
      }
      if (shape == kAsmDefaultShape) def_ms[prec] = avg;
      if (shape == 0 || avg < best_ms[prec]) {
        best_ms[prec] = avg;
        best[prec] = shape;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess) return fail(ctx, NRS_E_HIP, std::string("autotune: ") + hipGetErrorString(err));
  const int32_t c = size_class(pb->N, pb->Q);
  bool found = false;
  for (auto& e : ctx->tune)
    if (e.cls == c) {
      e.shape32 = best[0];
      e.shape64 = best[1];
      found = true;
    }
  if (!found) ctx->tune.push_back({c, best[0], best[1]});
  if (out) {
    out->size_class = c;
    asm_shape_dims(best[0], &out->block32, &out->strip32);
    asm_shape_dims(best[1], &out->block64, &out->strip64);
    out->ms32 = best_ms[0];
    out->ms64 = best_ms[1];
    out->default_ms32 = def_ms[0];
    out->default_ms64 = def_ms[1];
  }
  return NRS_OK;
}

nrs_status nrs_autotune_clear(nrs_ctx* ctx) {
  if (!ctx) return NRS_E_ARG;
  ctx->tune.clear();
  return NRS_OK;
}

nrs_status nrs_block_limit(nrs_ctx* ctx, int32_t* nb_max) {
  if (!ctx || !nb_max) return fail(ctx, NRS_E_ARG, "ctx and nb_max required");
  *nb_max = ctx->block_lim;
  return NRS_OK;
}

nrs_status nrs_block_invert(nrs_ctx* ctx, int32_t count, int32_t nb, double* blocks,
                            int32_t* singular) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (count < 0 || nb < 1 || !blocks || !singular)
    return fail(ctx, NRS_E_ARG, "bad block inversion arguments");
  if (nb > ctx->block_lim) return fail(ctx, NRS_E_UNSUPPORTED, "nb exceeds nrs_block_limit()");
  NRS_HIP(ctx, launch_block_inverse(count, nb, (int64_t)nb * nb, 0, nullptr, nb, blocks, singular,
                                    ctx->stream));
  return NRS_OK;
}

nrs_status nrs_block_model_fit(nrs_ctx* ctx, int32_t S, int32_t nb, int32_t H,
                               const double* inverses, double* model) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (nb < 1 || H < 0 || H > kBlockHarmonicsMax || S < 2 * H + 1 || !inverses || !model)
    return fail(ctx, NRS_E_ARG, "bad block model fit arguments");
  NRS_HIP(ctx, launch_block_fit(S, nb, H, inverses, model, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_block_model_eval(nrs_ctx* ctx, int32_t nb, int32_t H, const double* model,
                                int32_t count, const double* psi, double* blocks) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (nb < 1 || H < 0 || H > kBlockHarmonicsMax || count < 0 || !model ||
      (count > 0 && (!psi || !blocks)))
    return fail(ctx, NRS_E_ARG, "bad block model arguments");
  NRS_HIP(ctx, launch_block_model(count, 0, nullptr, 0, nb, H, model, psi, (int64_t)nb * nb,
                                  blocks, ctx->stream));
  return NRS_OK;
}

}  // extern "C"

namespace {

struct RkBuffers {
  SolveState* report;
  double *x, *X, *w, *u, *Ys, *K[4], *sol, *Ysave;
  int32_t* nu;
  float *phi, *my, *mz;   // network features / outputs (GMRES warm start)
  SolveBuffers sb;
  // adaptive Dormand-Prince: seven stage rates, the candidate state, its
  // error norm (device scalar)
  double *DK[7], *Ynew, *enorm;
  // passive tracers: stage rates, saved positions, field sources and sums
  int64_t P;
  FieldPlan fplan;
  double *TK[4], *ysave, *fpart;
  FieldSrc* src;
};

bool carve_rk(Arena& ar, const nrs_scene& sc, int32_t method, int64_t P, RkBuffers& rb,
              bool dopri = false) {
  const int64_t N = sc.N, Q = sc.Q, M = sc.M, n = 3 * N + 6 * M;
  rb.report = ar.take<SolveState>(1);
  rb.x = ar.take<double>(3 * N);
  rb.X = ar.take<double>(3 * Q);
  rb.w = ar.take<double>(Q);
  rb.u = ar.take<double>(3 * N);
  rb.nu = ar.take<int32_t>(Q);
  rb.Ys = ar.take<double>(12 * M);
  for (int i = 0; i < 4; ++i) rb.K[i] = ar.take<double>(12 * M);
  rb.Ysave = ar.take<double>(12 * M);
  rb.sol = ar.take<double>(n);
  rb.phi = rb.my = rb.mz = nullptr;
  if (krylov_warm(method)) {
    rb.phi = ar.take<float>(7 * N);
    rb.my = ar.take<float>(3 * N);
    rb.mz = ar.take<float>(6 * M);
  }
  carve_solve(ar, N, Q, sc.M, method, rb.sb);
  // tracers last: the report stays at the start of the workspace (nrs_query_info)
  rb.P = P;
  rb.fplan = field_plan(P, Q);
  for (int i = 0; i < 4; ++i) rb.TK[i] = P > 0 ? ar.take<double>(3 * P) : nullptr;
  rb.ysave = P > 0 ? ar.take<double>(3 * P) : nullptr;
  rb.fpart = P > 0 ? ar.take<double>((size_t)rb.fplan.cap * 3 * P) : nullptr;
  rb.src = P > 0 ? ar.take<FieldSrc>(Q) : nullptr;
  for (int i = 0; i < 7; ++i) rb.DK[i] = dopri ? ar.take<double>(12 * M) : nullptr;
  rb.Ynew = dopri ? ar.take<double>(12 * M) : nullptr;
  rb.enorm = dopri ? ar.take<double>(8) : nullptr;
  return !ar.overflow;
}

// One stage: geometry, nearest map and solve at the state rb.Ys and time tt,
// then the rates of the bodies into Kout.  warm: the previous solve of this
// workspace may seed a GMRES warm start.
nrs_status stage_solve(nrs_ctx* ctx, const nrs_scene& sc, const GroupTable& gt,
                       const int32_t* groupX, double eps, double mu, const double* ftext,
                       double tt, const nrs_options& o, RkBuffers& rb, bool warm, double* Kout,
                       bool reuse = false, const double* Ynext = nullptr, double anext = 0.0) {
  hipStream_t s = ctx->stream;
  NRS_HIP(ctx, launch_geometry(sc, tt, rb.Ys, rb.x, rb.X, rb.w, rb.u, s));
  NRS_HIP(ctx, launch_nearest(sc.N, rb.x, gt, sc.Q, rb.X, groupX, rb.nu, s));
  nrs_problem pb;
  pb.N = sc.N;
  pb.Q = sc.Q;
  pb.M = sc.M;
  pb.x = rb.x;
  pb.X = rb.X;
  pb.w = rb.w;
  pb.nu = rb.nu;
  pb.body = sc.body;
  pb.Y = rb.Ys;
  pb.eps = eps;
  pb.mu = mu;
  nrs_options os = o;
  // the learned block model takes each body's phase from the scene at tt
  rb.sb.phase_scene = &sc;
  rb.sb.phase_t = tt;
  if (krylov_warm(o.method)) {
    // warm start of this stage's GMRES solve
    os.x_init = nullptr;
    if (o.warm_start == NRS_WARM_PREVIOUS && warm) {
      os.x_init = rb.sol;
    } else if (o.warm_start == NRS_WARM_MODEL) {
      NRS_HIP(ctx, launch_features(sc.N, rb.x, rb.u, sc.s, sc.body, sc.M, rb.Ys, rb.phi, s));
      NRS_HIP(ctx, launch_mlp_forward(o.model_theta, sc.M, sc.M, sc.N, o.body_off, nullptr,
                                      rb.phi, rb.my, rb.mz, ctx->dflags, s));
      NRS_HIP(ctx, launch_to_lab(sc.N, sc.M, sc.body, rb.Ys, rb.my, rb.mz, o.model_scales,
                                 rb.sol, s));
      os.x_init = rb.sol;
      os.x_init_complete = o.method == NRS_GMRES;
    }
  }
  nrs_status st = solve_core(ctx, pb, rb.u, ftext, os, rb.sb, rb.sol, false, nullptr, reuse);
  if (st != NRS_OK) return st;
  // the report, the rates and (Ynext) the next RK4 stage's state
  NRS_HIP(ctx, launch_stage_end(rb.report, rb.sb.st, sc.M, sc.N, rb.Ys, rb.sol, Kout, Ynext, anext,
                                s));
  return NRS_OK;
}

nrs_status rk4_pass(nrs_ctx* ctx, const nrs_scene& sc, const GroupTable& gt,
                    const int32_t* groupX, double eps, double mu, const double* ftext, double* Y,
                    double* ytr, double t, double dt, const nrs_options& o, RkBuffers& rb,
                    bool prev_valid) {
  hipStream_t s = ctx->stream;
  const double c[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
  NRS_HIP(ctx, launch_state_init(rb.report, o.method, s));
  // stage 1 starts from Y; the end of stages 1-3 forms the next stage's state
  NRS_HIP(ctx, launch_rk_stage_state(sc.M, Y, nullptr, 0.0, rb.Ys, s));
  for (int stg = 0; stg < 4; ++stg) {
    // stages 2-4 may refine against the first stage's FP32 factors
    const bool reuse = stg > 0 && o.reuse_stage_factors && o.method == NRS_FP32_IR;
    nrs_status st = stage_solve(ctx, sc, gt, groupX, eps, mu, ftext, t + c[stg], o, rb,
                                stg > 0 || prev_valid, rb.K[stg], reuse, stg < 3 ? Y : nullptr,
                                stg < 3 ? c[stg + 1] : 0.0);
    if (st != NRS_OK) return st;
    if (rb.P > 0) {
      // this stage's flow (its geometry and forces) at the tracers' stage positions
      NRS_HIP(ctx, launch_field_sources(sc.N, sc.Q, rb.X, rb.w, rb.nu, rb.sol, rb.src, s));
      NRS_HIP(ctx, launch_field(rb.fplan, rb.P, sc.Q, ytr, stg ? rb.TK[stg - 1] : nullptr, c[stg],
                                rb.src, eps, mu, rb.fpart, rb.TK[stg], s));
    }
  }
  NRS_HIP(ctx, launch_rk_combine(sc.M, Y, rb.K[0], rb.K[1], rb.K[2], rb.K[3], dt, s));
  NRS_HIP(ctx, launch_tracer_combine(rb.P, ytr, rb.TK[0], rb.TK[1], rb.TK[2], rb.TK[3], dt, s));
  return NRS_OK;
}

// Field points per call: the grid of the pair kernel stays below 2^31 workgroups.
constexpr int64_t kMaxFieldPoints = (int64_t)1 << 28;

struct FieldBuffers {
  FieldSrc* src;   // [Q] gathered sources
  double* part;    // [chunks][3P] chunk sums
  double* K[4];    // [3P] RK stage rates (tracer steps)
};

bool carve_field(Arena& ar, int64_t P, int64_t Q, FieldBuffers& fb) {
  const FieldPlan fp = field_plan(P, Q);
  fb.src = ar.take<FieldSrc>(Q);
  fb.part = ar.take<double>((size_t)fp.cap * 3 * std::max<int64_t>(P, 1));
  for (int i = 0; i < 4; ++i) fb.K[i] = ar.take<double>(3 * std::max<int64_t>(P, 1));
  return !ar.overflow;
}

// A flow for the field sum: sources X, w, nu of N force points, densities f.
nrs_status check_flow(nrs_ctx* ctx, const nrs_problem* pb, const double* f) {
  if (!pb) return fail(ctx, NRS_E_ARG, "problem is NULL");
  if (pb->N <= 0 || pb->Q <= 0) return fail(ctx, NRS_E_ARG, "need N > 0, Q > 0");
  if (pb->N > (int64_t)1 << 20 || pb->Q > (int64_t)1 << 30)
    return fail(ctx, NRS_E_UNSUPPORTED, "N or Q too large");
  if (!pb->X || !pb->nu || !f) return fail(ctx, NRS_E_ARG, "X, nu and f required");
  if (!(pb->eps > 0.0) || !(pb->mu > 0.0) || !std::isfinite(pb->eps) || !std::isfinite(pb->mu))
    return fail(ctx, NRS_E_ARG, "eps and mu must be positive and finite");
  return NRS_OK;
}

nrs_status check_scene(nrs_ctx* ctx, const nrs_scene* sc) {
  if (!sc || sc->N <= 0 || sc->Q <= 0 || sc->M < 0 || sc->P < 0)
    return fail(ctx, NRS_E_ARG, "bad scene sizes");
  if (!sc->xi || !sc->body || !sc->part || !sc->s || !sc->ufix || !sc->Xi || !sc->bodyX ||
      !sc->partX || !sc->sX || !sc->w0 || (sc->P > 0 && !sc->wave))
    return fail(ctx, NRS_E_ARG, "scene arrays missing");
  return NRS_OK;
}

}  // namespace

extern "C" {

nrs_status nrs_rk4_tracers_workspace_size(nrs_ctx* ctx, const nrs_scene* sc, int32_t method,
                                          int64_t P, size_t* bytes) {
  nrs_status st = check_scene(ctx, sc);
  if (st) return st;
  if (!bytes) return fail(ctx, NRS_E_ARG, "bytes is NULL");
  if (P < 0 || P > kMaxFieldPoints) return fail(ctx, NRS_E_ARG, "tracer count out of range");
  if (method < NRS_FP64_LU || method > NRS_GMRES_BLOCK)
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  Arena ar(nullptr, 0);
  RkBuffers rb;
  carve_rk(ar, *sc, method, P, rb);
  *bytes = ar.used + 256;
  return NRS_OK;
}

nrs_status nrs_rk4_workspace_size(nrs_ctx* ctx, const nrs_scene* sc, int32_t method,
                                  size_t* bytes) {
  return nrs_rk4_tracers_workspace_size(ctx, sc, method, 0, bytes);
}

nrs_status nrs_rk4_step_tracers(nrs_ctx* ctx, const nrs_scene* sc, int32_t G,
                                const int32_t* group_off_host, const int32_t* groupX, double eps,
                                double mu, const double* ftext, double* Y, double t, double dt,
                                const nrs_options* opt, int64_t P, double* ytr, void* ws,
                                size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_scene(ctx, sc))) return st;
  if (sc->M <= 0 || !Y) return fail(ctx, NRS_E_ARG, "time stepping needs free bodies and Y");
  if (P < 0 || P > kMaxFieldPoints) return fail(ctx, NRS_E_ARG, "tracer count out of range");
  if (P > 0 && !ytr) return fail(ctx, NRS_E_ARG, "tracer positions required");
  if (!group_off_host || !groupX || G <= 0) return fail(ctx, NRS_E_ARG, "groups required");
  if (G > kMaxGroups) return fail(ctx, NRS_E_UNSUPPORTED, "too many groups");
  if (!(eps > 0.0) || !(mu > 0.0) || !std::isfinite(t) || !std::isfinite(dt))
    return fail(ctx, NRS_E_ARG, "eps, mu > 0 and finite t, dt required");
  GroupTable gt;
  gt.G = G;
  for (int g = 0; g <= G; ++g) gt.off[g] = group_off_host[g];
  if (gt.off[0] != 0 || gt.off[G] != sc->N) return fail(ctx, NRS_E_ARG, "group_off must span [0, N]");
  for (int g = 0; g < G; ++g)
    if (gt.off[g + 1] <= gt.off[g]) return fail(ctx, NRS_E_ARG, "every group needs a force point");
  nrs_options o = {};
  o.method = NRS_FP64_LU;
  if (opt) o = *opt;
  if (o.method < NRS_FP64_LU || o.method > NRS_GMRES_BLOCK)
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  if ((o.method == NRS_GMRES || gmres_ir(o.method) || o.method == NRS_GMRES_BLOCK) &&
      o.gmres_restart >= kGmresLd)
    return fail(ctx, NRS_E_UNSUPPORTED, "GMRES restart length must be below 64");
  if ((st = check_block_options(ctx, o, sc->M, false)) != NRS_OK) return st;
  Arena ar(ws, ws_bytes);
  RkBuffers rb;
  if (!carve_rk(ar, *sc, o.method, P, rb)) return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  NRS_HIP(ctx, hipMemcpyAsync(rb.Ysave, Y, 12 * sizeof(double) * sc->M, hipMemcpyDeviceToDevice, s));
  if (P > 0)
    NRS_HIP(ctx, hipMemcpyAsync(rb.ysave, ytr, 3 * sizeof(double) * P, hipMemcpyDeviceToDevice, s));
  if (krylov_warm(o.method) && o.warm_start == NRS_WARM_MODEL) {
    if (!o.model_theta || !o.body_off || !sc->s)
      return fail(ctx, NRS_E_ARG, "model warm start needs model_theta, body_off and scene s");
    if (!(o.model_scales[0] > 0) || !(o.model_scales[1] > 0) || !(o.model_scales[2] > 0))
      return fail(ctx, NRS_E_ARG, "model scales must be positive");
    if ((st = ctx_dev_flags(ctx)) != NRS_OK) return st;
  }
  if (o.ir_queue < 0) return fail(ctx, NRS_E_ARG, "ir_queue must be >= 0");
  const bool prev_valid = ctx->rk_prev_ws == ws;
  const int32_t hint = prev_valid ? ctx->rk_sweeps : 0;
  ctx->rk_prev_ws = nullptr;
  ctx->rk_sweeps = 0;
  // correction sweeps queued per stage of the factoring refinement forms:
  // ir_queue, else the previous step's largest need plus one (the step's one
  // host check below learns it), never more than max_refine
  const int32_t full = o.max_refine > 0 ? o.max_refine : 4;
  const bool adapt = (o.method == NRS_FP32_IR || o.method == NRS_FP32_GEPP_IR) &&
                     !o.reuse_stage_factors && !o.no_fallback;
  nrs_options oq = o;
  if (adapt) oq.max_refine = std::min(full, o.ir_queue > 0 ? o.ir_queue : (hint > 0 ? hint + 1 : full));
  if ((st = rk4_pass(ctx, *sc, gt, groupX, eps, mu, ftext, Y, ytr, t, dt, oq, rb, prev_valid)) !=
      NRS_OK)
    return st;
  ctx->rk_prev_ws = ws;
  if (o.no_fallback || o.method == NRS_FP64_LU) return NRS_OK;
  SolveState h;
  if ((st = read_state(ctx, rb.report, h)) != NRS_OK) return st;
  if (h.failed && adapt && oq.max_refine < full && !h.nonfinite && !h.sync_err) {
    // the queue was too short for a stage: the step again with max_refine sweeps
    NRS_HIP(ctx, hipMemcpyAsync(Y, rb.Ysave, 12 * sizeof(double) * sc->M, hipMemcpyDeviceToDevice, s));
    if (P > 0)
      NRS_HIP(ctx, hipMemcpyAsync(ytr, rb.ysave, 3 * sizeof(double) * P, hipMemcpyDeviceToDevice, s));
    oq.max_refine = full;
    if ((st = rk4_pass(ctx, *sc, gt, groupX, eps, mu, ftext, Y, ytr, t, dt, oq, rb, prev_valid)) !=
        NRS_OK)
      return st;
    if ((st = read_state(ctx, rb.report, h)) != NRS_OK) return st;
  }
  if (!h.failed) {
    if (adapt) ctx->rk_sweeps = std::max(1, h.iterations - 1);
    return NRS_OK;
  }
  // a stage missed its tolerance: redo the whole step with FP64 LU
  NRS_HIP(ctx, hipMemcpyAsync(Y, rb.Ysave, 12 * sizeof(double) * sc->M, hipMemcpyDeviceToDevice, s));
  if (P > 0)
    NRS_HIP(ctx, hipMemcpyAsync(ytr, rb.ysave, 3 * sizeof(double) * P, hipMemcpyDeviceToDevice, s));
  nrs_options o64 = o;
  o64.method = NRS_FP64_LU;
  if ((st = rk4_pass(ctx, *sc, gt, groupX, eps, mu, ftext, Y, ytr, t, dt, o64, rb, false)) != NRS_OK)
    return st;
  SolveState mark = {};
  if ((st = read_state(ctx, rb.report, mark)) != NRS_OK) return st;
  mark.fell_back = 1;
  NRS_HIP(ctx, hipMemcpyAsync(rb.report, &mark, sizeof(SolveState), hipMemcpyHostToDevice, s));
  NRS_HIP(ctx, hipStreamSynchronize(s));
  return NRS_OK;
}

nrs_status nrs_rk4_step(nrs_ctx* ctx, const nrs_scene* sc, int32_t G, const int32_t* group_off_host,
                        const int32_t* groupX, double eps, double mu, const double* ftext,
                        double* Y, double t, double dt, const nrs_options* opt, void* ws,
                        size_t ws_bytes) {
  return nrs_rk4_step_tracers(ctx, sc, G, group_off_host, groupX, eps, mu, ftext, Y, t, dt, opt, 0,
                              nullptr, ws, ws_bytes);
}

// ---- adaptive Dormand-Prince 5(4) time stepping ----

nrs_status nrs_dopri5_workspace_size(nrs_ctx* ctx, const nrs_scene* sc, int32_t method,
                                     size_t* bytes) {
  nrs_status st = check_scene(ctx, sc);
  if (st) return st;
  if (!bytes) return fail(ctx, NRS_E_ARG, "bytes is NULL");
  if (method < NRS_FP64_LU || method > NRS_GMRES_BLOCK)
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  Arena ar(nullptr, 0);
  RkBuffers rb;
  carve_rk(ar, *sc, method, 0, rb, true);
  *bytes = ar.used + 256;
  return NRS_OK;
}

nrs_status nrs_dopri5_integrate(nrs_ctx* ctx, const nrs_scene* sc, int32_t G,
                                const int32_t* group_off_host, const int32_t* groupX, double eps,
                                double mu, const double* ftext, double* Y, double t0, double t1,
                                double* h_io, double rtol, double atol, const nrs_options* opt,
                                int32_t max_steps, nrs_dopri5_stats* stats, void* ws,
                                size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_scene(ctx, sc))) return st;
  if (sc->M <= 0 || !Y) return fail(ctx, NRS_E_ARG, "time stepping needs free bodies and Y");
  if (!group_off_host || !groupX || G <= 0) return fail(ctx, NRS_E_ARG, "groups required");
  if (G > kMaxGroups) return fail(ctx, NRS_E_UNSUPPORTED, "too many groups");
  if (!(eps > 0.0) || !(mu > 0.0) || !std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0))
    return fail(ctx, NRS_E_ARG, "eps, mu > 0 and finite t0 <= t1 required");
  if (!h_io || !(*h_io > 0.0) || !std::isfinite(*h_io) || !(rtol > 0.0) || !(atol >= 0.0))
    return fail(ctx, NRS_E_ARG, "first step > 0, rtol > 0 and atol >= 0 required");
  GroupTable gt;
  gt.G = G;
  for (int g = 0; g <= G; ++g) gt.off[g] = group_off_host[g];
  if (gt.off[0] != 0 || gt.off[G] != sc->N) return fail(ctx, NRS_E_ARG, "group_off must span [0, N]");
  for (int g = 0; g < G; ++g)
    if (gt.off[g + 1] <= gt.off[g]) return fail(ctx, NRS_E_ARG, "every group needs a force point");
  nrs_options o = {};
  o.method = NRS_FP64_LU;
  if (opt) o = *opt;
  if (o.method < NRS_FP64_LU || o.method > NRS_GMRES_BLOCK)
    return fail(ctx, NRS_E_UNSUPPORTED, "method not implemented");
  if ((o.method == NRS_GMRES || gmres_ir(o.method) || o.method == NRS_GMRES_BLOCK) &&
      o.gmres_restart >= kGmresLd)
    return fail(ctx, NRS_E_UNSUPPORTED, "GMRES restart length must be below 64");
  if ((st = check_block_options(ctx, o, sc->M, false)) != NRS_OK) return st;
  if (krylov_warm(o.method) && o.warm_start == NRS_WARM_MODEL) {
    if (!o.model_theta || !o.body_off || !sc->s)
      return fail(ctx, NRS_E_ARG, "model warm start needs model_theta, body_off and scene s");
    if ((st = ctx_dev_flags(ctx)) != NRS_OK) return st;
  }
  Arena ar(ws, ws_bytes);
  RkBuffers rb;
  if (!carve_rk(ar, *sc, o.method, 0, rb, true))
    return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  const int64_t n12 = 12 * (int64_t)sc->M;
  const size_t bytes12 = n12 * sizeof(double);
  ctx->rk_prev_ws = nullptr;
  // Dormand-Prince 5(4): nodes, stage rows, error weights (5th minus 4th order)
  static const double kC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
  static const double kA[7][6] = {
      {0, 0, 0, 0, 0, 0},
      {1.0 / 5, 0, 0, 0, 0, 0},
      {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
      {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
      {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
      {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
      {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
  static const double kB4[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};
  double kE[7];
  for (int j = 0; j < 7; ++j) kE[j] = (j < 6 ? kA[6][j] : 0.0) - kB4[j];
  nrs_dopri5_stats sts = {};
  double t = t0, h = *h_io;
  bool rejected = false;
  // k1 = F(Y, t0)
  NRS_HIP(ctx, launch_state_init(rb.report, o.method, s));
  NRS_HIP(ctx, hipMemcpyAsync(rb.Ys, Y, bytes12, hipMemcpyDeviceToDevice, s));
  if ((st = stage_solve(ctx, *sc, gt, groupX, eps, mu, ftext, t, o, rb, false, rb.DK[0])) != NRS_OK)
    return st;
  sts.solves = 1;
  double* K[7];
  for (int i = 0; i < 7; ++i) K[i] = rb.DK[i];
  while (t < t1 && sts.accepted + sts.rejected < max_steps) {
    h = std::min(h, t1 - t);
    nrs_options oa = o;
    for (int pass = 0; pass < 2; ++pass) {
      // stages 2..7 (stage 7 at the candidate state y_new = Y + h sum a7j k_j)
      for (int stg = 1; stg < 7; ++stg) {
        RkComb cb;
        cb.count = stg;
        for (int j = 0; j < 7; ++j) {
          cb.K[j] = K[j];
          cb.c[j] = j < stg ? kA[stg][j] : 0.0;
        }
        double* dst = stg == 6 ? rb.Ynew : rb.Ys;
        NRS_HIP(ctx, launch_rk_lincomb(n12, Y, cb, h, dst, s));
        if (stg == 6) NRS_HIP(ctx, hipMemcpyAsync(rb.Ys, rb.Ynew, bytes12, hipMemcpyDeviceToDevice, s));
        if ((st = stage_solve(ctx, *sc, gt, groupX, eps, mu, ftext, t + kC[stg] * h, oa, rb, true,
                              K[stg])) != NRS_OK)
          return st;
        sts.solves += 1;
      }
      RkComb ce;
      ce.count = 7;
      for (int j = 0; j < 7; ++j) {
        ce.K[j] = K[j];
        ce.c[j] = kE[j];
      }
      NRS_HIP(ctx, launch_dp_error(n12, Y, rb.Ynew, ce, h, rtol, atol, rb.enorm, s));
      SolveState rep;
      NRS_HIP(ctx, hipMemcpyAsync(&rep, rb.report, sizeof(rep), hipMemcpyDeviceToHost, s));
      double nrm = 0.0;
      NRS_HIP(ctx, hipMemcpyAsync(&nrm, rb.enorm, sizeof(double), hipMemcpyDeviceToHost, s));
      NRS_HIP(ctx, hipStreamSynchronize(s));
      if (rep.nonfinite == 2) return fail(ctx, NRS_E_ARG, "nu outside [0, N) or body outside [-1, M)");
      const bool failed = rep.failed && oa.method != NRS_FP64_LU;
      if (failed && !o.no_fallback && pass == 0) {
        // a stage solve missed its tolerance: redo this attempt with FP64 LU
        NRS_HIP(ctx, launch_state_init(rb.report, NRS_FP64_LU, s));
        oa.method = NRS_FP64_LU;
        sts.fell_back = 1;
        continue;
      }
      if (failed) return fail(ctx, NRS_E_NOT_CONVERGED, "a stage solve did not converge");
      if (!std::isfinite(nrm)) return fail(ctx, NRS_E_NONFINITE, "non-finite error estimate");
      if (nrm <= 1.0) {
        double fac = nrm == 0.0 ? 10.0 : std::min(10.0, 0.9 * std::pow(nrm, -0.2));
        if (rejected) fac = std::min(1.0, fac);
        NRS_HIP(ctx, hipMemcpyAsync(Y, rb.Ynew, bytes12, hipMemcpyDeviceToDevice, s));
        std::swap(K[0], K[6]);   // first stage of the next step = last stage of this one
        t += h;
        h *= fac;
        rejected = false;
        sts.accepted += 1;
      } else {
        h *= std::max(0.2, 0.9 * std::pow(nrm, -0.2));
        rejected = true;
        sts.rejected += 1;
      }
      break;
    }
  }
  NRS_HIP(ctx, hipStreamSynchronize(s));
  sts.t = t;
  sts.h = h;
  *h_io = h;
  if (stats) *stats = sts;
  return NRS_OK;
}

// ---- flow at field points and tracers through precomputed flows ----

nrs_status nrs_field_workspace_size(nrs_ctx* ctx, int64_t P, int64_t Q, size_t* bytes) {
  if (!bytes) return fail(ctx, NRS_E_ARG, "bytes is NULL");
  if (P < 0 || P > kMaxFieldPoints || Q <= 0 || Q > ((int64_t)1 << 30))
    return fail(ctx, NRS_E_ARG, "P or Q out of range");
  Arena ar(nullptr, 0);
  FieldBuffers fb;
  carve_field(ar, P, Q, fb);
  *bytes = ar.used + 256;
  return NRS_OK;
}

nrs_status nrs_field_velocity(nrs_ctx* ctx, const nrs_problem* pb, const double* f, int64_t P,
                              const double* y, double* u, void* ws, size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if ((st = check_flow(ctx, pb, f))) return st;
  if (P < 0 || P > kMaxFieldPoints) return fail(ctx, NRS_E_ARG, "field point count out of range");
  if (P == 0) return NRS_OK;
  if (!y || !u) return fail(ctx, NRS_E_ARG, "y and u required");
  Arena ar(ws, ws_bytes);
  FieldBuffers fb;
  if (!carve_field(ar, P, pb->Q, fb)) return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  NRS_HIP(ctx, launch_field_sources(pb->N, pb->Q, pb->X, pb->w, pb->nu, f, fb.src, s));
  NRS_HIP(ctx, launch_field(field_plan(P, pb->Q), P, pb->Q, y, nullptr, 0.0, fb.src, pb->eps,
                            pb->mu, fb.part, u, s));
  return NRS_OK;
}

nrs_status nrs_tracer_rk4_step(nrs_ctx* ctx, const nrs_problem* flows, const double* const* f,
                               int64_t P, double* y, double dt, void* ws, size_t ws_bytes) {
  nrs_status st = use_device(ctx);
  if (st) return st;
  if (!flows || !f) return fail(ctx, NRS_E_ARG, "flows and f required");
  for (int k = 0; k < 3; ++k)
    if ((st = check_flow(ctx, &flows[k], f[k]))) return st;
  if (P < 0 || P > kMaxFieldPoints) return fail(ctx, NRS_E_ARG, "tracer count out of range");
  if (!std::isfinite(dt)) return fail(ctx, NRS_E_ARG, "dt must be finite");
  if (P == 0) return NRS_OK;
  if (!y) return fail(ctx, NRS_E_ARG, "tracer positions required");
  const int64_t Qmax = std::max(flows[0].Q, std::max(flows[1].Q, flows[2].Q));
  Arena ar(ws, ws_bytes);
  FieldBuffers fb;
  if (!carve_field(ar, P, Qmax, fb)) return fail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  // stages: flow at t, t + dt/2 (twice), t + dt
  const int which[4] = {0, 1, 1, 2};
  const double c[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
  for (int stg = 0; stg < 4; ++stg) {
    const nrs_problem& fl = flows[which[stg]];
    if (stg != 2)
      NRS_HIP(ctx, launch_field_sources(fl.N, fl.Q, fl.X, fl.w, fl.nu, f[which[stg]], fb.src, s));
    NRS_HIP(ctx, launch_field(field_plan(P, fl.Q), P, fl.Q, y, stg ? fb.K[stg - 1] : nullptr,
                              c[stg], fb.src, fl.eps, fl.mu, fb.part, fb.K[stg], s));
  }
  NRS_HIP(ctx, launch_tracer_combine(P, y, fb.K[0], fb.K[1], fb.K[2], fb.K[3], dt, s));
  return NRS_OK;
}

}  // extern "C"
