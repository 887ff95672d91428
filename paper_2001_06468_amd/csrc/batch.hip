// Many independent resistance / swimming problems of different sizes solved
// together: every factorisation of the batch runs in ONE launch of the tile
// LU (tasks of all systems interleaved band by band), and every triangular
// sweep of the batch in one launch per pass.  Assembly and the FP64 residual
// stay per system (they are short and have no cross-system sharing); those
// launches are spread over four streams so that small systems overlap.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nrs_internal.h"

using namespace nrs;

namespace {

nrs_status bfail(nrs_ctx* ctx, nrs_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

#define NRS_BHIP(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return bfail(ctx, NRS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

struct BatchLayout {
  int32_t* ctl;            // [0..3] LU ticket/exit/timeout, [4..5] trsv ticket/done, [6] trsv err
  LuSys<float>* lusys;     // [B]
  TrsvSys<float>* trsys;   // [B]
  int32_t* lu_pref;        // [2*nbands*B + 1]
  int32_t* tr_pref;        // [nsteps*B + 1]
  std::vector<SolveBuffers> sb;
  std::vector<int32_t> lu_pref_h, tr_pref_h;
  int32_t nbands = 0, nsteps = 0, lu_total = 0, tr_total = 0;
};

bool carve_batch(Arena& ar, int32_t B, const nrs_problem* pb, BatchLayout& L) {
  std::vector<int32_t> nts(B), nbs(B);
  for (int s = 0; s < B; ++s) {
    const int64_t n = 3 * pb[s].N + 6 * (int64_t)pb[s].M;
    nts[s] = (int32_t)lu_tiles_nt(n);
    nbs[s] = (int32_t)((n + 63) / 64);
  }
  lu_task_prefix(nts.data(), B, L.lu_pref_h, L.nbands);
  L.lu_total = L.lu_pref_h.back();
  // triangular-solve tickets: one per 64-row block, step by step
  L.nsteps = 0;
  for (int s = 0; s < B; ++s) L.nsteps = std::max(L.nsteps, nbs[s]);
  L.tr_pref_h.assign((size_t)L.nsteps * B + 1, 0);
  int32_t acc = 0;
  for (int k = 0; k < L.nsteps; ++k)
    for (int s = 0; s < B; ++s) {
      L.tr_pref_h[(size_t)k * B + s] = acc;
      if (k < nbs[s]) acc += 1;
    }
  L.tr_pref_h[(size_t)L.nsteps * B] = acc;
  L.tr_total = acc;
  L.ctl = ar.take<int32_t>(8);
  L.lusys = ar.take<LuSys<float>>(B);
  L.trsys = ar.take<TrsvSys<float>>(B);
  L.lu_pref = ar.take<int32_t>(L.lu_pref_h.size());
  L.tr_pref = ar.take<int32_t>(L.tr_pref_h.size());
  L.sb.resize(B);
  for (int s = 0; s < B; ++s) carve_solve(ar, pb[s].N, pb[s].Q, pb[s].M, NRS_FP32_IR, L.sb[s], false);
  return !ar.overflow;
}

nrs_status check_batch(nrs_ctx* ctx, int32_t B, const nrs_problem* pb) {
  if (B <= 0 || !pb) return bfail(ctx, NRS_E_ARG, "batch needs B > 0 problems");
  for (int s = 0; s < B; ++s) {
    const nrs_problem& p = pb[s];
    if (p.N <= 0 || p.Q <= 0 || p.M < 0 || !p.x || !p.X || !p.nu || !p.body ||
        (p.M > 0 && !p.Y) || !(p.eps > 0.0) || !(p.mu > 0.0))
      return bfail(ctx, NRS_E_ARG, "invalid problem " + std::to_string(s) + " in batch");
    if (3 * p.N + 6 * (int64_t)p.M > 262144 || p.N > (1 << 20))
      return bfail(ctx, NRS_E_UNSUPPORTED, "problem " + std::to_string(s) + " too large");
  }
  return NRS_OK;
}

// pinned staging for the batch descriptors; reuse waits for the last copy
nrs_status stage(nrs_ctx* ctx, size_t bytes, char** host) {
  if (ctx->staging_event) NRS_BHIP(ctx, hipEventSynchronize(ctx->staging_event));
  if (ctx->staging_cap < bytes) {
    if (ctx->staging) NRS_BHIP(ctx, hipHostFree(ctx->staging));
    ctx->staging = nullptr;
    ctx->staging_cap = 0;
    NRS_BHIP(ctx, hipHostMalloc(&ctx->staging, bytes));
    ctx->staging_cap = bytes;
  }
  if (!ctx->staging_event) NRS_BHIP(ctx, hipEventCreateWithFlags(&ctx->staging_event, hipEventDisableTiming));
  *host = static_cast<char*>(ctx->staging);
  return NRS_OK;
}

// Side streams and events of the context (created once, before any capture).
nrs_status aux_ready(nrs_ctx* ctx) {
  if (ctx->fork_ev) return NRS_OK;
  for (int j = 0; j < nrs_ctx::kAux; ++j) {
    NRS_BHIP(ctx, hipStreamCreateWithFlags(&ctx->aux[j], hipStreamNonBlocking));
    NRS_BHIP(ctx, hipEventCreateWithFlags(&ctx->join_ev[j], hipEventDisableTiming));
  }
  NRS_BHIP(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  return NRS_OK;
}

// The side streams wait for everything queued so far on the context's stream.
nrs_status fork_aux(nrs_ctx* ctx) {
  NRS_BHIP(ctx, hipEventRecord(ctx->fork_ev, ctx->stream));
  for (int j = 0; j < nrs_ctx::kAux; ++j)
    NRS_BHIP(ctx, hipStreamWaitEvent(ctx->aux[j], ctx->fork_ev, 0));
  return NRS_OK;
}

// The context's stream waits for everything queued on the side streams.
nrs_status join_aux(nrs_ctx* ctx) {
  for (int j = 0; j < nrs_ctx::kAux; ++j) {
    NRS_BHIP(ctx, hipEventRecord(ctx->join_ev[j], ctx->aux[j]));
    NRS_BHIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->join_ev[j], 0));
  }
  return NRS_OK;
}

// Stream of system k's per-system kernels between a fork and a join.
hipStream_t lane_stream(const nrs_ctx* ctx, int k) {
  const int j = k % (nrs_ctx::kAux + 1);
  return j == 0 ? ctx->stream : ctx->aux[j - 1];
}

// Host descriptors (systems, ticket prefixes) of a batch layout, in bytes.
size_t desc_bytes(const BatchLayout& L, int32_t B) {
  return sizeof(LuSys<float>) * B + sizeof(TrsvSys<float>) * B +
         sizeof(int32_t) * (L.lu_pref_h.size() + L.tr_pref_h.size());
}

// Enqueue the whole batched solve on the context's stream.  h: pinned host
// buffer for the descriptors (NULL: the context's staging buffer, reuse
// fenced by an event); nothing here synchronises, so it can be captured.
nrs_status enqueue_batch(nrs_ctx* ctx, int32_t B, const nrs_problem* problems,
                         const double* const* u, const double* const* ftext, int32_t max_refine,
                         double tol, bool norm, BatchLayout& L, char* h, bool record_event,
                         double* const* sol) {
  nrs_status st = NRS_OK;
  hipStream_t s = ctx->stream;
  // ---- descriptors -> device (one pinned staging copy) ----
  std::vector<LuSys<float>> lus(B);
  std::vector<TrsvSys<float>> trs(B);
  for (int k = 0; k < B; ++k) {
    const nrs_problem& p = problems[k];
    const int64_t n = 3 * p.N + 6 * (int64_t)p.M;
    SolveBuffers& sb = L.sb[k];
    lus[k].A = sb.A32;
    lus[k].lda = sb.lda;
    lus[k].n = n;
    lus[k].nt = lu_tiles_nt(n);
    lus[k].lperm = sb.perm;
    lus[k].ipiv = sb.ipiv;
    lus[k].done = sb.lu_done;
    lus[k].sing = &sb.st->singular;
    trs[k].LU = sb.A32;
    trs[k].lda = sb.lda;
    trs[k].n = n;
    trs[k].x = sb.d32;
    trs[k].rhs = reinterpret_cast<const float*>(sb.r);
    trs[k].perm = sb.perm;
    trs[k].flags = sb.tsync + 2;
    trs[k].epoch = trsv_epoch(sb.tsync, n);
    trs[k].xp = trsv_xp(sb.tsync, n);
    trs[k].stop = &sb.st->stop;
  }
  const size_t b_lu = sizeof(LuSys<float>) * B, b_tr = sizeof(TrsvSys<float>) * B;
  const size_t b_lp = sizeof(int32_t) * L.lu_pref_h.size(), b_tp = sizeof(int32_t) * L.tr_pref_h.size();
  if (!h) {
    if ((st = stage(ctx, b_lu + b_tr + b_lp + b_tp, &h))) return st;
  }
  std::memcpy(h, lus.data(), b_lu);
  std::memcpy(h + b_lu, trs.data(), b_tr);
  std::memcpy(h + b_lu + b_tr, L.lu_pref_h.data(), b_lp);
  std::memcpy(h + b_lu + b_tr + b_lp, L.tr_pref_h.data(), b_tp);
  NRS_BHIP(ctx, hipMemcpyAsync(L.lusys, h, b_lu, hipMemcpyHostToDevice, s));
  NRS_BHIP(ctx, hipMemcpyAsync(L.trsys, h + b_lu, b_tr, hipMemcpyHostToDevice, s));
  NRS_BHIP(ctx, hipMemcpyAsync(L.lu_pref, h + b_lu + b_tr, b_lp, hipMemcpyHostToDevice, s));
  NRS_BHIP(ctx, hipMemcpyAsync(L.tr_pref, h + b_lu + b_tr + b_lp, b_tp, hipMemcpyHostToDevice, s));
  if (record_event) NRS_BHIP(ctx, hipEventRecord(ctx->staging_event, s));
  NRS_BHIP(ctx, launch_fill_i32(L.ctl, 0, 8, s));

  // ---- per system: layout, right-hand side, FP32 assembly (systems spread
  // over the side streams) ----
  if ((st = fork_aux(ctx))) return st;
  for (int k = 0; k < B; ++k) {
    const nrs_problem& p = problems[k];
    SolveBuffers& sb = L.sb[k];
    const int64_t n = 3 * p.N + 6 * (int64_t)p.M;
    hipStream_t s = lane_stream(ctx, k);
    NRS_BHIP(ctx, launch_solve_begin(sb.st, NRS_FP32_IR, sb.tsync, trsv_sync_ints(n), sb.lu_done,
                                     lu_done_flag_ints(n), s));
    NRS_BHIP(ctx, launch_build_csr(p.N, p.Q, p.X, p.w, p.nu, sb.srt, sb.st, s));
    // the right-hand side, its FP32 copy and the body check in one launch
    NRS_BHIP(ctx, launch_rhs(p.N, p.M, u[k], ftext ? ftext[k] : nullptr, sb.b, s,
                             reinterpret_cast<float*>(sb.r), p.body, sb.st));
    NRS_BHIP(ctx, launch_assemble<float>(p, sb.srt, sb.A32, sb.lda, s,
                                         asm_shape_for(ctx, p.N, p.Q, 32)));
    if (norm) NRS_BHIP(ctx, launch_anorm32(n, sb.A32, sb.lda, sb.st, sb.red, s));
  }
  if ((st = join_aux(ctx))) return st;

  // ---- every factorisation in one launch ----
  LuBatch<float> lb;
  std::memset(&lb.one, 0, sizeof(lb.one));
  lb.sys = L.lusys;
  lb.pref = L.lu_pref;
  lb.B = B;
  lb.nbands = L.nbands;
  lb.total = L.lu_total;
  NRS_BHIP(ctx, launch_lu_tiles<float>(lb, L.ctl, s));

  TrsvBatch<float> tb;
  std::memset(&tb.one, 0, sizeof(tb.one));
  tb.sys = L.trsys;
  tb.pref = L.tr_pref;
  tb.B = B;
  tb.nsteps = L.nsteps;
  tb.total = L.tr_total;

  // ---- x0 = (LU)^-1 b, then refinement sweeps ----
  NRS_BHIP(ctx, launch_trsv_batch<float>(tb, 1, L.ctl + 4, L.ctl + 6, s));
  if ((st = fork_aux(ctx))) return st;
  for (int k = 0; k < B; ++k)
    NRS_BHIP(ctx, launch_ir_update32(3 * problems[k].N + 6 * (int64_t)problems[k].M, sol[k],
                                     L.sb[k].d32, tol, 1, L.sb[k].st, lane_stream(ctx, k)));
  for (int it = 0; it < max_refine; ++it) {
    // the FP64 residual of system k follows its update on the same stream
    for (int k = 0; k < B; ++k) {
      const nrs_problem& p = problems[k];
      SolveBuffers& sb = L.sb[k];
      const int64_t n = 3 * p.N + 6 * (int64_t)p.M;
      hipStream_t sk = lane_stream(ctx, k);
      NRS_BHIP(ctx, launch_apply(p, sb.srt, sol[k], sb.d64, sb.part, sb.chunks, &sb.st->stop, sk));
      NRS_BHIP(ctx, launch_ir_residual2(n, sb.b, sb.d64, sol[k], nullptr,
                                        reinterpret_cast<float*>(sb.r), nullptr, sb.st, 0, sk));
    }
    if ((st = join_aux(ctx))) return st;
    NRS_BHIP(ctx, launch_trsv_batch<float>(tb, 1, L.ctl + 4, L.ctl + 6, s));
    if ((st = fork_aux(ctx))) return st;
    for (int k = 0; k < B; ++k)
      NRS_BHIP(ctx, launch_ir_update32(3 * problems[k].N + 6 * (int64_t)problems[k].M, sol[k],
                                       L.sb[k].d32, tol, 0, L.sb[k].st, lane_stream(ctx, k)));
  }
  if ((st = join_aux(ctx))) return st;
  return NRS_OK;
}

constexpr size_t kMaxGraphs = 8;

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Hash of everything a captured batch depends on: sizes, every pointer,
// eps / mu, the workspace and the refinement settings.
uint64_t batch_key(int32_t B, const nrs_problem* pb, const double* const* u,
                   const double* const* ftext, double* const* sol, const void* ws,
                   size_t ws_bytes, int32_t max_refine, double tol) {
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, &B, sizeof(B));
  for (int k = 0; k < B; ++k) {
    h = fnv(h, &pb[k], sizeof(nrs_problem));
    h = fnv(h, &u[k], sizeof(u[k]));
    const double* f = ftext ? ftext[k] : nullptr;
    h = fnv(h, &f, sizeof(f));
    h = fnv(h, &sol[k], sizeof(sol[k]));
  }
  h = fnv(h, &ws, sizeof(ws));
  h = fnv(h, &ws_bytes, sizeof(ws_bytes));
  h = fnv(h, &max_refine, sizeof(max_refine));
  h = fnv(h, &tol, sizeof(tol));
  return h;
}

// Replay the graph captured for these arguments, capturing it first if it
// is new.  Every launch and copy of the asynchronous batched solve is in the
// graph; the descriptors come from a pinned buffer owned by the entry.
nrs_status graph_batch(nrs_ctx* ctx, int32_t B, const nrs_problem* problems,
                       const double* const* u, const double* const* ftext, int32_t max_refine,
                       double tol, void* ws, size_t ws_bytes, BatchLayout& L,
                       double* const* sol) {
  hipStream_t s = ctx->stream;
  const uint64_t key = batch_key(B, problems, u, ftext, sol, ws, ws_bytes, max_refine, tol);
  for (auto& g : ctx->graphs)
    if (g.key == key) {
      NRS_BHIP(ctx, hipGraphLaunch(g.exec, s));
      return NRS_OK;
    }
  void* hd = nullptr;
  NRS_BHIP(ctx, hipHostMalloc(&hd, desc_bytes(L, B)));
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    hipHostFree(hd);
    return bfail(ctx, NRS_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  const nrs_status st = enqueue_batch(ctx, B, problems, u, ftext, max_refine, tol, false, L,
                                      static_cast<char*>(hd), false, sol);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (st != NRS_OK || e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    hipHostFree(hd);
    if (st != NRS_OK) return st;
    return bfail(ctx, NRS_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    hipHostFree(hd);
    return bfail(ctx, NRS_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  if (ctx->graphs.size() >= kMaxGraphs) {
    NRS_BHIP(ctx, hipStreamSynchronize(s));
    hipGraphExecDestroy(ctx->graphs.front().exec);
    hipHostFree(ctx->graphs.front().host_desc);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back({key, exec, hd});
  NRS_BHIP(ctx, hipGraphLaunch(exec, s));
  return NRS_OK;
}

}  // namespace

extern "C" {

nrs_status nrs_solve_batched_workspace_size(nrs_ctx* ctx, int32_t B, const nrs_problem* problems,
                                            int32_t method, size_t* bytes) {
  nrs_status st = check_batch(ctx, B, problems);
  if (st) return st;
  if (!bytes) return bfail(ctx, NRS_E_ARG, "bytes is NULL");
  if (method != NRS_FP32_IR) return bfail(ctx, NRS_E_UNSUPPORTED, "batches use NRS_FP32_IR");
  Arena ar(nullptr, 0);
  BatchLayout L;
  carve_batch(ar, B, problems, L);
  *bytes = ar.used + 256;
  return NRS_OK;
}

nrs_status nrs_solve_batched(nrs_ctx* ctx, int32_t B, const nrs_problem* problems,
                             const double* const* u, const double* const* ftext,
                             const nrs_options* opt, void* ws, size_t ws_bytes,
                             double* const* sol, nrs_info* infos) {
  if (!ctx) return NRS_E_ARG;
  NRS_BHIP(ctx, hipSetDevice(ctx->device));
  nrs_status st = check_batch(ctx, B, problems);
  if (st) return st;
  if (!u || !sol) return bfail(ctx, NRS_E_ARG, "u and sol arrays required");
  for (int s = 0; s < B; ++s)
    if (!u[s] || !sol[s]) return bfail(ctx, NRS_E_ARG, "u[s] and sol[s] required");
  nrs_options o = {};
  o.method = NRS_FP32_IR;
  if (opt) o = *opt;
  if (o.method != NRS_FP32_IR) return bfail(ctx, NRS_E_UNSUPPORTED, "batches use NRS_FP32_IR");
  // refinement converges in one or two sweeps on these systems; the default
  // cap keeps the asynchronous form from queueing sweeps that would only
  // find every system converged
  const int32_t max_refine = o.max_refine > 0 ? o.max_refine : 3;
  const double tol = o.tol > 0 ? o.tol : 1e-9;
  Arena ar(ws, ws_bytes);
  BatchLayout L;
  if (!carve_batch(ar, B, problems, L)) return bfail(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t s = ctx->stream;
  if ((st = aux_ready(ctx))) return st;

  if (o.graph) {
    if (infos) return bfail(ctx, NRS_E_ARG, "graph replay is asynchronous: pass infos = NULL");
    if (!s) return bfail(ctx, NRS_E_UNSUPPORTED, "graph capture needs a non-default stream");
    return graph_batch(ctx, B, problems, u, ftext, max_refine, tol, ws, ws_bytes, L, sol);
  }
  if ((st = enqueue_batch(ctx, B, problems, u, ftext, max_refine, tol, infos != nullptr, L,
                          nullptr, true, sol)))
    return st;
  if (!infos) return NRS_OK;

  // ---- synchronous report: final FP64 backward error of every system ----
  if ((st = fork_aux(ctx))) return st;
  for (int k = 0; k < B; ++k) {
    const nrs_problem& p = problems[k];
    SolveBuffers& sb = L.sb[k];
    const int64_t n = 3 * p.N + 6 * (int64_t)p.M;
    hipStream_t sk = lane_stream(ctx, k);
    NRS_BHIP(ctx, launch_apply(p, sb.srt, sol[k], sb.d64, sb.part, sb.chunks, nullptr, sk));
    NRS_BHIP(ctx, launch_ir_residual2(n, sb.b, sb.d64, sol[k], sb.r, nullptr, nullptr, sb.st, 1, sk));
  }
  if ((st = join_aux(ctx))) return st;
  NRS_BHIP(ctx, hipStreamSynchronize(s));
  int32_t ctl_h[8];
  NRS_BHIP(ctx, hipMemcpy(ctl_h, L.ctl, sizeof(ctl_h), hipMemcpyDeviceToHost));
  std::vector<SolveState> hs(B);
  for (int k = 0; k < B; ++k)
    NRS_BHIP(ctx, hipMemcpy(&hs[k], L.sb[k].st, sizeof(SolveState), hipMemcpyDeviceToHost));
  if (ctl_h[2] || ctl_h[6])
    return bfail(ctx, NRS_E_HIP, "batched LU / solve: a bounded wait timed out");
  nrs_status worst = NRS_OK;
  std::vector<int> redo;
  for (int k = 0; k < B; ++k) {
    nrs_info& inf = infos[k];
    inf.method_used = NRS_FP32_IR;
    inf.fell_back = 0;
    inf.iterations = hs[k].iterations;
    inf.singular = hs[k].singular;
    inf.backward_error = hs[k].bwd;
    inf.correction = hs[k].corr;
    if (hs[k].nonfinite == 2)
      return bfail(ctx, NRS_E_ARG, "problem " + std::to_string(k) +
                                       ": nu outside [0, N) or body outside [-1, M)");
    const bool ok = hs[k].converged && !hs[k].failed && !hs[k].nonfinite;
    if (!ok) redo.push_back(k);
  }
  // Systems that did not converge are solved again one by one in FP64 with
  // partial pivoting; the workspace is reused from its start (the batched
  // work is complete).
  for (int k : redo) {
    if (o.no_fallback) {
      worst = NRS_E_NOT_CONVERGED;
      continue;
    }
    const nrs_problem& p = problems[k];
    if (solve_workspace_bytes(p.N, p.Q, p.M, NRS_FP64_LU) > ws_bytes)
      return bfail(ctx, NRS_E_WORKSPACE, "workspace too small for the FP64 fallback");
    nrs_options o64 = o;
    o64.method = NRS_FP64_LU;
    nrs_info i64 = {};
    st = nrs_solve(ctx, &p, u[k], ftext ? ftext[k] : nullptr, &o64, ws, ws_bytes, sol[k], &i64);
    infos[k] = i64;
    infos[k].fell_back = 1;
    if (st != NRS_OK) worst = st;
  }
  if (worst == NRS_E_NOT_CONVERGED) bfail(ctx, worst, "refinement did not converge (no fallback)");
  return worst;
}

}  // extern "C"
