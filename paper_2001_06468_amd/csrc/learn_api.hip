// C ABI of the learned warm start (include/nrs.h): validation and launches.
#include <string>

#include "nrs_internal.h"

using namespace nrs;

namespace {

#define NRS_LHIP(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return set_error(ctx, NRS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

nrs_status begin(nrs_ctx* ctx) {
  if (!ctx) return NRS_E_ARG;
  NRS_LHIP(ctx, hipSetDevice(ctx->device));
  return ctx_dev_flags(ctx);
}

size_t grad_ws_bytes(int32_t nsel) {
  return (size_t)nsel * (kMlpParams + 1) * sizeof(float) + 256;
}

size_t warm_ws_bytes(int64_t N, int32_t M) {
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(7 * N * sizeof(float)) + up(3 * N * sizeof(float)) + up(6 * (size_t)M * sizeof(float));
}

}  // namespace

extern "C" {

int64_t nrs_mlp_param_count(void) { return kMlpParams; }

nrs_status nrs_mlp_body_offsets(nrs_ctx* ctx, int64_t N, const int32_t* body, int32_t M,
                                int32_t* body_off) {
  nrs_status st = begin(ctx);
  if (st) return st;
  if (N <= 0 || M <= 0 || !body || !body_off) return set_error(ctx, NRS_E_ARG, "bad body map");
  int32_t* err = ctx->dflags + 1;
  int32_t* starts = ctx->dflags + 2;
  hipError_t e = launch_fill_i32(err, 0, 1, ctx->stream);
  if (e == hipSuccess) e = launch_body_off(N, M, body, body_off, starts, err, ctx->stream);
  int32_t h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess)
    return set_error(ctx, NRS_E_HIP, std::string("body offsets: ") + hipGetErrorString(e));
  if (h)
    return set_error(ctx, NRS_E_ARG,
                     "each body needs one contiguous run of at most 256 points, bodies in order");
  return NRS_OK;
}

nrs_status nrs_mlp_features(nrs_ctx* ctx, int64_t N, const double* x, const double* u,
                            const double* s, const int32_t* body, int32_t M, const double* Y,
                            float* phi) {
  nrs_status st = begin(ctx);
  if (st) return st;
  if (N <= 0 || M < 0 || !x || !u || !s || !body || !phi || (M > 0 && !Y))
    return set_error(ctx, NRS_E_ARG, "bad feature arguments");
  NRS_LHIP(ctx, launch_features(N, x, u, s, body, M, Y, phi, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_mlp_forward(nrs_ctx* ctx, const float* theta, int64_t N, int32_t M,
                           const int32_t* body_off, const int32_t* sel, int32_t nsel,
                           const float* phi, float* y, float* z) {
  nrs_status st = begin(ctx);
  if (st) return st;
  const int32_t nb = sel ? nsel : M;
  if (!theta || !body_off || !phi || !y || !z || N <= 0 || M <= 0 || nb <= 0)
    return set_error(ctx, NRS_E_ARG, "bad forward arguments");
  NRS_LHIP(ctx, launch_mlp_forward(theta, nb, M, N, body_off, sel, phi, y, z, ctx->dflags,
                                   ctx->stream));
  return NRS_OK;
}

nrs_status nrs_mlp_grad_workspace_size(int32_t nsel, size_t* bytes) {
  if (nsel <= 0 || !bytes) return NRS_E_ARG;
  *bytes = grad_ws_bytes(nsel);
  return NRS_OK;
}

nrs_status nrs_mlp_grad(nrs_ctx* ctx, const float* theta, int64_t N, int32_t M,
                        const int32_t* body_off, const int32_t* sel, int32_t nsel,
                        const float* phi, const float* t_pt, const float* t_body, float* grad,
                        void* ws, size_t ws_bytes) {
  nrs_status st = begin(ctx);
  if (st) return st;
  const int32_t nb = sel ? nsel : M;
  if (!theta || !body_off || !phi || !t_pt || !t_body || !grad || N <= 0 || M <= 0 || nb <= 0)
    return set_error(ctx, NRS_E_ARG, "bad gradient arguments");
  if (!ws || ws_bytes < grad_ws_bytes(nb)) return set_error(ctx, NRS_E_WORKSPACE, "workspace too small");
  NRS_LHIP(ctx, launch_mlp_grad(theta, M, N, body_off, sel, nb, phi, t_pt, t_body,
                                static_cast<float*>(ws), grad, ctx->dflags, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_adam_step(nrs_ctx* ctx, int64_t count, float* theta, const float* grad, float* m,
                         float* v, int32_t step, float lr, float beta1, float beta2, float eps) {
  nrs_status st = begin(ctx);
  if (st) return st;
  if (count <= 0 || !theta || !grad || !m || !v || step < 1 || !(lr > 0.f) ||
      !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return set_error(ctx, NRS_E_ARG, "bad Adam arguments");
  NRS_LHIP(ctx, launch_adam(count, theta, grad, m, v, step, lr, beta1, beta2, eps, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_mlp_targets(nrs_ctx* ctx, int64_t N, int32_t M, const int32_t* body,
                           const double* Y, const double* sol, const double* scales,
                           float* t_pt, float* t_body) {
  nrs_status st = begin(ctx);
  if (st) return st;
  if (N <= 0 || M <= 0 || !body || !Y || !sol || !scales || !t_pt || !t_body)
    return set_error(ctx, NRS_E_ARG, "bad target arguments");
  if (!(scales[0] > 0) || !(scales[1] > 0) || !(scales[2] > 0))
    return set_error(ctx, NRS_E_ARG, "scales must be positive");
  NRS_LHIP(ctx, launch_targets(N, M, body, Y, sol, scales, t_pt, t_body, ctx->stream));
  return NRS_OK;
}

nrs_status nrs_mlp_warm_start_workspace_size(int64_t N, int32_t M, size_t* bytes) {
  if (N <= 0 || M <= 0 || !bytes) return NRS_E_ARG;
  *bytes = warm_ws_bytes(N, M) + 256;
  return NRS_OK;
}

nrs_status nrs_mlp_warm_start(nrs_ctx* ctx, const float* theta, const double* scales, int64_t N,
                              int32_t M, const int32_t* body, const int32_t* body_off,
                              const double* x, const double* u, const double* s,
                              const double* Y, double* x0, void* ws, size_t ws_bytes) {
  nrs_status st = begin(ctx);
  if (st) return st;
  if (!theta || !scales || N <= 0 || M <= 0 || !body || !body_off || !x || !u || !s || !Y || !x0)
    return set_error(ctx, NRS_E_ARG, "bad warm-start arguments");
  if (!(scales[0] > 0) || !(scales[1] > 0) || !(scales[2] > 0))
    return set_error(ctx, NRS_E_ARG, "scales must be positive");
  Arena ar(ws, ws_bytes);
  float* phi = ar.take<float>(7 * N);
  float* y = ar.take<float>(3 * N);
  float* z = ar.take<float>(6 * (size_t)M);
  if (ar.overflow) return set_error(ctx, NRS_E_WORKSPACE, "workspace too small");
  hipStream_t sm = ctx->stream;
  NRS_LHIP(ctx, launch_features(N, x, u, s, body, M, Y, phi, sm));
  NRS_LHIP(ctx, launch_mlp_forward(theta, M, M, N, body_off, nullptr, phi, y, z, ctx->dflags, sm));
  NRS_LHIP(ctx, launch_to_lab(N, M, body, Y, y, z, scales, x0, sm));
  return NRS_OK;
}

nrs_status nrs_mlp_status(nrs_ctx* ctx, int32_t* flags) {
  nrs_status st = begin(ctx);
  if (st) return st;
  if (!flags) return set_error(ctx, NRS_E_ARG, "flags is NULL");
  NRS_LHIP(ctx, hipMemcpyAsync(flags, ctx->dflags, sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
  NRS_LHIP(ctx, launch_fill_i32(ctx->dflags, 0, 1, ctx->stream));
  NRS_LHIP(ctx, hipStreamSynchronize(ctx->stream));
  return NRS_OK;
}

}  // extern "C"
