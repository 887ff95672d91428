// Mixed-precision iterative refinement (FP32 factors, FP64 residual and
// update), status bookkeeping, and the RK4 time-stepping kernels (Sec. 4:
// Y' = F(Y, t) with Y = [X0; B]).
#include "nrs_internal.h"

namespace nrs {

namespace {

constexpr int kRedThreads = 1024;

__device__ inline double block_max(double v, double* sh) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  if (tid < 64) {
    double w = tid < (int)(blockDim.x >> 6) ? sh[tid] : 0.0;
    for (int off = 32; off > 0; off >>= 1) w = fmax(w, __shfl_xor(w, off));
    if (tid == 0) sh[0] = w;
  }
  __syncthreads();
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline bool finite(double v) { return v == v && fabs(v) <= 1.7976931348623157e308; }

__global__ void k_state_init(SolveState* st, int32_t method) {
  if (threadIdx.x == 0) {
    SolveState z = {};
    z.method_used = method;
    *st = z;
  }
}

// The start of a solve in one launch: the status record, and the
// triangular-solve and tile-LU synchronisation words zeroed.
__global__ void k_solve_begin(SolveState* st, int32_t method, int32_t* __restrict__ a, int64_t na,
                              int32_t* __restrict__ b, int64_t nb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) {
    SolveState z = {};
    z.method_used = method;
    *st = z;
  }
  if (i < na) a[i] = 0;
  if (i < nb) b[i] = 0;
}

// |A|_inf = max_i sum_j |a_ij| (column-major).  Stage 1: thread = row,
// grid.y = column chunk, partial sums part[chunk][row]; stage 2: per-row sum
// of the chunks in order and block maxima; stage 3: maximum of the maxima.
template <class T>
__global__ void k_rowsum(int64_t n, const T* __restrict__ A, int64_t lda, int64_t cw,
                         double* __restrict__ part) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = blockIdx.y * cw, j1 = min<int64_t>(n, j0 + cw);
  double s = 0.0;
  for (int64_t j = j0; j < j1; ++j) s += fabs((double)A[i + j * lda]);
  part[blockIdx.y * n + i] = s;
}

__global__ void k_rowsum_rows(int64_t n, int64_t chunks, const double* __restrict__ part,
                              double* __restrict__ red) {
  __shared__ double sh[64];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n)
    for (int64_t c = 0; c < chunks; ++c) s += part[c * n + i];
  const double m = block_max(s, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = m;
}

__global__ void k_rowsum_final(int nblk, const double* red, SolveState* st) {
  __shared__ double sh[64];
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v = fmax(v, red[i]);
  v = block_max(v, sh);
  if (threadIdx.x == 0) st->anorm = v;
}

// Equilibration of the FP32 matrix (row, then column scaling by powers of
// two, so that the scaled matrix D_r A D_c is exact and the largest entry of
// every row and column has magnitude in [1, 2)):
//   r_i = max_j |a_ij|,  dr_i = 2^-floor(log2 r_i);
//   c_j = max_i dr_i |a_ij|,  dc_j = 2^-floor(log2 c_j);   (1 for zero rows / columns)
// Row maxima: thread = row over a chunk of 64 columns, combined with an
// integer atomic maximum on the FP32 bit patterns (non-negative values order
// as their bits).
__device__ inline float pow2_scale(float v) {
  return v > 0.f ? ldexpf(1.f, -ilogbf(v)) : 1.f;
}

__global__ void k_eq_rowmax(int64_t n, const float* __restrict__ A, int64_t lda,
                            uint32_t* __restrict__ rmax) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = (int64_t)blockIdx.y * 64, j1 = min<int64_t>(n, j0 + 64);
  float m = 0.f;
  for (int64_t j = j0; j < j1; ++j) m = fmaxf(m, fabsf(A[i + j * lda]));
  atomicMax(&rmax[i], __float_as_uint(m));
}

// One workgroup per column: c_j over the row-scaled column, then dc_j; the
// first n threads of the grid also turn the row maxima into dr.
__global__ void k_eq_colscale(int64_t n, const float* __restrict__ A, int64_t lda,
                              const uint32_t* __restrict__ rmax, float* __restrict__ dr,
                              float* __restrict__ dc) {
  __shared__ float sh[4];
  const int64_t j = blockIdx.x;
  const float* col = A + j * lda;
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    m = fmaxf(m, fabsf(col[i]) * pow2_scale(__uint_as_float(rmax[i])));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) dc[j] = pow2_scale(fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3])));
  const int64_t g = j * blockDim.x + threadIdx.x;
  if (g < n) dr[g] = pow2_scale(__uint_as_float(rmax[g]));
}

__global__ void k_eq_apply(int64_t n, float* __restrict__ A, int64_t lda,
                           const float* __restrict__ dr, const float* __restrict__ dc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = (int64_t)blockIdx.y * 64, j1 = min<int64_t>(n, j0 + 64);
  const float r = dr[i];
  for (int64_t j = j0; j < j1; ++j) A[i + j * lda] *= r * dc[j];
}

// b32 = FP32(scale * a) (scale may be NULL)
__global__ void k_convert_scaled(int64_t n, const double* __restrict__ a,
                                 const float* __restrict__ scale, float* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)(scale ? a[i] * (double)scale[i] : a[i]);
}

// r = b - A x (FP64), r in the correction precision; backward error from
// |r|, |x| (x is the solution the residual was taken at) and |b|.
__global__ __launch_bounds__(kRedThreads) void k_ir_residual(int64_t n,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ Ax,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ r,
                                                             float* __restrict__ r32,
                                                             double* __restrict__ r64,
                                                             SolveState* st, int force,
                                                             const float* __restrict__ eqr) {
  __shared__ double sh[64];
  if (!force && (st->converged || st->failed)) return;
  double rmax = 0.0, bmax = 0.0, xmax = 0.0;
  bool ok = true;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) {
    const double v = b[i] - Ax[i];
    ok = ok && finite(v);
    if (r) r[i] = v;
    if (r32) r32[i] = (float)(eqr ? v * (double)eqr[i] : v);
    if (r64) r64[i] = v;
    rmax = fmax(rmax, fabs(v));
    bmax = fmax(bmax, fabs(b[i]));
    xmax = fmax(xmax, fabs(x[i]));
  }
  rmax = block_max(rmax, sh);
  bmax = block_max(bmax, sh);
  xmax = block_max(xmax, sh);
  const int bad = __syncthreads_or(!ok);
  if (threadIdx.x == 0) {
    const double den = st->anorm * xmax + bmax;
    st->bwd = den > 0.0 ? rmax / den : 0.0;
    if (bad) {
      st->nonfinite = 1;
      st->failed = 1;
      st->stop = 1;
    }
  }
}

// x += d; convergence when |d|_inf <= tol |x|_inf or when the predicted next
// correction is (see below); failure when the correction stops contracting
// or turns non-finite.
template <class T>
__global__ __launch_bounds__(kRedThreads) void k_ir_update(int64_t n, double* __restrict__ x,
                                                           const T* __restrict__ d, double tol,
                                                           int32_t first, SolveState* st,
                                                           const float* __restrict__ eqc) {
  __shared__ double sh[64];
  if (st->converged || st->failed) return;
  double dmax = 0.0, xmax = 0.0;
  bool ok = true;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) {
    const double dv = eqc ? (double)d[i] * (double)eqc[i] : (double)d[i];
    const double xv = first ? dv : x[i] + dv;
    ok = ok && finite(xv);
    x[i] = xv;
    dmax = fmax(dmax, fabs(dv));
    xmax = fmax(xmax, fabs(xv));
  }
  dmax = block_max(dmax, sh);
  xmax = block_max(xmax, sh);
  const int bad = __syncthreads_or(!ok);
  if (threadIdx.x == 0) {
    const double c = xmax > 0.0 ? dmax / xmax : 0.0;
    st->iterations += 1;
    if (bad) {
      st->nonfinite = 1;
      st->failed = 1;
    } else if (!first) {
      // Converged when this correction, or the next one predicted from the
      // contraction rho = c / c_prev (the initial solve counts as a
      // correction of relative size 1), is below tol: with geometric
      // convergence the error left after this update is about c * rho.  The
      // first correction has no measured contraction (rho is then the
      // initial solve's relative change), and that prediction fell short of
      // the error left by up to ~30x on small channel and filament systems,
      // so it must clear tol by a factor of 10.
      const double rho = c / st->prev_corr;
      const double margin = st->prev_corr == 1.0 ? 10.0 : 1.0;
      if (c <= tol || (rho <= 0.5 && c * rho * margin <= tol)) {
        st->converged = 1;
      } else if (st->iterations > 2 && c > 0.9 * st->prev_corr) {
        st->failed = 1;
      }
    }
    st->prev_corr = first ? 1.0 : c;
    st->corr = c;
    st->stop = st->converged || st->failed;
  }
}

template <class T>
__global__ void k_convert(int64_t n, const double* __restrict__ a, T* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (T)a[i];
}


// body[m] must lie in [-1, M): anything else is an argument error.
// ---- time stepping ----

__global__ void k_rk_stage_state(int32_t M, const double* __restrict__ Y,
                                 const double* __restrict__ K, double a, double* __restrict__ Ys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 12 * M) Ys[i] = K ? Y[i] + a * K[i] : Y[i];
}

// dx0/dt = U; dB/dt = [Omega]x B (column i of B is body axis i).
__device__ inline void body_rates(int b, int64_t N, const double* __restrict__ Ys,
                                  const double* __restrict__ sol, double* __restrict__ K) {
  const double* uw = sol + 3 * N + 6 * (int64_t)b;
  const double* B = Ys + 12 * b + 3;
  double* k = K + 12 * b;
  k[0] = uw[0];
  k[1] = uw[1];
  k[2] = uw[2];
  const double o0 = uw[3], o1 = uw[4], o2 = uw[5];
  for (int c = 0; c < 3; ++c) {
    const double e0 = B[0 * 3 + c], e1 = B[1 * 3 + c], e2 = B[2 * 3 + c];
    k[3 + 0 * 3 + c] = o1 * e2 - o2 * e1;
    k[3 + 1 * 3 + c] = o2 * e0 - o0 * e2;
    k[3 + 2 * 3 + c] = o0 * e1 - o1 * e0;
  }
}

__global__ void k_rk_rates(int32_t M, int64_t N, const double* __restrict__ Ys,
                           const double* __restrict__ sol, double* __restrict__ K) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < M) body_rates(b, N, Ys, sol, K);
}

// Y += dt/6 (K1 + 2 K2 + 2 K3 + K4), then modified Gram-Schmidt on the
// columns of each body frame.
__global__ void k_rk_combine(int32_t M, double* __restrict__ Y, const double* __restrict__ K1,
                             const double* __restrict__ K2, const double* __restrict__ K3,
                             const double* __restrict__ K4, double dt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= M) return;
  double* y = Y + 12 * b;
  for (int i = 0; i < 12; ++i) {
    const int j = 12 * b + i;
    y[i] = y[i] + (dt / 6.0) * (K1[j] + 2.0 * K2[j] + 2.0 * K3[j] + K4[j]);
  }
  double c[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) c[k][r] = y[3 + 3 * r + k];
  double n0 = sqrt(c[0][0] * c[0][0] + c[0][1] * c[0][1] + c[0][2] * c[0][2]);
  for (int r = 0; r < 3; ++r) c[0][r] /= n0;
  double p = c[0][0] * c[1][0] + c[0][1] * c[1][1] + c[0][2] * c[1][2];
  for (int r = 0; r < 3; ++r) c[1][r] -= p * c[0][r];
  double n1 = sqrt(c[1][0] * c[1][0] + c[1][1] * c[1][1] + c[1][2] * c[1][2]);
  for (int r = 0; r < 3; ++r) c[1][r] /= n1;
  p = c[0][0] * c[2][0] + c[0][1] * c[2][1] + c[0][2] * c[2][2];
  for (int r = 0; r < 3; ++r) c[2][r] -= p * c[0][r];
  p = c[1][0] * c[2][0] + c[1][1] * c[2][1] + c[1][2] * c[2][2];
  for (int r = 0; r < 3; ++r) c[2][r] -= p * c[1][r];
  double n2 = sqrt(c[2][0] * c[2][0] + c[2][1] * c[2][1] + c[2][2] * c[2][2]);
  for (int r = 0; r < 3; ++r) c[2][r] /= n2;
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) y[3 + 3 * r + k] = c[k][r];
}

// Fold one stage's solve status into the step report.
__device__ inline void accumulate_state(SolveState* total, const SolveState* stage) {
  total->iterations = max(total->iterations, stage->iterations);
  total->failed |= stage->failed || (!stage->converged && stage->method_used != NRS_FP64_LU);
  total->singular |= stage->singular;
  total->nonfinite |= stage->nonfinite;
  total->fell_back |= stage->fell_back;
  total->bwd = fmax(total->bwd, stage->bwd);
  total->corr = fmax(total->corr, stage->corr);
  total->method_used = stage->method_used;
  total->converged = !total->failed;
}

__global__ void k_state_accumulate(SolveState* total, const SolveState* stage) {
  if (threadIdx.x == 0) accumulate_state(total, stage);
}

// Bodies up to which one workgroup ends a stage (12 state words per body).
constexpr int32_t kStageEndBodies = 1024;

// The end of an RK stage solve in one workgroup: the stage's status folded
// into the step report, the rates K of the free bodies from the solution
// (as k_rk_rates), and with Y != NULL the next stage's state Ys = Y + a K.
__global__ void k_stage_end(SolveState* total, const SolveState* stage, int32_t M, int64_t N,
                            double* __restrict__ Ys, const double* __restrict__ sol,
                            double* __restrict__ K, const double* __restrict__ Y, double a) {
  if (threadIdx.x == 0) accumulate_state(total, stage);
  for (int b = threadIdx.x; b < M; b += blockDim.x) body_rates(b, N, Ys, sol, K);
  if (Y) {
    __syncthreads();  // every rate is written and every read of Ys done
    for (int64_t i = threadIdx.x; i < 12 * (int64_t)M; i += blockDim.x) Ys[i] = Y[i] + a * K[i];
  }
}

inline dim3 grid1(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_state_init(SolveState* st, int32_t method, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, method);
  return hipGetLastError();
}

template <class T>
static hipError_t anorm(int64_t n, const T* A, int64_t lda, SolveState* st, double* scratch,
                        hipStream_t s) {
  const int64_t chunks = rowsum_chunks(n);
  const int64_t cw = (n + chunks - 1) / chunks;
  const unsigned nb = (unsigned)((n + 255) / 256);
  double* part = scratch;
  double* red = scratch + chunks * n;  // nb <= 1024 maxima for n <= 262144
  hipLaunchKernelGGL(k_rowsum<T>, dim3(nb, (unsigned)chunks), dim3(256), 0, s, n, A, lda, cw,
                     part);
  hipLaunchKernelGGL(k_rowsum_rows, dim3(nb), dim3(256), 0, s, n, chunks, part, red);
  hipLaunchKernelGGL(k_rowsum_final, dim3(1), dim3(256), 0, s, (int)nb, red, st);
  return hipGetLastError();
}

hipError_t launch_anorm32(int64_t n, const float* A, int64_t lda, SolveState* st, double* red,
                          hipStream_t s) {
  return anorm<float>(n, A, lda, st, red, s);
}

hipError_t launch_anorm64(int64_t n, const double* A, int64_t lda, SolveState* st, double* red,
                          hipStream_t s) {
  return anorm<double>(n, A, lda, st, red, s);
}

hipError_t launch_ir_residual2(int64_t n, const double* b, const double* Ax, const double* x,
                               double* r, float* r32, double* r64, SolveState* st, int force,
                               hipStream_t s, const float* eqr) {
  hipLaunchKernelGGL(k_ir_residual, dim3(1), dim3(kRedThreads), 0, s, n, b, Ax, x, r, r32, r64,
                     st, force, eqr);
  return hipGetLastError();
}

hipError_t launch_ir_update32(int64_t n, double* x, const float* d, double tol, int32_t first,
                              SolveState* st, hipStream_t s, const float* eqc) {
  hipLaunchKernelGGL(k_ir_update<float>, dim3(1), dim3(kRedThreads), 0, s, n, x, d, tol, first,
                     st, eqc);
  return hipGetLastError();
}

hipError_t launch_convert_f32(int64_t n, const double* a, float* b, hipStream_t s,
                              const float* scale) {
  if (scale)
    hipLaunchKernelGGL(k_convert_scaled, grid1(n, 256), dim3(256), 0, s, n, a, scale, b);
  else
    hipLaunchKernelGGL(k_convert<float>, grid1(n, 256), dim3(256), 0, s, n, a, b);
  return hipGetLastError();
}

hipError_t launch_equilibrate(int64_t n, float* A, int64_t lda, float* dr, float* dc,
                              uint32_t* rmax, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(rmax), 0, n, s);
  if (e != hipSuccess) return e;
  const dim3 g2((unsigned)((n + 255) / 256), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(k_eq_rowmax, g2, dim3(256), 0, s, n, A, lda, rmax);
  hipLaunchKernelGGL(k_eq_colscale, dim3((unsigned)n), dim3(256), 0, s, n, A, lda, rmax, dr, dc);
  hipLaunchKernelGGL(k_eq_apply, g2, dim3(256), 0, s, n, A, lda, dr, dc);
  return hipGetLastError();
}


hipError_t launch_rk_stage_state(int32_t M, const double* Y, const double* K, double a,
                                 double* Ys, hipStream_t s) {
  hipLaunchKernelGGL(k_rk_stage_state, grid1(12 * (int64_t)M, 256), dim3(256), 0, s, M, Y, K, a,
                     Ys);
  return hipGetLastError();
}

// ---- adaptive Dormand-Prince 5(4) ----

// out = Y + h sum_j c_j K_j over the 12M state entries (up to 7 stage rates).
__global__ void k_rk_lincomb(int64_t n, const double* __restrict__ Y, RkComb cb, double h,
                             double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < cb.count; ++j) acc += cb.c[j] * cb.K[j][i];
  out[i] = Y[i] + h * acc;
}

// RMS norm of the error estimate e = h sum_j e_j K_j scaled by
// atol + rtol max(|y|, |y_new|); one workgroup, fixed-order reduction.
__global__ __launch_bounds__(kRedThreads) void k_dp_error(int64_t n, const double* __restrict__ Y,
                                                         const double* __restrict__ Yn, RkComb cb,
                                                         double h, double rtol, double atol,
                                                         double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) {
    double e = 0.0;
    for (int j = 0; j < cb.count; ++j) e += cb.c[j] * cb.K[j][i];
    const double sc = atol + rtol * fmax(fabs(Y[i]), fabs(Yn[i]));
    const double q = h * e / sc;
    acc = fma(q, q, acc);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = n > 0 ? sqrt(sh[0] / (double)n) : 0.0;
}

hipError_t launch_rk_lincomb(int64_t n, const double* Y, const RkComb& cb, double h, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rk_lincomb, grid1(n, 256), dim3(256), 0, s, n, Y, cb, h, out);
  return hipGetLastError();
}

hipError_t launch_dp_error(int64_t n, const double* Y, const double* Yn, const RkComb& cb, double h,
                           double rtol, double atol, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_error, dim3(1), dim3(kRedThreads), 0, s, n, Y, Yn, cb, h, rtol, atol,
                     out);
  return hipGetLastError();
}

hipError_t launch_rk_combine(int32_t M, double* Y, const double* K1, const double* K2,
                             const double* K3, const double* K4, double dt, hipStream_t s) {
  hipLaunchKernelGGL(k_rk_combine, grid1(M, 64), dim3(64), 0, s, M, Y, K1, K2, K3, K4, dt);
  return hipGetLastError();
}

hipError_t launch_solve_begin(SolveState* st, int32_t method, int32_t* a, int64_t na, int32_t* b,
                              int64_t nb, hipStream_t s) {
  const int64_t m = std::max<int64_t>(1, std::max(na, nb));
  hipLaunchKernelGGL(k_solve_begin, grid1(m, 256), dim3(256), 0, s, st, method, a, na, b, nb);
  return hipGetLastError();
}

hipError_t launch_stage_end(SolveState* total, const SolveState* stage, int32_t M, int64_t N,
                            double* Ys, const double* sol, double* K, const double* Y, double a,
                            hipStream_t s) {
  if (M > kStageEndBodies) {  // many bodies: the three steps as full-grid launches
    hipLaunchKernelGGL(k_state_accumulate, dim3(1), dim3(64), 0, s, total, stage);
    hipLaunchKernelGGL(k_rk_rates, grid1(M, 256), dim3(256), 0, s, M, N, Ys, sol, K);
    if (Y)
      hipLaunchKernelGGL(k_rk_stage_state, grid1(12 * (int64_t)M, 256), dim3(256), 0, s, M, Y, K,
                         a, Ys);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_stage_end, dim3(1), dim3(256), 0, s, total, stage, M, N, Ys, sol, K, Y, a);
  return hipGetLastError();
}

}  // namespace nrs
