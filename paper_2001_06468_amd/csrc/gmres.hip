// Restarted GMRES(m) in FP64 on the stored operator (Saad and Schultz,
// 1986), used from a warm start (learned or previous solution) with the LU
// path as fallback.
//
// The operator is kept row-major (the transpose of the assembled column-major
// matrix) so one wavefront computes one row of A v with coalesced loads.  The
// Krylov basis V is row-major too, [n][64]: lane i of the wavefront that owns
// row r holds V[r][i], so the Gram-Schmidt dot products accumulate in
// registers next to the product that produced w[r].  Arnoldi uses classical
// Gram-Schmidt applied twice (CGS2).  Each step is three launches:
//   step1: w = A v_k (v_k = previous w / |w|, stored into V[:, k]) and
//          partial dots V^T w;
//   step2: w -= V h1, partial dots V^T w;
//   step3: w -= V h2, partial |w|^2;
// the last workgroup of each launch reduces the partials in a fixed order
// (deterministic) and step3's last workgroup also applies the Givens
// rotations, updates the residual estimate and decides whether the cycle
// stops.  Every kernel returns at once when the state says the solve is done
// or the cycle has stopped, so the host can queue steps ahead of the check.
#include <cmath>

#include "nrs_internal.h"

namespace nrs {
namespace {

constexpr int kThreads = 1024;
constexpr int kWavesG = kThreads / 64;
constexpr int kMaxBlocks = 256;     // one workgroup per CU at most: short partial lists

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double lane_h(const double* h, int lane, int k) {
  return lane <= k ? h[lane] : 0.0;
}

__device__ inline bool halted(const GmresState* st) {
  return st->done | st->stop | st->fail;
}

// y[r] = sum_c A[r][c] x[c] for one row, by one wavefront (result in every lane)
__device__ inline double row_dot(const double* __restrict__ Ar, const double* __restrict__ x,
                                 int64_t n, int lane) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t c = lane;
  for (; c + 192 < n; c += 256) {
    a0 = fma(Ar[c], x[c], a0);
    a1 = fma(Ar[c + 64], x[c + 64], a1);
    a2 = fma(Ar[c + 128], x[c + 128], a2);
    a3 = fma(Ar[c + 192], x[c + 192], a3);
  }
  for (; c < n; c += 64) a0 = fma(Ar[c], x[c], a0);
  return wave_sum_d((a0 + a1) + (a2 + a3));
}

// Last-workgroup detection: returns true in every thread of the workgroup
// that arrives last (partials of all workgroups are then visible).
__device__ inline bool last_block(int32_t* counter) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
  }
  return false;
}

// Sum partial[b][i] over the grid's blocks, i < cnt: 16 groups of 64 threads
// each add every 16th block (independent loads), then the group sums are
// added in a fixed order (deterministic).  Called by all threads.
__device__ inline void reduce_partials(const double* __restrict__ part, int nb, int cnt,
                                       double* __restrict__ out) {
  __shared__ double s_g[kWavesG][kGmresLd];
  const int i = threadIdx.x & 63, grp = threadIdx.x >> 6;
  double s0 = 0.0, s1 = 0.0;
  int b = grp;
  for (; b + kWavesG < nb; b += 2 * kWavesG) {
    s0 += part[(int64_t)b * kGmresLd + i];
    s1 += part[(int64_t)(b + kWavesG) * kGmresLd + i];
  }
  if (b < nb) s0 += part[(int64_t)b * kGmresLd + i];
  s_g[grp][i] = s0 + s1;
  __syncthreads();
  if (threadIdx.x < cnt) {
    double t = 0.0;
    for (int g = 0; g < kWavesG; ++g) t += s_g[g][threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// r = b - A x into w, |r|^2 partials; last block: beta, |b| (first call),
// convergence test and the start of a new cycle.
__global__ __launch_bounds__(kThreads) void k_gm_residual(GmresArgs a) {
  GmresState* st = a.st;
  if (st->done | st->fail) return;
  __shared__ double s_p[kWavesG][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc = 0.0, accb = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kWavesG + w; r < a.n;
       r += (int64_t)gridDim.x * kWavesG) {
    {
      const double ax = row_dot(a.AT + r * a.ld, a.x, a.n, lane);
      const double br = a.b[r];
      const double rr = br - ax;
      if (lane == 0) a.w0[r] = rr;
      acc = fma(rr, rr, acc);
      accb = fma(br, br, accb);
    }
  }
  if (lane == 0) {
    s_p[w][0] = acc;
    s_p[w][1] = accb;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int q = 0; q < kWavesG; ++q) s += s_p[q][threadIdx.x];
    a.part[(int64_t)blockIdx.x * kGmresLd + threadIdx.x] = s;
  }
  if (!last_block(&st->counter)) return;
  __shared__ double s_r[2];
  reduce_partials(a.part, gridDim.x, 2, s_r);
  __syncthreads();
  if (threadIdx.x == 0) {
    st->counter = 0;
    const double beta = sqrt(s_r[0]);
    if (st->bnorm < 0.0) st->bnorm = sqrt(s_r[1]);
    st->beta = beta;
    if (!isfinite(beta)) {
      st->fail = 1;
    } else if (beta <= st->tol * st->bnorm) {
      st->done = 1;
    } else {
      st->nrm = beta;
      st->g[0] = beta;
      st->k = 0;
      st->stop = 0;
      st->cur = 0;   // w0 holds the unnormalised first basis vector
    }
    st->halt = st->done | st->stop | st->fail;
  }
}

// Step 1 of Arnoldi step k: v_k = w_cur / nrm into V[:, k]; w_next = A v_k;
// partial dots V[:, 0..k]^T w_next.
__global__ __launch_bounds__(kThreads) void k_gm_step1(GmresArgs a) {
  GmresState* st = a.st;
  if (halted(st)) return;
  const int k = st->k;
  const double* __restrict__ vin = st->cur ? a.w1 : a.w0;
  double* __restrict__ wout = st->cur ? a.w0 : a.w1;
  const double s = 1.0 / st->nrm;
  __shared__ double s_p[kWavesG][kGmresLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kWavesG + w; r < a.n;
       r += (int64_t)gridDim.x * kWavesG) {
    {
      const double vr = vin[r] * s;
      const double y = row_dot(a.AT + r * a.ld, vin, a.n, lane) * s;
      double* Vr = a.V + r * kGmresLd;
      if (lane == 0) {
        Vr[k] = vr;
        wout[r] = y;
      }
      const double vi = lane < k ? Vr[lane] : (lane == k ? vr : 0.0);
      acc = fma(vi, y, acc);
    }
  }
  s_p[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    double t = 0.0;
    for (int q = 0; q < kWavesG; ++q) t += s_p[q][lane];
    a.part[(int64_t)blockIdx.x * kGmresLd + lane] = t;
  }
  if (!last_block(&st->counter)) return;
  reduce_partials(a.part, gridDim.x, k + 1, st->h1);
  __syncthreads();
  if (threadIdx.x == 0) st->counter = 0;
}

// Steps 2 and 3: w -= V h (h = h1 or h2), then partial dots (step 2) or the
// partial |w|^2 (step 3, whose last block finishes the Arnoldi step).
template <bool LAST>
__global__ __launch_bounds__(kThreads) void k_gm_orth(GmresArgs a) {
  GmresState* st = a.st;
  if (halted(st)) return;
  const int k = st->k;
  double* __restrict__ wv = st->cur ? a.w0 : a.w1;
  const double hl = lane_h(LAST ? st->h2 : st->h1, threadIdx.x & 63, k);
  __shared__ double s_p[kWavesG][kGmresLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kWavesG + w; r < a.n;
       r += (int64_t)gridDim.x * kWavesG) {
    {
      const double vi = lane <= k ? a.V[r * kGmresLd + lane] : 0.0;
      const double nw = wv[r] - wave_sum_d(vi * hl);
      if (lane == 0) wv[r] = nw;
      acc = LAST ? fma(nw, nw, acc) : fma(vi, nw, acc);
    }
  }
  s_p[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    double t = 0.0;
    for (int q = 0; q < kWavesG; ++q) t += s_p[q][lane];
    a.part[(int64_t)blockIdx.x * kGmresLd + lane] = t;
  }
  if (!last_block(&st->counter)) return;
  if (!LAST) {
    reduce_partials(a.part, gridDim.x, k + 1, st->h2);
    __syncthreads();
    if (threadIdx.x == 0) st->counter = 0;
    return;
  }
  __shared__ double s_n[1];
  reduce_partials(a.part, gridDim.x, 1, s_n);   // lane-0 column: every lane holds |w|^2
  __syncthreads();
  if (threadIdx.x != 0) return;
  st->counter = 0;
  // every lane's partial holds the same |w|^2 contribution of its rows; the
  // lane-0 column was summed above
  const double nrm = sqrt(s_n[0]);
  double* Hk = st->H + (int64_t)k * (kGmresLd + 1);
  for (int i = 0; i <= k; ++i) Hk[i] = st->h1[i] + st->h2[i];
  Hk[k + 1] = nrm;
  for (int i = 0; i < k; ++i) {
    const double t0 = st->cs[i] * Hk[i] + st->sn[i] * Hk[i + 1];
    Hk[i + 1] = -st->sn[i] * Hk[i] + st->cs[i] * Hk[i + 1];
    Hk[i] = t0;
  }
  const double den = hypot(Hk[k], Hk[k + 1]);
  double c = 1.0, sn = 0.0;
  if (den > 0.0) {
    c = Hk[k] / den;
    sn = Hk[k + 1] / den;
  }
  st->cs[k] = c;
  st->sn[k] = sn;
  Hk[k] = den;
  Hk[k + 1] = 0.0;
  st->g[k + 1] = -sn * st->g[k];
  st->g[k] = c * st->g[k];
  st->k = k + 1;
  st->iters += 1;
  st->nrm = nrm;
  st->cur ^= 1;
  if (!isfinite(nrm) || !isfinite(st->g[k + 1])) {
    st->fail = 1;
  } else if (fabs(st->g[k + 1]) <= st->tol * st->bnorm || nrm == 0.0 || k + 1 >= st->m ||
             st->iters >= st->max_iter) {
    st->stop = 1;
  }
  st->halt = st->done | st->stop | st->fail;
}

// End of a cycle: y = R^-1 g (upper triangular, k x k, solved redundantly in
// every block by wave 0), x += V[:, 0..k-1] y.
__global__ __launch_bounds__(kThreads) void k_gm_update(GmresArgs a) {
  GmresState* st = a.st;
  if (st->done | st->fail) return;
  const int k = st->k;
  if (k <= 0) return;
  __shared__ double s_y[kGmresLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (w == 0) {
    // lane i holds y_i; back substitution, one broadcast per column
    const int64_t ldh = kGmresLd + 1;
    double yi = lane < k ? st->g[lane] : 0.0;
    for (int j = k - 1; j >= 0; --j) {
      const double rjj = st->H[(int64_t)j * ldh + j];
      const double yj = __shfl(yi, j, 64) / rjj;
      if (lane == j) yi = yj;
      if (lane < j) yi -= st->H[(int64_t)j * ldh + lane] * yj;
    }
    s_y[lane] = lane < k ? yi : 0.0;
  }
  __syncthreads();
  const double yl = s_y[lane];
  const double* __restrict__ basis = a.Z ? a.Z : a.V;   // x += Z y (flexible) or V y
  for (int64_t r = (int64_t)blockIdx.x * kWavesG + w; r < a.n;
       r += (int64_t)gridDim.x * kWavesG) {
    {
      const double vi = lane < k ? basis[r * kGmresLd + lane] : 0.0;
      const double d = wave_sum_d(vi * yl);
      if (lane == 0) a.x[r] += d;
    }
  }
}

// ---- flexible GMRES (Saad, 1993) with the low-precision LU as right
// preconditioner: x = x0 + Z y with z_k = M^-1 v_k; the operator products
// A x and A z_k come from the matrix-free FP64 product, so no FP64 matrix is
// stored.  The Arnoldi bookkeeping (CGS2, Givens rotations, stop rules) is the
// same as above. ----

// r = b - Ax into w0, |r|^2 and |b|^2 partials (one row per thread); the last
// block decides convergence or starts a cycle, as k_gm_residual.
__global__ __launch_bounds__(kThreads) void k_fg_residual(GmresArgs a,
                                                         const double* __restrict__ Ax) {
  GmresState* st = a.st;
  if (st->done | st->fail) return;
  __shared__ double s_p[kWavesG][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc = 0.0, accb = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < a.n;
       r += (int64_t)gridDim.x * kThreads) {
    const double br = a.b[r];
    const double rr = br - Ax[r];
    a.w0[r] = rr;
    acc = fma(rr, rr, acc);
    accb = fma(br, br, accb);
  }
  acc = wave_sum_d(acc);
  accb = wave_sum_d(accb);
  if (lane == 0) {
    s_p[w][0] = acc;
    s_p[w][1] = accb;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int q = 0; q < kWavesG; ++q) t += s_p[q][threadIdx.x];
    a.part[(int64_t)blockIdx.x * kGmresLd + threadIdx.x] = t;
  }
  if (!last_block(&st->counter)) return;
  __shared__ double s_r[2];
  reduce_partials(a.part, gridDim.x, 2, s_r);
  __syncthreads();
  if (threadIdx.x == 0) {
    st->counter = 0;
    const double beta = sqrt(s_r[0]);
    if (st->bnorm < 0.0) st->bnorm = sqrt(s_r[1]);
    st->beta = beta;
    if (!isfinite(beta)) {
      st->fail = 1;
    } else if (beta <= st->tol * st->bnorm) {
      st->done = 1;
    } else {
      st->nrm = beta;
      st->g[0] = beta;
      st->k = 0;
      st->stop = 0;
      st->cur = 0;
    }
    st->halt = st->done | st->stop | st->fail;
  }
}

// v_k = w_cur / nrm into V[:, k], and its FP32 copy for the preconditioner.
__global__ void k_fg_begin(GmresArgs a, float* __restrict__ v32) {
  const GmresState* st = a.st;
  if (st->halt) return;
  const int k = st->k;
  const double* __restrict__ vin = st->cur ? a.w1 : a.w0;
  const double s = 1.0 / st->nrm;
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < a.n) {
    const double v = vin[r] * s;
    a.V[r * kGmresLd + k] = v;
    v32[r] = (float)(a.eqr ? v * (double)a.eqr[r] : v);
  }
}

// z_k = M^-1 v_k (FP32 result of the triangular solves) into Z[:, k] and zv.
__global__ void k_fg_zstore(GmresArgs a, const float* __restrict__ d32, double* __restrict__ zv) {
  const GmresState* st = a.st;
  if (st->halt) return;
  const int k = st->k;
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < a.n) {
    const double z = a.eqc ? (double)d32[r] * (double)a.eqc[r] : (double)d32[r];
    a.Z[r * kGmresLd + k] = z;
    zv[r] = z;
  }
}

// w = A z_k (given) into the next basis buffer; partial dots V[:, 0..k]^T w,
// reduced by the last block into h1 (the first Gram-Schmidt pass).
__global__ __launch_bounds__(kThreads) void k_fg_dots(GmresArgs a, const double* __restrict__ Aw) {
  GmresState* st = a.st;
  if (st->halt) return;
  const int k = st->k;
  double* __restrict__ wout = st->cur ? a.w0 : a.w1;
  __shared__ double s_p[kWavesG][kGmresLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kWavesG + w; r < a.n;
       r += (int64_t)gridDim.x * kWavesG) {
    const double y = Aw[r];
    if (lane == 0) wout[r] = y;
    const double vi = lane <= k ? a.V[r * kGmresLd + lane] : 0.0;
    acc = fma(vi, y, acc);
  }
  s_p[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    double t = 0.0;
    for (int q = 0; q < kWavesG; ++q) t += s_p[q][lane];
    a.part[(int64_t)blockIdx.x * kGmresLd + lane] = t;
  }
  if (!last_block(&st->counter)) return;
  reduce_partials(a.part, gridDim.x, k + 1, st->h1);
  __syncthreads();
  if (threadIdx.x == 0) st->counter = 0;
}

__global__ void k_fg_report(SolveState* st, const GmresState* g) {
  if (threadIdx.x == 0) {
    st->converged = g->done;
    st->failed = !g->done;
    st->iterations += g->iters;
    if (g->fail) st->nonfinite |= 1;
    st->corr = g->bnorm > 0.0 ? g->beta / g->bnorm : 0.0;
  }
}

// Row-major copy of a column-major matrix: AT[r * ld + c] = A[r + c * lda].
__global__ void k_transpose64(int64_t n, const double* __restrict__ A, int64_t lda,
                              double* __restrict__ AT, int64_t ld) {
  __shared__ double t[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    t[j][tx] = (r < n && c < n) ? A[r + c * lda] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + j, c = c0 + tx;
    if (r < n && c < n) AT[r * ld + c] = t[tx][j];
  }
}

// ---- rigid-body completion of an initial guess ----
//
// For body b with points m (r_m = x_m - x0_b) and weights W_m (or 1), the
// 6 x 6 system G v = h with G = sum W_m C_m^T C_m, C_m = [I | -[r_m]x],
// h = sum W_m (v_m, r_m x v_m) - target_b.  With v = f and W the patch
// weights, f_m - C_m v satisfies the force and torque balance rows exactly
// (projection).  With v = the velocity residual and W = 1, v are the (U,
// Omega) that fit the residual best in the least-squares sense.
constexpr int kMomThreads = 256;

__global__ __launch_bounds__(kMomThreads) void k_body_moments(
    int64_t N, int32_t M, const double* __restrict__ x, const double* __restrict__ Y,
    const int32_t* __restrict__ body, const double* __restrict__ W,
    const double* __restrict__ v, double vsign, const double* __restrict__ target,
    double* __restrict__ out) {
  const int b = blockIdx.x;
  if (b >= M) return;
  const double* y0 = Y + (int64_t)b * 12;
  double acc[27];   // G upper part (21) + h (6)
#pragma unroll
  for (int i = 0; i < 27; ++i) acc[i] = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += kMomThreads) {
    if (body[m] != b) continue;
    const double wm = W ? W[m] : 1.0;
    const double r0 = x[m] - y0[0], r1 = x[N + m] - y0[1], r2 = x[2 * N + m] - y0[2];
    const double v0 = vsign * v[m], v1 = vsign * v[N + m], v2 = vsign * v[2 * N + m];
    // C^T C = [[I, -[r]x], [[r]x, |r|^2 I - r r^T]]; stored row-major upper triangle
    const double rr = r0 * r0 + r1 * r1 + r2 * r2;
    const double Gm[6][6] = {
        {1, 0, 0, 0, r2, -r1},
        {0, 1, 0, -r2, 0, r0},
        {0, 0, 1, r1, -r0, 0},
        {0, -r2, r1, rr - r0 * r0, -r0 * r1, -r0 * r2},
        {r2, 0, -r0, -r1 * r0, rr - r1 * r1, -r1 * r2},
        {-r1, r0, 0, -r2 * r0, -r2 * r1, rr - r2 * r2}};
    int q = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i; j < 6; ++j) acc[q++] += wm * Gm[i][j];
    acc[21] += wm * v0;
    acc[22] += wm * v1;
    acc[23] += wm * v2;
    acc[24] += wm * (r1 * v2 - r2 * v1);
    acc[25] += wm * (r2 * v0 - r0 * v2);
    acc[26] += wm * (r0 * v1 - r1 * v0);
  }
  __shared__ double red[kMomThreads / 64][27];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const double t = wave_sum_d(acc[i]);
    if (lane == 0) red[w][i] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double G[6][7];
  int q = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      double t = 0.0;
      for (int k = 0; k < kMomThreads / 64; ++k) t += red[k][q];
      G[i][j] = G[j][i] = t;
      ++q;
    }
  for (int i = 0; i < 6; ++i) {
    double t = 0.0;
    for (int k = 0; k < kMomThreads / 64; ++k) t += red[k][21 + i];
    G[i][6] = t - (target ? target[(int64_t)b * 6 + i] : 0.0);
  }
  // a small ridge keeps a body whose points are (nearly) collinear solvable
  double dmax = 0.0;
  for (int i = 0; i < 6; ++i) dmax = fmax(dmax, G[i][i]);
  for (int i = 0; i < 6; ++i) G[i][i] += 1e-12 * dmax;
  // Gaussian elimination with partial pivoting on the 6 x 7 augmented matrix
  bool ok = true;
  for (int c = 0; c < 6; ++c) {
    int p = c;
    for (int i = c + 1; i < 6; ++i)
      if (fabs(G[i][c]) > fabs(G[p][c])) p = i;
    if (!(fabs(G[p][c]) > 0.0)) {
      ok = false;
      break;
    }
    if (p != c)
      for (int j = 0; j < 7; ++j) {
        const double t = G[c][j];
        G[c][j] = G[p][j];
        G[p][j] = t;
      }
    for (int i = c + 1; i < 6; ++i) {
      const double f = G[i][c] / G[c][c];
      for (int j = c; j < 7; ++j) G[i][j] -= f * G[c][j];
    }
  }
  double sol[6] = {0, 0, 0, 0, 0, 0};
  if (ok)
    for (int i = 5; i >= 0; --i) {
      double t = G[i][6];
      for (int j = i + 1; j < 6; ++j) t -= G[i][j] * sol[j];
      sol[i] = t / G[i][i];
    }
  for (int i = 0; i < 6; ++i) out[(int64_t)b * 6 + i] = sol[i];
}

// f_m -= a_b + c_b x r_m for the points of body b (v = (a, c) from k_body_moments)
__global__ void k_project_apply(int64_t N, int32_t M, const double* __restrict__ x,
                                const double* __restrict__ Y, const int32_t* __restrict__ body,
                                const double* __restrict__ ac, double* __restrict__ f) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int32_t b = body[m];
  if (b < 0 || b >= M) return;
  const double* y0 = Y + (int64_t)b * 12;
  const double* v = ac + (int64_t)b * 6;
  const double r0 = x[m] - y0[0], r1 = x[N + m] - y0[1], r2 = x[2 * N + m] - y0[2];
  f[m] -= v[0] + (v[4] * r2 - v[5] * r1);
  f[N + m] -= v[1] + (v[5] * r0 - v[3] * r2);
  f[2 * N + m] -= v[2] + (v[3] * r1 - v[4] * r0);
}

// out = b - A x (rows of the stored row-major operator), one wavefront per row
__global__ __launch_bounds__(kThreads) void k_gm_resid(int64_t n, const double* __restrict__ AT,
                                                        int64_t ld, const double* __restrict__ xv,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * kWavesG + w; r < n;
       r += (int64_t)gridDim.x * kWavesG) {
    {
      const double ax = row_dot(AT + r * ld, xv, n, lane);
      if (lane == 0) out[r] = b[r] - ax;
    }
  }
}

__global__ void k_gm_init(GmresState* st, double tol, int32_t m, int32_t max_iter) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->stop = 0;
    st->fail = 0;
    st->k = 0;
    st->iters = 0;
    st->cur = 0;
    st->counter = 0;
    st->m = m;
    st->max_iter = max_iter;
    st->tol = tol;
    st->bnorm = -1.0;
    st->beta = 0.0;
    st->nrm = 1.0;
    st->halt = 0;
    st->skip_true = 1;
  }
}

__global__ void k_gm_report(SolveState* st, const GmresState* g) {
  if (threadIdx.x == 0) {
    st->converged = g->done;
    st->failed = !g->done;
    st->iterations = g->iters;
    if (g->fail) st->nonfinite |= 1;
    st->corr = g->bnorm > 0.0 ? g->beta / g->bnorm : 0.0;
  }
}

}  // namespace

hipError_t launch_rigid_completion(int64_t N, int32_t M, const double* x, const double* Y,
                                   const int32_t* body, const double* W, const double* ftext,
                                   const double* AT, int64_t ld, const double* b, double* x0,
                                   double* res, double* small, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const int64_t n = 3 * N + 6 * (int64_t)M;
  const unsigned pb = (unsigned)((N + 255) / 256);
  // forces onto the force / torque balance
  hipLaunchKernelGGL(k_body_moments, dim3((unsigned)M), dim3(kMomThreads), 0, s, N, M, x, Y, body, W,
                     x0, 1.0, ftext, small);
  hipLaunchKernelGGL(k_project_apply, dim3(pb), dim3(256), 0, s, N, M, x, Y, body, small, x0);
  // (U, Omega) = least-squares rigid fit of -(u - A_s f)
  hipError_t e = launch_fill_f64(x0 + 3 * N, 0.0, 6 * (int64_t)M, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gm_resid, dim3((unsigned)gmres_blocks(n)), dim3(kThreads), 0, s, n, AT, ld,
                     x0, b, res);
  hipLaunchKernelGGL(k_body_moments, dim3((unsigned)M), dim3(kMomThreads), 0, s, N, M, x, Y, body,
                     nullptr, res, -1.0, nullptr, x0 + 3 * N);
  return hipGetLastError();
}

hipError_t launch_gmres_report(SolveState* st, const GmresState* g, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_report, dim3(1), dim3(64), 0, s, st, g);
  return hipGetLastError();
}

int64_t gmres_blocks(int64_t n) {
  const int64_t b = (n + kWavesG - 1) / kWavesG;
  return b < kMaxBlocks ? b : kMaxBlocks;
}

hipError_t launch_transpose64(int64_t n, const double* A, int64_t lda, double* AT, int64_t ld,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_transpose64, dim3(g, g), dim3(256), 0, s, n, A, lda, AT, ld);
  return hipGetLastError();
}

hipError_t launch_gmres_init(GmresState* st, double tol, int32_t m, int32_t max_iter,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, s, st, tol, m, max_iter);
  return hipGetLastError();
}

hipError_t launch_gmres_residual(const GmresArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_residual, dim3((unsigned)gmres_blocks(a.n)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gmres_steps(const GmresArgs& a, int32_t count, hipStream_t s) {
  const dim3 g((unsigned)gmres_blocks(a.n));
  for (int i = 0; i < count; ++i) {
    hipLaunchKernelGGL(k_gm_step1, g, dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_gm_orth<false>, g, dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_gm_orth<true>, g, dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fgmres_residual(const GmresArgs& a, const double* Ax, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_residual, dim3((unsigned)gmres_blocks(a.n)), dim3(kThreads), 0, s, a, Ax);
  return hipGetLastError();
}

hipError_t launch_fgmres_begin(const GmresArgs& a, float* v32, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_begin, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, v32);
  return hipGetLastError();
}

hipError_t launch_fgmres_zstore(const GmresArgs& a, const float* d32, double* zv, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_zstore, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, d32,
                     zv);
  return hipGetLastError();
}

hipError_t launch_fgmres_orth(const GmresArgs& a, const double* Aw, hipStream_t s) {
  const dim3 g((unsigned)gmres_blocks(a.n));
  hipLaunchKernelGGL(k_fg_dots, g, dim3(kThreads), 0, s, a, Aw);
  hipLaunchKernelGGL(k_gm_orth<false>, g, dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_gm_orth<true>, g, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fgmres_report(SolveState* st, const GmresState* g, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_report, dim3(1), dim3(64), 0, s, st, g);
  return hipGetLastError();
}

hipError_t launch_gmres_update(const GmresArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_update, dim3((unsigned)gmres_blocks(a.n)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace nrs
