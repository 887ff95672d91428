// Block-diagonal right preconditioner of the flexible GMRES form NRS_GMRES_BLOCK:
// one dense block per free body, covering the body's 3 N_b force unknowns and
// its 6 rigid-body unknowns (the rows of the swimming problem of Sec. 4 that
// belong to the body).  The block is either the exact inverse of that
// diagonal block of the assembled FP64 matrix (lab frame), or the inverse
// predicted by a model learned from the method's own blocks (body frame).
//
// The learned model: every free body of a scene of identical swimmers has,
// in its own frame, a diagonal block that depends only on the phase psi of
// its beat (the travelling-wave argument k s - psi with psi = omega t - phi),
// because the regularized stokeslet, the nearest map within the body's group,
// the patch weights and the rigid-body rows are all unchanged by a rotation
// and translation of the body.  The inverse K(psi) of that block is stored as
// a truncated Fourier series in psi,
//   K(psi) = C_0 + sum_{h=1..H} (C_ch cos h psi + C_sh sin h psi),
// fitted to inverses at S equally spaced phases (S >= 2H + 1, where the
// discrete Fourier sums are the least-squares fit).  In the lab frame the
// block of body b is R_b K(psi_b) R_b^T with R_b the body's rotation acting
// on every point's force vector and on U and Omega.
//
// Block layout: unknown j of a body's block is force component j / N_b of
// the body's point j % N_b for j < 3 N_b, then U_x, U_y, U_z, Omega_x,
// Omega_y, Omega_z.  Blocks are column-major (entry (r, c) at c * nb + r).
#include <cmath>

#include "nrs_internal.h"

namespace nrs {
namespace {

constexpr int kInvThreads = 1024;   // 16 waves
constexpr int kPrecThreads = 1024;

// Order of body b's block, or 0 when the body cannot be preconditioned: its
// points are not a run [off[b], off[b+1]) inside [0, N), the block exceeds
// nb_lim, or it differs from the model's order nb_model (> 0).
__device__ inline int body_order(const int32_t* __restrict__ off, int32_t b, int64_t N,
                                 int32_t nb_lim, int32_t nb_model) {
  const int64_t lo = off[b], hi = off[b + 1];
  if (lo < 0 || hi > N || hi <= lo) return 0;
  const int64_t nb = 3 * (hi - lo) + 6;
  if (nb > nb_lim || (nb_model > 0 && nb != nb_model)) return 0;
  return (int)nb;
}

// Global unknown of row r of body b's block (nbp points from lo).
__device__ inline int64_t block_row(int r, int nbp, int64_t N, int64_t lo, int32_t b) {
  return r < 3 * nbp ? (int64_t)(r / nbp) * N + lo + (r % nbp)
                     : 3 * N + 6 * (int64_t)b + (r - 3 * nbp);
}

// Error bits of the block set-up: 4 = a block above the device limit,
// 8 = a body whose order differs from the model's.
__global__ void k_block_check(int32_t M, int64_t N, const int32_t* __restrict__ off,
                              int32_t nb_lim, int32_t nb_model, int32_t* __restrict__ err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= M) return;
  const int64_t lo = off[b], hi = off[b + 1];
  if (lo < 0 || hi > N || hi <= lo) return;   // reported by the body-run check
  const int64_t nb = 3 * (hi - lo) + 6;
  if (nb > nb_lim) atomicOr(err, 4);
  if (nb_model > 0 && nb != nb_model) atomicOr(err, 8);
}

// psi[b] = omega t - phi of the first wave point of body b (0 if none).
__global__ void k_body_phase(int32_t M, int64_t N, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ part, const double* __restrict__ wave,
                             int32_t P, double t, double* __restrict__ psi) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= M) return;
  const int64_t lo = off[b], hi = off[b + 1];
  double v = 0.0;
  if (lo >= 0 && hi <= N)
    for (int64_t m = lo; m < hi; ++m) {
      const int32_t p = part[m];
      if (p >= 0 && p < P) {
        v = wave[6 * (int64_t)p + 4] * t - wave[6 * (int64_t)p + 5];
        break;
      }
    }
  psi[b] = v;
}

// Diagonal block of each body from the stored FP64 matrix (column-major, lda).
__global__ void k_block_extract(int64_t N, const int32_t* __restrict__ off, int32_t nb_lim,
                                const double* __restrict__ A, int64_t lda, int64_t stride,
                                double* __restrict__ blocks) {
  const int32_t b = blockIdx.y;
  const int nb = body_order(off, b, N, nb_lim, 0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (nb == 0 || e >= nb * nb) return;
  const int c = e / nb, r = e - c * nb;
  const int nbp = (nb - 6) / 3;
  const int64_t lo = off[b];
  blocks[(size_t)b * stride + e] = A[block_row(r, nbp, N, lo, b) + block_row(c, nbp, N, lo, b) * lda];
}

// In-place Gauss-Jordan inversion with partial pivoting of one block per
// workgroup, the block held in registers: lane l owns rows l, l + 64,
// l + 128 and wave w columns w, w + 16, ...  Rows are not interchanged: step
// k takes as pivot the unused row p_k with the largest |a_pk| (lowest index
// on ties), scales it by 1 / a_pk (its column-k entry becoming 1 / a_pk) and
// eliminates column k from every other row (their column-k entries becoming
// -a_ik / a_pk).  The stored array is then the inverse of the row-permuted
// block with its rows in pivot-row order, so entry (i, c) is written to
// (step at which row i was the pivot, pivot row of step c).  The elimination
// treats the block as row-major; on a column-major block it therefore
// inverts the transpose, whose row-major inverse is the column-major inverse
// of the block.  Orders: off == NULL -> every block nb_uniform; else body
// b's order (skipped if 0).  sing |= 1 on a zero or non-finite pivot (the
// output is then not an inverse).
//
// One barrier per step: the wave that owns column k finds the pivot with a
// wave reduction and publishes the column, the pivot row index and value
// (LDS slots double-buffered by step parity); after the barrier every wave
// takes the pivot row's entries of its own columns from the owning lane by
// shuffles and updates its entries.
constexpr int kInvWaves = kInvThreads / 64;                    // 16
constexpr int kInvRowsL = (kBlockMax + 63) / 64;               // rows per lane
constexpr int kInvColsW = (kBlockMax + kInvWaves - 1) / kInvWaves;   // columns per wave

__global__ __launch_bounds__(kInvThreads) void k_block_inverse(int32_t nb_uniform, int64_t stride,
                                                               int64_t N,
                                                               const int32_t* __restrict__ off,
                                                               int32_t nb_lim,
                                                               double* __restrict__ blocks,
                                                               int32_t* __restrict__ sing) {
  __shared__ double colk[2][kBlockMax];
  __shared__ double s_d[2];
  __shared__ int s_p[2];
  __shared__ int32_t step_of[kBlockMax];   // step at which the row was the pivot
  __shared__ int32_t pivot_of[kBlockMax];  // pivot row of each step
  const int32_t b = blockIdx.x;
  const int nb = off ? body_order(off, b, N, nb_lim, 0) : nb_uniform;
  if (nb <= 0 || nb > kBlockMax) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* g = blocks + (size_t)b * stride;
  double reg[kInvRowsL][kInvColsW];
#pragma unroll
  for (int q = 0; q < kInvRowsL; ++q)
#pragma unroll
    for (int j = 0; j < kInvColsW; ++j) {
      const int i = lane + 64 * q, c = w + kInvWaves * j;
      reg[q][j] = (c < nb && i < nb) ? g[(size_t)i * nb + c] : 0.0;
    }
  // columns of this wave below nb (wave-uniform): j < jn
  const int jn = nb > w ? (nb - w + kInvWaves - 1) / kInvWaves : 0;
  uint32_t used = 0;   // bit q: row lane + 64 q was a pivot
  bool zero = false;
  // column slots of rows past nb stay zero (no wave writes them; the first
  // barrier below orders these stores before any read)
  for (int i = nb + tid; i < kBlockMax; i += kInvThreads) colk[0][i] = colk[1][i] = 0.0;
  for (int k = 0; k < nb; ++k) {
    const int buf = k & 1;
    if (w == (k & (kInvWaves - 1))) {
      const int jk = k / kInvWaves;
      double best = -1.0, bd = 0.0;
      int bi = nb;
#pragma unroll
      for (int q = 0; q < kInvRowsL; ++q) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < kInvColsW; ++j)
          if (j == jk) a = reg[q][j];
        const int i = lane + 64 * q;
        if (i < nb) {
          colk[buf][i] = a;
          double v = fabs(a);
          if (!(v >= 0.0)) v = -0.5;   // a NaN ranks below every number
          if (!((used >> q) & 1u) && v > best) {
            best = v;
            bd = a;
            bi = i;
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o);
        const double od = __shfl_xor(bd, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bd = od;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_p[buf] = bi;
        s_d[buf] = bd;
        step_of[bi] = k;
        pivot_of[k] = bi;
      }
    }
    __syncthreads();
    const int p = s_p[buf];
    const double d = s_d[buf];
    double f[kInvRowsL];
#pragma unroll
    for (int q = 0; q < kInvRowsL; ++q) f[q] = colk[buf][lane + 64 * q];
    if (d == 0.0 || !isfinite(d)) zero = true;
    const double dinv = 1.0 / d;
    // the pivot row's entries of this wave's columns, from the lane owning it
    const int lp = p & 63, qp = p >> 6;
    if (lane == lp) used |= 1u << qp;
    double pr[kInvColsW];
#pragma unroll
    for (int j = 0; j < kInvColsW; ++j) {
      double v = reg[0][j];
#pragma unroll
      for (int q = 1; q < kInvRowsL; ++q)
        if (q == qp) v = reg[q][j];
      pr[j] = __shfl(v, lp);
    }
    // one multiply and one FMA per entry: a_ic <- keep_i keep_c a_ic - f_i r_c
    // with r the scaled pivot row (1 / a_pk in column k), f_i = a_ik and
    // keep = 1, except the pivot row (f = -1, keep = 0: it becomes r) and
    // column k (keep = 0: it becomes -a_ik / a_pk).  Rows past nb hold
    // zeros throughout (their column entries are zero); columns past nb are
    // skipped.
    double fe[kInvRowsL], kr[kInvRowsL];
#pragma unroll
    for (int q = 0; q < kInvRowsL; ++q) {
      const bool piv_row = lane + 64 * q == p;
      fe[q] = piv_row ? -1.0 : f[q];
      kr[q] = piv_row ? 0.0 : 1.0;
    }
#pragma unroll
    for (int j = 0; j < kInvColsW; ++j) {
      if (j < jn) {   // wave-uniform
        const int c = w + kInvWaves * j;
        const double kc = c == k ? 0.0 : 1.0;
        const double prj = c == k ? dinv : pr[j] * dinv;
#pragma unroll
        for (int q = 0; q < kInvRowsL; ++q) reg[q][j] = fma(-fe[q], prj, (kr[q] * kc) * reg[q][j]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kInvRowsL; ++q)
#pragma unroll
    for (int j = 0; j < kInvColsW; ++j) {
      const int i = lane + 64 * q, c = w + kInvWaves * j;
      if (c < nb && i < nb) g[(size_t)step_of[i] * nb + pivot_of[c]] = reg[q][j];
    }
  if (zero && tid == 0) atomicOr(sing, 1);
}

// Fourier coefficients of S inverses at phases 2 pi s / S:
// model[0] = (1/S) sum K_s, model[2h-1] = (2/S) sum cos(h psi_s) K_s,
// model[2h] = (2/S) sum sin(h psi_s) K_s.
__global__ void k_block_fit(int32_t S, int32_t nb, int32_t H, const double* __restrict__ inv,
                            double* __restrict__ model) {
  const int64_t nn = (int64_t)nb * nb;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nn) return;
  for (int h = 0; h <= H; ++h) {
    double sc = 0.0, ss = 0.0;
    for (int s = 0; s < S; ++s) {
      const double k = inv[(size_t)s * nn + e];
      const double ang = 2.0 * kPi * (double)(((int64_t)h * s) % S) / (double)S;
      sc = fma(k, cos(ang), sc);
      ss = fma(k, sin(ang), ss);
    }
    if (h == 0) {
      model[e] = sc / S;
    } else {
      model[(size_t)(2 * h - 1) * nn + e] = 2.0 * sc / S;
      model[(size_t)(2 * h) * nn + e] = 2.0 * ss / S;
    }
  }
}

// K(psi_b) of the model for each of `count` blocks: grid (tiles, count).
// off != NULL: the blocks of bodies (skipped unless the body's order is nb).
__global__ void k_block_model(int64_t N, const int32_t* __restrict__ off, int32_t nb_lim, int32_t nb,
                              int32_t H, const double* __restrict__ model,
                              const double* __restrict__ psi, int64_t stride,
                              double* __restrict__ blocks) {
  __shared__ double cs[2 * kBlockHarmonicsMax + 1];
  const int32_t b = blockIdx.y;
  if (off && body_order(off, b, N, nb_lim, nb) == 0) return;
  const double ps = psi[b];
  if ((int)threadIdx.x <= 2 * H) {
    const int h = (threadIdx.x + 1) / 2;
    cs[threadIdx.x] = threadIdx.x == 0 ? 1.0 : ((threadIdx.x & 1) ? cos(h * ps) : sin(h * ps));
  }
  __syncthreads();
  const int64_t nn = (int64_t)nb * nb;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nn) return;
  double k = 0.0;
  for (int j = 0; j <= 2 * H; ++j) k = fma(cs[j], model[(size_t)j * nn + e], k);
  blocks[(size_t)b * stride + e] = k;
}

// First half of z_k = M^-1 v_k: normalise the new basis vector into V[:, k]
// and copy it to Z[:, k] and zv (the identity on rows outside every block).
__global__ void k_prec_begin(GmresArgs a, double* __restrict__ zv) {
  const GmresState* st = a.st;
  if (st->halt) return;
  const int k = st->k;
  const double* __restrict__ vin = st->cur ? a.w1 : a.w0;
  const double s = 1.0 / st->nrm;
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < a.n) {
    const double v = vin[r] * s;
    a.V[r * kGmresLd + k] = v;
    a.Z[r * kGmresLd + k] = v;
    zv[r] = v;
  }
}

// Second half: every body's rows of z_k = K_b v_k (one workgroup per body).
// ROT: K_b is body-frame, applied as R_b K_b R_b^T with R_b from Y.
template <bool ROT>
__global__ __launch_bounds__(kPrecThreads) void k_prec_block(GmresArgs a, int64_t N,
                                                             const int32_t* __restrict__ off,
                                                             int32_t nb_lim, int32_t nb_model,
                                                             const double* __restrict__ Y,
                                                             const double* __restrict__ blocks,
                                                             int64_t stride,
                                                             double* __restrict__ zv) {
  __shared__ double vb[kBlockMax];
  __shared__ double part[kPrecThreads / 128][kBlockMax];
  const GmresState* st = a.st;
  const int32_t b = blockIdx.x;
  // independent loads together: the state words and the body's range
  const int32_t halt = st->halt;
  const int k = st->k;
  const int nb = body_order(off, b, N, nb_lim, nb_model);
  if (halt || nb == 0) return;
  const int nbp = (nb - 6) / 3;
  const int64_t lo = off[b];
  const int tid = threadIdx.x, tx = tid & 127, ty = tid >> 7;
  // v_k from zv, which holds it on every row (written with V[:, k])
  for (int r = tid; r < nb; r += kPrecThreads) vb[r] = zv[block_row(r, nbp, N, lo, b)];
  __syncthreads();
  // B row-major at Y + 12 b + 3: lab = B body, body = B^T lab.  The
  // 3-vectors of the block: point g < nbp at (g, nbp + g, 2 nbp + g), then
  // U and Omega at 3 nbp + 3 (g - nbp) + (0, 1, 2).
  const double* B = ROT ? Y + 12 * (int64_t)b + 3 : nullptr;
  if (ROT) {
    for (int g = tid; g < nbp + 2; g += kPrecThreads) {
      const int i0 = g < nbp ? g : 3 * nbp + 3 * (g - nbp);
      const int st3 = g < nbp ? nbp : 1;
      const double l0 = vb[i0], l1 = vb[i0 + st3], l2 = vb[i0 + 2 * st3];
      for (int j = 0; j < 3; ++j) vb[i0 + j * st3] = B[j] * l0 + B[3 + j] * l1 + B[6 + j] * l2;
    }
    __syncthreads();
  }
  const double* K = blocks + (size_t)b * stride;
  for (int r = tx; r < nb; r += 128) {
    double s = 0.0;
    for (int c = ty; c < nb; c += kPrecThreads / 128) s = fma(K[(size_t)c * nb + r], vb[c], s);
    part[ty][r] = s;
  }
  __syncthreads();
  for (int r = tid; r < nb; r += kPrecThreads) {
    double s = 0.0;
    for (int u = 0; u < kPrecThreads / 128; ++u) s += part[u][r];
    vb[r] = s;
  }
  __syncthreads();
  if (ROT) {
    for (int g = tid; g < nbp + 2; g += kPrecThreads) {
      const int i0 = g < nbp ? g : 3 * nbp + 3 * (g - nbp);
      const int st3 = g < nbp ? nbp : 1;
      const double b0 = vb[i0], b1 = vb[i0 + st3], b2 = vb[i0 + 2 * st3];
      for (int i = 0; i < 3; ++i) vb[i0 + i * st3] = B[3 * i] * b0 + B[3 * i + 1] * b1 + B[3 * i + 2] * b2;
    }
    __syncthreads();
  }
  for (int r = tid; r < nb; r += kPrecThreads) {
    const int64_t gr = block_row(r, nbp, N, lo, b);
    a.Z[gr * kGmresLd + k] = vb[r];
    zv[gr] = vb[r];
  }
}

// ---- one-workgroup flexible GMRES for n <= kGmresSmallN: thread t owns rows
// t, t + 1024, ... (at most kRows) in registers; sums over rows are reduced
// within the workgroup in a fixed order (deterministic). ----
constexpr int kOne = 1024;
// rows per thread: 4 or 8 (n <= 4096, kGmresSmallN), so that small systems
// hold only the registers they use
inline int rows_for(int64_t n) { return n <= 4 * kOne ? 4 : 8; }

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// out[c] = sum over the workgroup of v[c] (c < CNT); every thread calls it.
template <int CNT>
__device__ inline void group_sum(double (&v)[CNT], double* __restrict__ s_part,
                                 double* __restrict__ out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < CNT; ++c) {
    const double t = wsum(v[c]);
    if (lane == 0) s_part[w * CNT + c] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < CNT) {
    double t = 0.0;
    for (int q = 0; q < kOne / 64; ++q) t += s_part[q * CNT + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// Next basis vector v = w / nrm into V[:, col], Z[:, col] and zv.
template <int kRows>
__device__ inline void store_basis(const GmresArgs& a, int col, const double (&wr)[kRows],
                                   double scale, double* __restrict__ zv) {
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const int64_t r = threadIdx.x + (int64_t)j * kOne;
    if (r < a.n) {
      const double v = wr[j] * scale;
      a.V[r * kGmresLd + col] = v;
      a.Z[r * kGmresLd + col] = v;
      zv[r] = v;
    }
  }
}

// r = b - Ax; |r|, |b| (first call); converged, failed, or a new cycle with
// v_0 = r / |r| stored.
template <int kRows>
__global__ __launch_bounds__(kOne) void k_bg_residual(GmresArgs a, const double* __restrict__ Ax,
                                                      int32_t only_if_stopped,
                                                      double* __restrict__ zv) {
  GmresState* st = a.st;
  if (st->done | st->fail) return;
  if (only_if_stopped && !st->stop) return;
  __shared__ double s_part[(kOne / 64) * 2];
  __shared__ double s_r[2];
  __shared__ double s_scale;
  __shared__ int s_new;
  __shared__ double s_bt[2];   // |b| (negative before the first residual), tol
  if (threadIdx.x == 0) {
    s_bt[0] = st->bnorm;
    s_bt[1] = st->tol;
  }
  double rr[kRows];
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const int64_t r = threadIdx.x + (int64_t)j * kOne;
    rr[j] = 0.0;
    if (r < a.n) {
      const double br = a.b[r];
      rr[j] = br - Ax[r];
      acc[0] = fma(rr[j], rr[j], acc[0]);
      acc[1] = fma(br, br, acc[1]);
    }
  }
  group_sum<2>(acc, s_part, s_r);
  if (threadIdx.x == 0) {
    const double beta = sqrt(s_r[0]);
    double bnorm = s_bt[0];
    if (bnorm < 0.0) {
      bnorm = sqrt(s_r[1]);
      st->bnorm = bnorm;
    }
    st->beta = beta;
    int fresh = 0;
    if (!isfinite(beta)) {
      st->fail = 1;
    } else if (beta <= s_bt[1] * bnorm) {
      st->done = 1;
    } else {
      st->nrm = beta;
      st->g[0] = beta;
      st->k = 0;
      st->stop = 0;
      st->cur = 0;
      fresh = 1;
    }
    st->halt = !fresh;   // done or failed, else a new cycle (this kernel runs only when
                         // neither was set before)
    st->skip_true = 1;
    s_new = fresh;
    s_scale = fresh ? 1.0 / beta : 0.0;
  }
  __syncthreads();
  if (s_new) store_basis<kRows>(a, 0, rr, s_scale, zv);
}

// Arnoldi step k on w = A z_k (CGS2): h1 = V^T w, w -= V h1, h2 = V^T w,
// w -= V h2, then the Givens rotations and stop rules; v_{k+1} = w / |w|.
template <int kRows>
__global__ __launch_bounds__(kOne) void k_bg_orth(GmresArgs a, const double* __restrict__ Aw,
                                                  double* __restrict__ zv) {
  GmresState* st = a.st;
  if (st->halt) return;
  const int k = st->k;
  constexpr int kDotW = 4;   // basis columns per pass over the rows (past the cached ones)
  __shared__ double s_part[(kOne / 64) * 8];
  __shared__ double s_h[2][kGmresLd];
  __shared__ double s_n[1];
  __shared__ double s_scale;
  __shared__ int s_next;
  // the Givens state, staged in LDS by one round of parallel loads issued
  // before the passes over the rows (thread 0's rotations then read no
  // global memory)
  __shared__ double s_cs[kGmresLd], s_sn[kGmresLd], s_hk[kGmresLd + 1];
  __shared__ double s_sc[3];   // g[k], tol, |b|
  __shared__ int s_si[3];      // m, iterations, max_iter
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    if (l < k) {
      s_cs[l] = st->cs[l];
      s_sn[l] = st->sn[l];
    }
    if (l == 0) {
      s_sc[0] = st->g[k];
      s_sc[1] = st->tol;
      s_sc[2] = st->bnorm;
      s_si[0] = st->m;
      s_si[1] = st->iters;
      s_si[2] = st->max_iter;
    }
  }
  // w and the first kVC basis columns of every row in one burst of loads,
  // kept in registers for both Gram-Schmidt passes
  constexpr int kVC = kRows == 4 ? 6 : 3;
  double wr[kRows];
  double vc[kRows][kVC];
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const int64_t r = threadIdx.x + (int64_t)j * kOne;
    wr[j] = r < a.n ? Aw[r] : 0.0;
#pragma unroll
    for (int c = 0; c < kVC; ++c) vc[j][c] = (r < a.n && c <= k) ? a.V[r * kGmresLd + c] : 0.0;
  }
  for (int pass = 0; pass < 2; ++pass) {
    double* h = s_h[pass];
    {
      double acc[kVC];
#pragma unroll
      for (int c = 0; c < kVC; ++c) {
        acc[c] = 0.0;
#pragma unroll
        for (int j = 0; j < kRows; ++j) acc[c] = fma(vc[j][c], wr[j], acc[c]);
      }
      group_sum<kVC>(acc, s_part, h);   // zero for columns past k
    }
    for (int i0 = kVC; i0 <= k; i0 += kDotW) {
      double acc[kDotW];
#pragma unroll
      for (int c = 0; c < kDotW; ++c) acc[c] = 0.0;
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const int64_t r = threadIdx.x + (int64_t)j * kOne;
        if (r < a.n) {
          const double* Vr = a.V + r * kGmresLd + i0;
#pragma unroll
          for (int c = 0; c < kDotW; ++c)
            if (i0 + c <= k) acc[c] = fma(Vr[c], wr[j], acc[c]);
        }
      }
      group_sum<kDotW>(acc, s_part, h + i0);
    }
    double hc[kVC];
#pragma unroll
    for (int c = 0; c < kVC; ++c) hc[c] = h[c];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int64_t r = threadIdx.x + (int64_t)j * kOne;
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < kVC; ++c) t = fma(vc[j][c], hc[c], t);
      if (r < a.n) {
        const double* Vr = a.V + r * kGmresLd;
        for (int i = kVC; i <= k; ++i) t = fma(Vr[i], h[i], t);
      }
      wr[j] -= t;
    }
  }
  double nn[1] = {0.0};
#pragma unroll
  for (int j = 0; j < kRows; ++j) nn[0] = fma(wr[j], wr[j], nn[0]);
  group_sum<1>(nn, s_part, s_n);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(s_n[0]);
    double* hk = s_hk;
    for (int i = 0; i <= k; ++i) hk[i] = s_h[0][i] + s_h[1][i];
    hk[k + 1] = nrm;
    for (int i = 0; i < k; ++i) {
      const double t0 = s_cs[i] * hk[i] + s_sn[i] * hk[i + 1];
      hk[i + 1] = -s_sn[i] * hk[i] + s_cs[i] * hk[i + 1];
      hk[i] = t0;
    }
    const double den = hypot(hk[k], hk[k + 1]);
    double c = 1.0, sn = 0.0;
    if (den > 0.0) {
      c = hk[k] / den;
      sn = hk[k + 1] / den;
    }
    hk[k] = den;
    hk[k + 1] = 0.0;
    double* Hk = st->H + (int64_t)k * (kGmresLd + 1);
    for (int i = 0; i <= k + 1; ++i) Hk[i] = hk[i];
    st->cs[k] = c;
    st->sn[k] = sn;
    const double gk1 = -sn * s_sc[0];
    st->g[k + 1] = gk1;
    st->g[k] = c * s_sc[0];
    st->k = k + 1;
    const int iters = s_si[1] + 1;
    st->iters = iters;
    st->nrm = nrm;
    int fail = 0, stop = 0;
    if (!isfinite(nrm) || !isfinite(gk1)) {
      fail = 1;
    } else if (fabs(gk1) <= s_sc[1] * s_sc[2] || nrm == 0.0 || k + 1 >= s_si[0] ||
               iters >= s_si[2]) {
      stop = 1;
    }
    // done is 0 here (the kernel returns at once on a halted state)
    st->fail = fail;
    st->stop = stop;
    st->halt = stop | fail;
    st->skip_true = !stop | fail;
    s_next = !(stop | fail) && nrm > 0.0 && k + 1 < kGmresLd;
    s_scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
  __syncthreads();
  if (s_next) store_basis<kRows>(a, k + 1, wr, s_scale, zv);
}

// End of a stopped cycle: y = R^-1 g (wave 0, back substitution), x += Z y.
__global__ __launch_bounds__(kOne) void k_bg_update(GmresArgs a) {
  GmresState* st = a.st;
  if (!st->stop || st->done || st->fail) return;
  const int k = st->k;
  if (k <= 0) return;
  __shared__ double s_y[kGmresLd];
  __shared__ double s_H[kGmresLd * (kGmresLd + 1)];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int ldh = kGmresLd + 1;
  // the leading k columns of the triangular factor, in LDS (parallel loads)
  for (int e = threadIdx.x; e < k * ldh; e += kOne) s_H[e] = st->H[e];
  if (w == 0) s_y[lane] = lane < k ? st->g[lane] : 0.0;
  __syncthreads();
  if (w == 0) {
    double yi = s_y[lane];
    for (int j = k - 1; j >= 0; --j) {
      const double yj = __shfl(yi, j, 64) / s_H[j * ldh + j];
      if (lane == j) yi = yj;
      if (lane < j) yi -= s_H[j * ldh + lane] * yj;
    }
    s_y[lane] = lane < k ? yi : 0.0;
  }
  __syncthreads();
  for (int64_t r = threadIdx.x; r < a.n; r += kOne) {
    const double* Zr = a.Z + r * kGmresLd;
    double d = 0.0;
    for (int i = 0; i < k; ++i) d = fma(Zr[i], s_y[i], d);
    a.x[r] += d;
  }
}

}  // namespace

hipError_t launch_block_check(int32_t M, int64_t N, const int32_t* off, int32_t nb_lim,
                              int32_t nb_model, int32_t* err, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_check, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, N, off,
                     nb_lim, nb_model, err);
  return hipGetLastError();
}

hipError_t launch_body_phase(int32_t M, int64_t N, const int32_t* off, const int32_t* part,
                             const double* wave, int32_t P, double t, double* psi, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_body_phase, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, N, off,
                     part, wave, P, t, psi);
  return hipGetLastError();
}

hipError_t launch_block_extract(int32_t M, int64_t N, const int32_t* off, int32_t nb_lim,
                                const double* A, int64_t lda, double* blocks, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const dim3 g((unsigned)((nb_lim * nb_lim + 255) / 256), (unsigned)M);
  hipLaunchKernelGGL(k_block_extract, g, dim3(256), 0, s, N, off, nb_lim, A, lda, kBlockStride,
                     blocks);
  return hipGetLastError();
}

hipError_t launch_block_inverse(int32_t count, int32_t nb_uniform, int64_t stride, int64_t N,
                                const int32_t* off, int32_t nb_lim, double* blocks, int32_t* sing,
                                hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_inverse, dim3((unsigned)count), dim3(kInvThreads), 0, s, nb_uniform,
                     stride, N, off, nb_lim, blocks, sing);
  return hipGetLastError();
}

hipError_t launch_block_fit(int32_t S, int32_t nb, int32_t H, const double* inv, double* model,
                            hipStream_t s) {
  const int64_t nn = (int64_t)nb * nb;
  hipLaunchKernelGGL(k_block_fit, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, S, nb, H,
                     inv, model);
  return hipGetLastError();
}

hipError_t launch_block_model(int32_t count, int64_t N, const int32_t* off, int32_t nb_lim,
                              int32_t nb, int32_t H, const double* model, const double* psi,
                              int64_t stride, double* blocks, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 g((unsigned)(((int64_t)nb * nb + 255) / 256), (unsigned)count);
  hipLaunchKernelGGL(k_block_model, g, dim3(256), 0, s, N, off, nb_lim, nb, H, model, psi, stride,
                     blocks);
  return hipGetLastError();
}

hipError_t launch_prec_block(const GmresArgs& a, int32_t M, int64_t N, const int32_t* off,
                             int32_t nb_lim, int32_t nb_model, const double* Y,
                             const double* blocks, double* zv, bool begin, hipStream_t s) {
  if (begin)
    hipLaunchKernelGGL(k_prec_begin, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, zv);
  if (M > 0) {
    if (Y)
      hipLaunchKernelGGL(k_prec_block<true>, dim3((unsigned)M), dim3(kPrecThreads), 0, s, a, N, off,
                         nb_lim, nb_model, Y, blocks, kBlockStride, zv);
    else
      hipLaunchKernelGGL(k_prec_block<false>, dim3((unsigned)M), dim3(kPrecThreads), 0, s, a, N,
                         off, nb_lim, nb_model, Y, blocks, kBlockStride, zv);
  }
  return hipGetLastError();
}

hipError_t launch_bg_residual(const GmresArgs& a, const double* Ax, bool only_if_stopped,
                              double* zv, hipStream_t s) {
  if (a.n > kGmresSmallN) return hipErrorInvalidValue;
  const int32_t f = only_if_stopped;
  switch (rows_for(a.n)) {
    case 4: hipLaunchKernelGGL(k_bg_residual<4>, dim3(1), dim3(kOne), 0, s, a, Ax, f, zv); break;
    default: hipLaunchKernelGGL(k_bg_residual<8>, dim3(1), dim3(kOne), 0, s, a, Ax, f, zv); break;
  }
  return hipGetLastError();
}

hipError_t launch_bg_orth(const GmresArgs& a, const double* Aw, double* zv, hipStream_t s) {
  if (a.n > kGmresSmallN) return hipErrorInvalidValue;
  switch (rows_for(a.n)) {
    case 4: hipLaunchKernelGGL(k_bg_orth<4>, dim3(1), dim3(kOne), 0, s, a, Aw, zv); break;
    default: hipLaunchKernelGGL(k_bg_orth<8>, dim3(1), dim3(kOne), 0, s, a, Aw, zv); break;
  }
  return hipGetLastError();
}

hipError_t launch_bg_update(const GmresArgs& a, hipStream_t s) {
  if (a.n > kGmresSmallN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bg_update, dim3(1), dim3(kOne), 0, s, a);
  return hipGetLastError();
}

}  // namespace nrs
