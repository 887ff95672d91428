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

constexpr int kInvThreads = 1024;   // 16 waves: 128 columns x 8 row groups
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
// workgroup, the block held in LDS: row interchanges during the elimination,
// the matching column interchanges of the inverse afterwards in reverse
// order.  The elimination treats the block as row-major; on a column-major
// block it therefore inverts the transpose, whose row-major inverse is the
// column-major inverse of the block.  Orders: off == NULL -> every block
// nb_uniform; else body b's order (skipped if 0).  sing |= 1 on a zero or
// non-finite pivot (the block is then left partly eliminated).
__global__ __launch_bounds__(kInvThreads) void k_block_inverse(int32_t nb_uniform, int64_t stride,
                                                               int64_t N,
                                                               const int32_t* __restrict__ off,
                                                               int32_t nb_lim,
                                                               double* __restrict__ blocks,
                                                               int32_t* __restrict__ sing) {
  extern __shared__ double Ab[];
  __shared__ double colk[kBlockMax];
  __shared__ int32_t piv[kBlockMax];
  __shared__ double s_v[kInvThreads / 64];
  __shared__ int s_i[kInvThreads / 64];
  __shared__ int s_p;
  const int32_t b = blockIdx.x;
  const int nb = off ? body_order(off, b, N, nb_lim, 0) : nb_uniform;
  if (nb <= 0 || nb > kBlockMax) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tx = tid & 127, ty = tid >> 7;
  double* g = blocks + (size_t)b * stride;
  for (int e = tid; e < nb * nb; e += kInvThreads) Ab[e] = g[e];
  __syncthreads();
  bool zero = false;
  for (int k = 0; k < nb; ++k) {
    double best = -1.0;
    int bi = nb;
    if (k + tid < nb) {
      const double v = fabs(Ab[(k + tid) * nb + k]);
      if (v > best) {   // false for NaN: such a row is never chosen
        best = v;
        bi = k + tid;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_v[w] = best;
      s_i[w] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      int q = 0;
      for (int u = 1; u < kInvThreads / 64; ++u)
        if (s_v[u] > s_v[q] || (s_v[u] == s_v[q] && s_i[u] < s_i[q])) q = u;
      const int p = s_i[q] < nb ? s_i[q] : k;
      s_p = p;
      piv[k] = p;
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int c = tid; c < nb; c += kInvThreads) {
        const double t = Ab[k * nb + c];
        Ab[k * nb + c] = Ab[p * nb + c];
        Ab[p * nb + c] = t;
      }
    __syncthreads();
    const double d = Ab[k * nb + k];
    if (d == 0.0 || !isfinite(d)) {
      zero = true;
      continue;
    }
    const double dinv = 1.0 / d;
    for (int i = tid; i < nb; i += kInvThreads) colk[i] = Ab[i * nb + k];
    __syncthreads();
    for (int c = tid; c < nb; c += kInvThreads) Ab[k * nb + c] = c == k ? dinv : Ab[k * nb + c] * dinv;
    __syncthreads();
    // every other row: row_i -= colk[i] * row_k; column k of the inverse
    // takes -colk[i] / d in place
    for (int i = ty; i < nb; i += kInvThreads / 128) {
      if (i == k) continue;
      const double f = colk[i];
      for (int c = tx; c < nb; c += 128)
        Ab[i * nb + c] = c == k ? -f * dinv : fma(-f, Ab[k * nb + c], Ab[i * nb + c]);
    }
    __syncthreads();
  }
  for (int k = nb - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int r = tid; r < nb; r += kInvThreads) {
        const double t = Ab[r * nb + k];
        Ab[r * nb + k] = Ab[r * nb + p];
        Ab[r * nb + p] = t;
      }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += kInvThreads) g[e] = Ab[e];
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
  if (st->halt) return;
  const int k = st->k;
  const int32_t b = blockIdx.x;
  const int nb = body_order(off, b, N, nb_lim, nb_model);
  if (nb == 0) return;
  const int nbp = (nb - 6) / 3;
  const int64_t lo = off[b];
  const int tid = threadIdx.x, tx = tid & 127, ty = tid >> 7;
  for (int r = tid; r < nb; r += kPrecThreads) vb[r] = a.V[block_row(r, nbp, N, lo, b) * kGmresLd + k];
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

}  // namespace

size_t block_inverse_lds(int32_t nb) { return (size_t)nb * nb * sizeof(double); }

int32_t block_order_limit(size_t lds_per_block) {
  // static LDS of the inversion kernel: colk, piv and the reduction slots
  const size_t fixed = kBlockMax * (sizeof(double) + sizeof(int32_t)) +
                       (kInvThreads / 64) * (sizeof(double) + sizeof(int)) + 64;
  if (lds_per_block <= fixed) return 0;
  int32_t nb = (int32_t)std::sqrt((double)(lds_per_block - fixed) / sizeof(double));
  while (nb > 0 && block_inverse_lds(nb) + fixed > lds_per_block) --nb;
  return nb < kBlockMax ? nb : kBlockMax;
}

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
  const int32_t nb_max = off ? nb_lim : nb_uniform;
  hipLaunchKernelGGL(k_block_inverse, dim3((unsigned)count), dim3(kInvThreads),
                     (unsigned)block_inverse_lds(nb_max), s, nb_uniform, stride, N, off, nb_lim,
                     blocks, sing);
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
                             const double* blocks, double* zv, hipStream_t s) {
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

}  // namespace nrs
