// Dense LU factorisation with row pivoting and triangular solves (the
// linear-algebra step 3 of Sec. 4), FP32 and FP64.
//
// This file holds the partial-pivoting form (GEPP); static block pivoting
// lives in lu_tiles.hip.  Right-looking blocked algorithm with panel width kNb:
//   panel   : one workgroup factors the n-k x jb panel (pivot search over the
//             whole column);
//   swap    : one wavefront per column applies the panel's row interchanges
//             (lanes hold the jb pivot rows, interchanges with rows below the
//             panel are resolved in registers) and, right of the panel, solves
//             with the unit lower jb x jb block (the U12 row block);
//   update  : A22 -= L21 U12 on the matrix cores (16x16x4 MFMA, FP32 or FP64),
//             128 x 128 output tile per workgroup.
// The composite row permutation is carried along as an extra column so that
// solves can gather the right-hand side in one pass.
#include <algorithm>

#include "nrs_internal.h"

namespace nrs {

namespace {

constexpr int kNb = 64;
constexpr int kPanelThreads = 1024;

template <class T>
__device__ inline T absval(T v) {
  return v < T(0) ? -v : v;
}

template <class T>
__global__ __launch_bounds__(kPanelThreads) void k_getf2(int64_t n, int64_t k, int jb, int scope,
                                                         T* __restrict__ A, int64_t lda,
                                                         int32_t* __restrict__ ipiv,
                                                         int32_t* __restrict__ sing) {
  __shared__ T s_val[kPanelThreads / 64];
  __shared__ int64_t s_idx[kPanelThreads / 64];
  __shared__ int64_t s_piv;
  __shared__ T s_row[kNb];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t kend = k + jb;
  const int64_t rend = scope ? kend : n;
  for (int64_t j = k; j < kend; ++j) {
    T* colj = A + j * lda;
    T best = T(-1);
    int64_t bi = j;
    for (int64_t i = j + tid; i < rend; i += kPanelThreads) {
      const T v = absval(colj[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const T ov = __shfl_xor(best, off);
      const int64_t oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_val[wid] = best;
      s_idx[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      T b = s_val[0];
      int64_t bidx = s_idx[0];
      for (int w = 1; w < kPanelThreads / 64; ++w) {
        if (s_val[w] > b || (s_val[w] == b && s_idx[w] < bidx)) {
          b = s_val[w];
          bidx = s_idx[w];
        }
      }
      s_piv = bidx;
      ipiv[j] = (int32_t)bidx;
    }
    __syncthreads();
    const int64_t p = s_piv;
    if (p != j && tid < jb) {
      T* c = A + (k + tid) * lda;
      const T t = c[j];
      c[j] = c[p];
      c[p] = t;
    }
    __syncthreads();
    const int w = (int)(kend - j);
    if (tid < w) s_row[tid] = A[j + (j + tid) * lda];
    __syncthreads();
    const T piv = s_row[0];
    if (piv == T(0)) {
      if (tid == 0) *sing = 1;
      continue;
    }
    for (int64_t i = j + 1 + tid; i < n; i += kPanelThreads) {
      const T l = colj[i] / piv;
      colj[i] = l;
      for (int c = 1; c < w; ++c) A[i + (j + c) * lda] -= l * s_row[c];
    }
    __syncthreads();
  }
}

// Panel factorisation with partial pivoting spread over G workgroups (a
// cooperative launch, so all of them are resident): workgroup g holds rows
// k + g R .. k + (g+1) R - 1 of the jb-column panel in LDS.  Per column one
// grid-wide barrier: before it, every workgroup publishes its largest
// remaining entry (value, row, and that row's jb entries) and the owner of
// the column's diagonal row publishes that row; after it, every workgroup
// reduces the G candidates to the same pivot (largest magnitude, lowest row
// on ties, as LAPACK), swaps in LDS where it owns one of the two rows, and
// applies the rank-1 update to its rows.  Candidates are double-buffered by
// column parity, so one barrier per column suffices.
constexpr int kCoopThreads = 256;
constexpr int kSlot = 72;          // doubles per candidate: value, row, 64 entries, pad
constexpr int kCoopMaxG = 256;
constexpr int64_t kCoopSpin = 1 << 24;

template <class T>
inline int64_t coop_rows(int64_t m) {
  // all rows in one workgroup when they fit in 120 KiB of LDS (no grid-wide
  // barrier at all), else at least 64 rows and at most kCoopMaxG workgroups
  if (m * kNb * (int64_t)sizeof(T) <= 120 * 1024) return m;
  return std::max<int64_t>(64, (m + kCoopMaxG - 1) / kCoopMaxG);
}

template <class T>
__global__ __launch_bounds__(kCoopThreads) void k_getf2_coop(int64_t n, int64_t k, int jb,
                                                             int64_t R, T* __restrict__ A,
                                                             int64_t lda,
                                                             int32_t* __restrict__ ipiv,
                                                             int32_t* __restrict__ sing,
                                                             double* __restrict__ slots,
                                                             int32_t* __restrict__ bar) {
  extern __shared__ __align__(16) unsigned char coop_lds[];
  T* P = reinterpret_cast<T*>(coop_lds);            // [jb][R] column-major panel rows
  __shared__ T s_prow[kNb];                         // pivot row
  __shared__ T s_top[kNb];                          // the diagonal row before the swap
  __shared__ double s_v[kCoopThreads / 64];
  __shared__ int64_t s_i[kCoopThreads / 64];
  __shared__ int64_t s_p;
  __shared__ int s_w;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int64_t r0 = k + (int64_t)g * R;
  const int nr = (int)std::max<int64_t>(0, std::min<int64_t>(n, r0 + R) - r0);
  for (int c = wid; c < jb; c += kCoopThreads / 64)
    for (int r = lane; r < nr; r += 64) P[c * R + r] = A[(r0 + r) + (k + c) * lda];
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    const int64_t gj = k + j;                       // diagonal row of this column
    double* slot = slots + (size_t)((j & 1) * kCoopMaxG + g) * kSlot;
    double* top = slots + (size_t)(2 * kCoopMaxG + (j & 1)) * kSlot;
    // local candidate: largest |a| over this workgroup's rows >= gj
    double best = -1.0;
    int64_t bi = n;
    for (int r = tid; r < nr; r += kCoopThreads) {
      if (r0 + r < gj) continue;
      const double v = fabs((double)P[j * R + r]);
      if (v > best || (v == best && r0 + r < bi)) {
        best = v;
        bi = r0 + r;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int64_t oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_v[wid] = best;
      s_i[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kCoopThreads / 64; ++w)
        if (s_v[w] > best || (s_v[w] == best && s_i[w] < bi)) {
          best = s_v[w];
          bi = s_i[w];
        }
      slot[0] = best;
      slot[1] = (double)bi;
      s_p = bi;
    }
    __syncthreads();
    if (G == 1) {
      // one workgroup holds every row: the pivot is the local one
      const int64_t p = s_p;
      if (tid < jb) {
        s_prow[tid] = P[tid * R + (p - r0)];
        s_top[tid] = P[tid * R + (gj - r0)];
      }
      if (tid == 0) ipiv[gj] = (int32_t)p;
      __syncthreads();
      if (p != gj && tid < jb) {
        P[tid * R + (p - r0)] = s_top[tid];
        P[tid * R + (gj - r0)] = s_prow[tid];
      }
    } else {
      const int64_t mine = s_p;
      if (tid < jb) {
        slot[2 + tid] = (mine >= r0 && mine < r0 + nr) ? (double)P[tid * R + (mine - r0)] : 0.0;
        if (gj >= r0 && gj < r0 + nr) top[2 + tid] = (double)P[tid * R + (gj - r0)];
      }
      // grid-wide barrier (bounded wait; a timeout raises bit 1 of the
      // singular flag and the launch still completes)
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int32_t target = (j + 1) * G;
        atomicAdd(bar, 1);
        int64_t spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kCoopSpin) {
            atomicOr(sing, 2);
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
      }
      __syncthreads();
      // the pivot: the candidates reduced in the same order by every
      // workgroup; the diagonal row is fetched in the same round
      const double* cand = slots + (size_t)((j & 1) * kCoopMaxG) * kSlot;
      if (tid >= kCoopThreads - 64 && tid - (kCoopThreads - 64) < jb)
        s_top[tid - (kCoopThreads - 64)] = (T)__hip_atomic_load(
            &top[2 + tid - (kCoopThreads - 64)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      best = -1.0;
      bi = n;
      for (int q = tid; q < G; q += kCoopThreads) {
        const double v = __hip_atomic_load(&cand[(size_t)q * kSlot], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        const int64_t i = (int64_t)__hip_atomic_load(&cand[(size_t)q * kSlot + 1],
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v > best || (v == best && i < bi)) {
          best = v;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int64_t oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_v[wid] = best;
        s_i[wid] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        int wbest = 0;
        for (int w = 1; w < kCoopThreads / 64; ++w)
          if (s_v[w] > s_v[wbest] || (s_v[w] == s_v[wbest] && s_i[w] < s_i[wbest])) wbest = w;
        s_p = s_i[wbest];
      }
      __syncthreads();
      const int64_t p = s_p;
      const int pw = (int)((p - k) / R);   // the workgroup whose rows hold row p
      if (tid < jb)
        s_prow[tid] = (T)__hip_atomic_load(&cand[(size_t)pw * kSlot + 2 + tid], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      if (g == 0 && tid == 0) ipiv[gj] = (int32_t)p;
      __syncthreads();
      if (p != gj && tid < jb) {
        if (p >= r0 && p < r0 + nr) P[tid * R + (p - r0)] = s_top[tid];
        if (gj >= r0 && gj < r0 + nr) P[tid * R + (gj - r0)] = s_prow[tid];
      }
    }
    __syncthreads();
    const T piv = s_prow[j];
    if (piv == T(0)) {
      if (g == 0 && tid == 0) atomicOr(sing, 1);
      continue;
    }
    // rank-1 update of this workgroup's rows below the diagonal row: the
    // multipliers first, then (row, column) pairs over all threads
    const int rlo = (int)std::max<int64_t>(0, gj + 1 - r0);
    for (int r = rlo + tid; r < nr; r += kCoopThreads) P[j * R + r] /= piv;
    __syncthreads();
    for (int c = j + 1 + wid; c < jb; c += kCoopThreads / 64) {
      const T u = s_prow[c];
      for (int r = (int)rlo + lane; r < nr; r += 64) P[c * R + r] -= P[j * R + r] * u;
    }
    __syncthreads();
  }
  for (int c = wid; c < jb; c += kCoopThreads / 64)
    for (int r = lane; r < nr; r += 64) A[(r0 + r) + (k + c) * lda] = P[c * R + r];
}

// Columns handled: [0, k) (interchanges only), [k+jb, n) (interchanges and
// the unit-lower solve for U12), and the permutation column (interchanges
// only): one wavefront per column.
template <class T>
__global__ __launch_bounds__(256) void k_laswp_trsm(int64_t n, int64_t k, int jb,
                                                    T* __restrict__ A, int64_t lda,
                                                    const int32_t* __restrict__ ipiv,
                                                    int32_t* __restrict__ perm) {
  __shared__ T sL[kNb * kNb];
  __shared__ int32_t sp[kNb];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x < jb) sp[threadIdx.x] = ipiv[k + threadIdx.x];
  for (int e = threadIdx.x; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    sL[e] = A[(k + r) + (k + c) * lda];
  }
  __syncthreads();
  const int64_t nleft = k, nright = n - k - jb;
  const int64_t cid = blockIdx.x * 4 + w;
  if (cid > nleft + nright) return;
  const bool is_perm = cid == nleft + nright;
  const bool solve = !is_perm && cid >= nleft;
  T* col = nullptr;
  if (!is_perm) col = A + (cid < nleft ? cid : cid + jb) * lda;
  const int64_t kend = k + jb;
  const bool mine = lane < jb;
  T reg = T(0), slot = T(0), outval = T(0);
  int64_t pl = -1;
  bool outside = false, final_w = false;
  if (mine) {
    pl = sp[lane];
    outside = pl >= kend;
    final_w = outside;
    reg = is_perm ? (T)perm[k + lane] : col[k + lane];
    if (outside) slot = is_perm ? (T)perm[pl] : col[pl];
  }
  for (int j = 0; j < jb; ++j) {
    const int64_t p = sp[j];
    if (p < kend) {
      const int pj = (int)(p - k);
      if (pj != j) {
        const T a = __shfl(reg, j);
        const T b = __shfl(reg, pj);
        if (lane == j) reg = b;
        if (lane == pj) reg = a;
      }
    } else {
      const T a = __shfl(reg, j);
      const T b = __shfl(slot, j);
      if (lane == j) {
        reg = b;
        outval = a;
      }
      if (mine && lane > j && pl == p) slot = a;
      if (mine && lane < j && pl == p) final_w = false;
    }
  }
  if (solve) {
    for (int t = 0; t < jb; ++t) {
      const T xt = __shfl(reg, t);
      if (mine && lane > t) reg -= sL[lane + t * jb] * xt;
    }
  }
  if (mine) {
    if (is_perm) {
      perm[k + lane] = (int32_t)reg;
      if (final_w) perm[pl] = (int32_t)outval;
    } else {
      col[k + lane] = reg;
      if (final_w) col[pl] = outval;
    }
  }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
// Output row held in register r of lane l (column is l % 16): the FP32
// instruction gives each lane four consecutive rows, the FP64 one rows
// l/16 + 4r (measured on gfx950).
template <>
struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int kGT = 128;       // output tile edge per workgroup
constexpr int kGK = 64;        // the panel width: every update is rank 64 (K <= kGK)
constexpr int kGES = kGT + 2;  // column stride of the epilogue tile

// LDS of one update tile: the A panel [kGK][kGT] and the B panel [kGT][kGK]
// (k contiguous per column) in 16-byte chunks of E elements, XOR-swizzled so
// that each matrix-core operand read touches every bank once:
//   A: (k, row) at k*kGT + E*((row/E) ^ sa(k)) + row%E,  sa = 8(k%2) (FP64), 4(k%4) (FP32)
//   B: (k, col) at kGK*kGT + col*kGK + E*((k/E) ^ (col%16)) + k%E
// then the output tile [col][row] (stride kGES) for the coalesced epilogue.
template <class T>
struct GemmLds {
  static constexpr int E = 16 / (int)sizeof(T);
  static constexpr int kSize =
      2 * kGK * kGT > kGT * kGES ? 2 * kGK * kGT : kGT * kGES;
  static __device__ inline int sa(int k) { return sizeof(T) == 8 ? 8 * (k & 1) : 4 * (k & 3); }
  static __device__ inline int a_at(int k, int row) {
    return k * kGT + E * ((row / E) ^ sa(k)) + row % E;
  }
  static __device__ inline int b_at(int k, int col) {
    return kGK * kGT + col * kGK + E * ((k / E) ^ (col & 15)) + k % E;
  }
};

// The A and B panels of an interior tile straight into LDS: each wave-wide
// 16-byte global-to-LDS load fills 1 KB (64 lanes x one chunk) in the layout
// of GemmLds; returns once this wave's loads have landed.
template <class T>
__device__ inline void gemm_panels_lds(T* S, const T* __restrict__ Ap, const T* __restrict__ Bp,
                                       int64_t lda, int64_t i0, int64_t j0, int wid, int lane) {
  typedef GemmLds<T> G;
  constexpr int E = G::E;
  constexpr int kPer = 1024 / (int)sizeof(T);   // elements per wave-wide load
  constexpr int kLoads = kGK * kGT / kPer;       // per panel
  for (int q = wid; q < kLoads; q += 4) {
    const int e = q * kPer + lane * E;           // A: (k, slot) of this lane
    const int k = e / kGT, p = (e % kGT) / E;
    const T* g = Ap + (i0 + E * (p ^ G::sa(k))) + (int64_t)k * lda;
    __builtin_amdgcn_global_load_lds(g, S + q * kPer, 16, 0, 0);
  }
  for (int q = wid; q < kLoads; q += 4) {
    const int e = q * kPer + lane * E;           // B: (column, slot) of this lane
    const int col = e / kGK, p = (e % kGK) / E;
    const T* g = Bp + E * (p ^ (col & 15)) + (j0 + col) * lda;
    __builtin_amdgcn_global_load_lds(g, S + kGK * kGT + q * kPer, 16, 0, 0);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// C (m x nc) -= A (m x K) * B (K x nc); all column-major with leading dim lda,
// K <= kGK.  256 threads = 2 x 2 waves, each wave a 64 x 64 sub-tile of 4 x 4
// MFMA blocks.  MFMA 16x16x4 operand layout: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the output row of register r is Mfma<T>::row(l, r), the
// column l%16.  Interior tiles of a full panel (dma != 0: 16-byte aligned
// panels) load both panels with 16-byte global-to-LDS loads; edge tiles load
// element by element with zeros outside.  The products run over k up to K
// rounded up to 32, in increasing k, and C is updated through LDS one column
// per 64 lanes.
template <class T>
__global__ __launch_bounds__(256) void k_gemm_update(int64_t m, int64_t nc, int K,
                                                     const T* __restrict__ Ap,
                                                     const T* __restrict__ Bp,
                                                     T* __restrict__ C, int64_t lda, int dma) {
  typedef GemmLds<T> G;
  constexpr int E = G::E;
  __shared__ __align__(16) T S[G::kSize];
  typedef typename Mfma<T>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = blockIdx.x * (int64_t)kGT, j0 = blockIdx.y * (int64_t)kGT;
  const int wr = (wid >> 1) * 64, wc = (wid & 1) * 64;
  if (dma && K == kGK && i0 + kGT <= m && j0 + kGT <= nc) {
    gemm_panels_lds<T>(S, Ap, Bp, lda, i0, j0, wid, lane);
  } else {
    for (int e = tid; e < kGK * kGT; e += 256) {   // A: rows fastest (coalesced)
      const int row = e % kGT, k = e / kGT;
      const int64_t gi = i0 + row;
      S[G::a_at(k, row)] = (gi < m && k < K) ? Ap[gi + (int64_t)k * lda] : T(0);
    }
    for (int e = tid; e < kGK * kGT; e += 256) {   // B: k fastest (coalesced)
      const int k = e % kGK, col = e / kGK;
      const int64_t gj = j0 + col;
      S[G::b_at(k, col)] = (gj < nc && k < K) ? Bp[k + gj * lda] : T(0);
    }
  }
  __syncthreads();
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = T(0);
  const int kend = ((K + 31) / 32) * 32;
  const int li = lane & 15;
  for (int kk = 0; kk < kend; kk += 4) {
    const int kr = kk + (lane >> 4);
    T av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = S[G::a_at(kr, wr + a * 16 + li)];
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = S[G::b_at(kr, wc + b * 16 + li)];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::run(av[a], bv[b], acc[a][b]);
  }
  __syncthreads();  // every operand read is done: the tile becomes the output
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        S[(wc + b * 16 + li) * kGES + wr + a * 16 + Mfma<T>::row(lane, r)] = acc[a][b][r];
  __syncthreads();
  // C -= tile, 16 of the wave's columns at a time: every load of a batch is
  // issued before its stores (C's columns could alias for the compiler, so a
  // store would otherwise hold back the next column's load)
  constexpr int kBatch = 16;
  for (int c0 = 0; c0 < kGT / 4; c0 += kBatch) {
    T cv[kBatch][kGT / 64];
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
      const int64_t gj = j0 + wid + 4 * (c0 + t);
#pragma unroll
      for (int h = 0; h < kGT / 64; ++h) {
        const int64_t gi = i0 + 64 * h + lane;
        cv[t][h] = (gj < nc && gi < m) ? C[gi + gj * lda] : T(0);
      }
    }
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
      const int col = wid + 4 * (c0 + t);
      const int64_t gj = j0 + col;
#pragma unroll
      for (int h = 0; h < kGT / 64; ++h) {
        const int64_t gi = i0 + 64 * h + lane;
        if (gj < nc && gi < m) C[gi + gj * lda] = cv[t][h] - S[col * kGES + 64 * h + lane];
      }
    }
  }
}

__global__ void k_iota(int32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// x = b[perm] (perm may be NULL: plain copy)
template <class T>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const T* __restrict__ b,
                         T* __restrict__ x, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = perm ? b[perm[i]] : b[i];
}

// Sequential composition of LAPACK-style interchanges into a permutation
// (used only when a caller supplies ipiv without the permutation column).
__global__ void k_ipiv_to_perm(int64_t n, const int32_t* __restrict__ ipiv, int32_t* perm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t j = 0; j < n; ++j) {
    const int32_t p = ipiv[j];
    const int32_t t = perm[j];
    perm[j] = perm[p];
    perm[p] = t;
  }
}

// Multi-workgroup triangular solves (the FP64 form; FP32 uses k_trsv32
// below).  Row block b (64 rows) is owned by one
// workgroup; blocks are handed out by an atomic ticket in dispatch order, so
// a workgroup only ever waits for blocks whose owners are already running.
// It folds in the contribution of each solved block as its flag appears,
// then solves its diagonal block with one wavefront and publishes it.
// sync[0] = ticket, sync[1] = finished count, sync[2 + b] = flag of block b;
// the last workgroup to finish clears them, so the buffer is zero between
// calls (it must be zero before the first).  Waits are bounded: a wait that
// times out sets *err and the kernel still runs to completion.
constexpr int kTb = 64;
constexpr int kTrsvThreads = 256;
constexpr int64_t kSpinLimit = 1 << 22;
// s_waitcnt operand that waits for vmcnt = 0 and leaves expcnt and lgkmcnt at
// their maxima (gfx9 layout: vmcnt in bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8).
constexpr int kWaitVmem = 0x0F70;

// Orders a wavefront's LDS accesses around a hand-over between its lanes.
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ inline T bcast_lane(T v, int lane);
template <>
__device__ inline float bcast_lane<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <>
__device__ inline double bcast_lane<double>(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// LOCALP: the factors come from the tile LU with static block pivoting; the
// interchanges of block row b (lperm, block-local) are applied to the
// partial result b_b - sum_k L_bk y_k before the diagonal solve.
// The diagonal block is read into registers before any wait, and every wait
// consumes all blocks published so far.
// The lower pass takes its right-hand side from rhs (gathered through perm for
// scope 0, read directly for scope 1); the upper pass works in place on x.
// Batched form: the tickets of one launch are numbered step by step (system by
// system inside a step, see TrsvBatch); system s owns flags sys[s].flags.
// ctl[0] = ticket, ctl[1] = finished count of the launch.
template <class T, bool UPPER, bool LOCALP>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv(TrsvBatch<T> bt, int32_t* __restrict__ ctl,
                                                       int32_t* __restrict__ err) {
  __shared__ int s_t, s_jend;
  __shared__ T s_part[kTrsvThreads / 64][kTb];
  __shared__ T s_x[kTb];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_t = atomicAdd(&ctl[0], 1);
  __syncthreads();
  const int32_t tk = s_t;
  int64_t kstep;
  int sidx;
  if (bt.sys == nullptr) {
    kstep = tk;
    sidx = 0;
  } else {
    int lo = 0, hi = bt.nsteps * bt.B;  // pref[lo] <= tk < pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (bt.pref[mid] <= tk) lo = mid; else hi = mid;
    }
    kstep = lo / bt.B;
    sidx = lo % bt.B;
  }
  const TrsvSys<T> sy = bt.sys ? bt.sys[sidx] : bt.one;
  const bool skip = tk >= bt.total || (sy.stop && *sy.stop);
  const int64_t n = sy.n, lda = sy.lda;
  const T* __restrict__ LU = sy.LU;
  T* __restrict__ x = sy.x;
  const T* __restrict__ rhs = sy.rhs;
  const int32_t* __restrict__ lperm = sy.perm;
  int32_t* flags = sy.flags;
  const int64_t nblk = (n + kTb - 1) / kTb;
  const int64_t b = UPPER ? nblk - 1 - kstep : kstep;
  const int64_t r0 = b * kTb;
  const int rows = skip ? 0 : (int)min<int64_t>(kTb, n - r0);
  const int64_t row = r0 + lane;
  if (!skip) {
  // this block row's tile of the last dependency (the one on the critical
  // path), fetched before any wait
  const int64_t jl = UPPER ? b + 1 : b - 1;
  const bool has_jl = UPPER ? (b + 1 < nblk) : (b >= 1);
  T pa[16];
  {
    const int64_t c0 = jl * kTb + w * 16;
    const int cn = has_jl ? (int)max<int64_t>(0, min<int64_t>(16, n - c0)) : 0;
#pragma unroll
    for (int c = 0; c < 16; ++c) pa[c] = (c < cn && row < n) ? LU[row + (c0 + c) * lda] : T(0);
  }
  T dg[kTb];   // diagonal block row of this lane (wave 0)
  if (w == 0) {
#pragma unroll
    for (int c = 0; c < kTb; ++c)
      dg[c] = (c < rows && lane < rows) ? LU[row + (r0 + c) * lda] : T(0);
  }
  T acc = T(0);
  const int64_t jstep = UPPER ? -1 : 1;
  int64_t j = UPPER ? nblk - 1 : 0;
  constexpr int kPoller = 64;   // first lane of wave 1
  while (j != b) {
    if (tid == kPoller) {
      int64_t spins = 0;
      while (ld_relaxed(&flags[j]) == 0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicExch(err, 1);
          break;
        }
        if ((spins & 255) == 0 && ld_relaxed(err)) break;
      }
      int64_t je = j + jstep;
      while (je != b && ld_relaxed(&flags[je]) != 0) je += jstep;
      // the L1 invalidation must be complete before the barrier lets the
      // other waves read the published blocks
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(kWaitVmem);
      s_jend = (int)je;
    }
    __syncthreads();
    const int64_t jend = s_jend;
    __syncthreads();
    for (; j != jend; j += jstep) {
      // wave w covers columns j*64 + w*16 .. +16 of this block row; all 32
      // loads are issued before the first product
      const int64_t c0 = j * kTb + w * 16;
      const int cn = (int)max<int64_t>(0, min<int64_t>(16, n - c0));
      T a[16], xv[16];
      if (j == jl) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          a[c] = pa[c];
          xv[c] = c < cn ? x[c0 + c] : T(0);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const bool ok = c < cn && row < n;
          a[c] = ok ? LU[row + (c0 + c) * lda] : T(0);
          xv[c] = c < cn ? x[c0 + c] : T(0);
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) acc += a[c] * xv[c];
    }
  }
  s_part[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    T v = T(0);
    if (lane < rows) {
      v = UPPER ? x[row] : (LOCALP ? rhs[row] : rhs[lperm[row]]);
      for (int q = 0; q < kTrsvThreads / 64; ++q) v -= s_part[q][lane];
    }
    if (LOCALP && !UPPER) {
      s_x[lane] = v;
      __builtin_amdgcn_wave_barrier();
      if (lane < rows) v = s_x[lperm[row] - r0];
      __builtin_amdgcn_wave_barrier();
    }
    if (!UPPER) {
#pragma unroll
      for (int c = 0; c < kTb; ++c) {
        if (c < rows) {
          const T xc = bcast_lane<T>(v, c);
          if (lane > c) v -= dg[c] * xc;
        }
      }
    } else {
#pragma unroll
      for (int c = kTb - 1; c >= 0; --c) {
        if (c < rows) {
          if (lane == c) v = v / dg[c];
          const T xc = bcast_lane<T>(v, c);
          if (lane < c) v -= dg[c] * xc;
        }
      }
    }
    if (lane < rows) x[row] = v;
  }
  __syncthreads();
  if (tid == 0) st_release(&flags[b], 1);
  }  // !skip
  // the last workgroup of the launch clears every flag and the counters
  if (tid == 0) s_t = atomicAdd(&ctl[1], 1);
  __syncthreads();
  if (s_t == (int)gridDim.x - 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int q = 0; q < bt.B; ++q) {
      const TrsvSys<T> sq = bt.sys ? bt.sys[q] : bt.one;
      const int64_t nb = (sq.n + kTb - 1) / kTb;
      for (int64_t e = tid; e < nb; e += kTrsvThreads) sq.flags[e] = 0;
    }
    __syncthreads();
    if (tid == 0) {
      ctl[0] = 0;
      ctl[1] = 0;
    }
  }
}

// FP32 triangular solves.  Block row b (64 rows) is solved by one workgroup
// as x_b = c_b - M_b x_l, where l is the block solved just before it (b - 1
// for the lower pass, b + 1 for the upper), D_b the diagonal block (unit
// lower for the lower pass, with the block-local interchanges folded into its
// inverse as columns), and
//   M_b = D_b^-1 A_bl          (matrix cores, formed before any wait),
//   c_b = D_b^-1 (r_b - sum_{j other than l} A_bj x_j)   (folded in as the
//         solved blocks appear).
// The step on the critical path is therefore one 64 x 64 product by a single
// wavefront: poll the 64 words of x_l, multiply, publish.  Solved blocks are
// published as tagged 64-bit words (a tag per pass and launch, value bits), so
// a consumer's poll also delivers the data; the last workgroup bumps the
// epoch.  One launch runs both passes: tickets [0, total) are the lower pass,
// [total, 2 total) the upper one, whose workgroups form D^-1 and M while the
// lower pass runs and take their right-hand side from its tagged words.
template <bool LOCALP>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv32(TrsvBatch<float> bt,
                                                         int32_t* __restrict__ ctl,
                                                         int32_t* __restrict__ err) {
  typedef float floatx4 __attribute__((ext_vector_type(4)));
  constexpr int kLd = kTb + 1;
  __shared__ int s_t;
  __shared__ float s_part[kTrsvThreads / 64][kTb];
  __shared__ float s_x[kTb];
  // diagonal block (rows 16-byte aligned for the broadcast reads of the
  // inversion) and D^-1 (odd stride for the column reads that follow)
  __shared__ __align__(16) float s_d[kTb][kTb + 4];
  __shared__ float s_di[kTb][kLd];
  __shared__ float s_l[kTb][kLd];  // A_bl (row-major), then M
  __shared__ float s_w[kTrsvThreads / 64][16];  // per-wave copy of the polled values
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_t = atomicAdd(&ctl[0], 1);
  __syncthreads();
  const int32_t tk0 = s_t;
  const bool UPPER = tk0 >= bt.total;
  const int32_t tk = UPPER ? tk0 - bt.total : tk0;
  int64_t kstep;
  int sidx;
  if (bt.sys == nullptr) {
    kstep = tk;
    sidx = 0;
  } else {
    int lo = 0, hi = bt.nsteps * bt.B;  // pref[lo] <= tk < pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (bt.pref[mid] <= tk) lo = mid; else hi = mid;
    }
    kstep = lo / bt.B;
    sidx = lo % bt.B;
  }
  const TrsvSys<float> sy = bt.sys ? bt.sys[min(sidx, bt.B - 1)] : bt.one;
  const bool skip = tk >= bt.total || (sy.stop && *sy.stop);
  if (!skip) {
    const int64_t n = sy.n, lda = sy.lda;
    const float* __restrict__ LU = sy.LU;
    const uint32_t tagl = 2u * ((uint32_t)*sy.epoch & 0x3fffffffu) + 1u;  // lower pass
    const uint32_t tag = UPPER ? tagl + 1u : tagl;
    const int64_t nblk = (n + kTb - 1) / kTb;
    const int64_t b = UPPER ? nblk - 1 - kstep : kstep;
    const int64_t r0 = b * kTb;
    const int rows = (int)min<int64_t>(kTb, n - r0);
    const int64_t row = r0 + lane;
    const int64_t jl = UPPER ? b + 1 : b - 1;
    const bool has_jl = UPPER ? (b + 1 < nblk) : (b >= 1);
    // the lower pass's right-hand side, fetched before any wait (the upper
    // pass takes its own from the lower pass's words below)
    float rv = 0.f;
    if (!UPPER && w == 0 && lane < rows) rv = LOCALP ? sy.rhs[row] : sy.rhs[sy.perm[row]];
    // A_bl (16 columns per wave) and the identity-padded diagonal block
    {
      const int64_t c0 = jl * kTb + w * 16;
      const int cn = has_jl ? (int)max<int64_t>(0, min<int64_t>(16, n - c0)) : 0;
      float pa[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) pa[c] = (c < cn && row < n) ? LU[row + (c0 + c) * lda] : 0.f;
#pragma unroll
      for (int c = 0; c < 16; ++c) s_l[lane][w * 16 + c] = pa[c];
    }
    for (int e = tid; e < kTb * kTb; e += kTrsvThreads) {
      const int i = e & (kTb - 1), c = e >> 6;
      float v = (i == c) ? 1.f : 0.f;
      if (i < rows && c < rows) v = LU[r0 + i + (r0 + c) * lda];
      s_d[i][c] = v;
    }
    __syncthreads();
    if (w == 0) {
      // the lower pass of the tile LU's factors applies the block row's
      // interchanges first: (D^-1 P)[i][p(c)] = D^-1[i][c]
      const int pc = (LOCALP && !UPPER && lane < rows) ? sy.perm[row] - (int)r0 : lane;
      float xc[kTb];  // column `lane` of D^-1
      if (!UPPER) {
        // unit lower: X[i][c] = [i == c] - sum_{k < i} L[i][k] X[k][c]
#pragma unroll
        for (int i = 0; i < kTb; ++i) {
          float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
          for (int k = 0; k + 3 < i; k += 4) {
            s0 += s_d[i][k] * xc[k];
            s1 += s_d[i][k + 1] * xc[k + 1];
            s2 += s_d[i][k + 2] * xc[k + 2];
            s3 += s_d[i][k + 3] * xc[k + 3];
          }
#pragma unroll
          for (int k = i & ~3; k < i; ++k) s0 += s_d[i][k] * xc[k];
          const float sum = (s0 + s1) + (s2 + s3);
          xc[i] = i < lane ? 0.f : (i == lane ? 1.f : -sum);
        }
      } else {
        // upper: X[i][c] = ([i == c] - sum_{k > i} U[i][k] X[k][c]) / U[i][i]
#pragma unroll
        for (int i = kTb - 1; i >= 0; --i) {
          float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
          for (int k = i + 1; k + 3 < kTb; k += 4) {
            s0 += s_d[i][k] * xc[k];
            s1 += s_d[i][k + 1] * xc[k + 1];
            s2 += s_d[i][k + 2] * xc[k + 2];
            s3 += s_d[i][k + 3] * xc[k + 3];
          }
#pragma unroll
          for (int k = kTb - ((kTb - 1 - i) & 3); k < kTb; ++k) s0 += s_d[i][k] * xc[k];
          const float sum = (s0 + s1) + (s2 + s3);
          xc[i] = i > lane ? 0.f : ((i == lane ? 1.f : 0.f) - sum) / s_d[i][i];
        }
      }
      wave_sync_lds();
      float* dcol = &s_di[0][pc];
#pragma unroll
      for (int i = 0; i < kTb; ++i) dcol[i * kLd] = xc[i];
    }
    __syncthreads();
    // M = D^-1 A_bl: wave w forms rows 16w..16w+15
    if (has_jl) {
      floatx4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < kTb / 4; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const float a = s_di[w * 16 + (lane & 15)][k];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, s_l[k][t * 16 + (lane & 15)], acc[t], 0,
                                                       0, 0);
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_l[w * 16 + 4 * (lane >> 4) + r][t * 16 + (lane & 15)] = acc[t][r];
    }
    // r_b - sum_{j other than l} A_bj x_j: each wavefront polls the 16 tagged
    // words it needs, block by block
    float part = 0.f;
    {
      const int64_t jstep = UPPER ? -1 : 1;
      for (int64_t j = UPPER ? nblk - 1 : 0; j != b && j != jl; j += jstep) {
        const int64_t c0 = j * kTb + w * 16;
        const int cn = (int)max<int64_t>(0, min<int64_t>(16, n - c0));
        float a[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = (c < cn && row < n) ? LU[row + (c0 + c) * lda] : 0.f;
        // lanes 0..15 poll one word each; the values reach the wave through LDS
        uint64_t wd = (uint64_t)tag << 32;
        int64_t spins = 0;
        for (;;) {
          if (lane < cn)
            wd = __hip_atomic_load(&sy.xp[c0 + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (__all((uint32_t)(wd >> 32) == tag)) break;
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicExch(err, 1);
            break;
          }
          if ((spins & 255) == 0 && ld_relaxed(err)) break;
          __builtin_amdgcn_s_sleep(1);
        }
        wave_sync_lds();
        if (lane < 16) s_w[w][lane] = __uint_as_float((uint32_t)wd);
        wave_sync_lds();
#pragma unroll
        for (int c = 0; c < 16; ++c) part += a[c] * s_w[w][c];
      }
    }
    s_part[w][lane] = part;
    __syncthreads();
    if (w == 0) {
      if (UPPER) {  // this block of the lower pass's solution
        uint64_t wd = (uint64_t)tagl << 32;
        int64_t spins = 0;
        for (;;) {
          if (lane < rows)
            wd = __hip_atomic_load(&sy.xp[row], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (__all((uint32_t)(wd >> 32) == tagl)) break;
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicExch(err, 1);
            break;
          }
          if ((spins & 255) == 0 && ld_relaxed(err)) break;
          __builtin_amdgcn_s_sleep(1);
        }
        rv = __uint_as_float((uint32_t)wd);
      }
      float v = 0.f;
      if (lane < rows) {
        v = rv;
#pragma unroll
        for (int q = 0; q < kTrsvThreads / 64; ++q) v -= s_part[q][lane];
      }
      s_x[lane] = v;
      wave_sync_lds();
      // c = D^-1 r (row `lane`)
      float o0 = 0.f, o1 = 0.f, o2 = 0.f, o3 = 0.f;
#pragma unroll
      for (int c = 0; c < kTb; c += 4) {
        o0 += s_di[lane][c] * s_x[c];
        o1 += s_di[lane][c + 1] * s_x[c + 1];
        o2 += s_di[lane][c + 2] * s_x[c + 2];
        o3 += s_di[lane][c + 3] * s_x[c + 3];
      }
      v = (o0 + o1) + (o2 + o3);
      if (has_jl) {
        float mr[kTb];
#pragma unroll
        for (int c = 0; c < kTb; ++c) mr[c] = s_l[lane][c];
        // lane k polls word k of x_l; the values reach every lane through LDS
        const int64_t c0 = jl * kTb;
        const int cn = (int)min<int64_t>(kTb, n - c0);
        uint64_t wd = (uint64_t)tag << 32;
        int64_t spins = 0;
        for (;;) {
          if (lane < cn)
            wd = __hip_atomic_load(&sy.xp[c0 + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (__all((uint32_t)(wd >> 32) == tag)) break;
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicExch(err, 1);
            break;
          }
          if ((spins & 255) == 0 && ld_relaxed(err)) break;
          __builtin_amdgcn_s_sleep(1);
        }
        wave_sync_lds();
        s_x[lane] = __uint_as_float((uint32_t)wd);
        wave_sync_lds();
        float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
#pragma unroll
        for (int c = 0; c < kTb; c += 4) {
          q0 += mr[c] * s_x[c];
          q1 += mr[c + 1] * s_x[c + 1];
          q2 += mr[c + 2] * s_x[c + 2];
          q3 += mr[c + 3] * s_x[c + 3];
        }
        v -= (q0 + q1) + (q2 + q3);
      }
      if (lane < rows) {
        if (UPPER) sy.x[row] = v;  // the lower pass's result lives in its words only
        const uint64_t word = ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v);
        __hip_atomic_store(&sy.xp[row], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }  // !skip
  // the last workgroup of the launch bumps every epoch and clears the counters
  if (tid == 0) s_t = atomicAdd(&ctl[1], 1);
  __syncthreads();
  if (s_t == (int)gridDim.x - 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid == 0) {
      for (int q = 0; q < bt.B; ++q) {
        const TrsvSys<float> sq = bt.sys ? bt.sys[q] : bt.one;
        *sq.epoch = (int32_t)(((uint32_t)*sq.epoch + 1u) & 0x7fffffffu);
      }
      ctl[0] = 0;
      ctl[1] = 0;
    }
  }
}

inline dim3 grid1(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

size_t gepp_scratch_bytes(int64_t n) {
  return (size_t)(2 * kCoopMaxG + 2) * kSlot * sizeof(double) +
         (size_t)((n + kNb - 1) / kNb + 64) * sizeof(int32_t) + 256;
}

namespace {

// Panel of columns k .. k+jb-1 over rows k .. n-1: spread over workgroups
// (cooperative launch) when its rows fit their LDS, else one workgroup.
template <class T>
hipError_t launch_panel(int64_t n, int64_t k, int jb, T* A, int64_t lda, int32_t* ipiv,
                        int32_t* sing, void* scratch, hipStream_t s) {
  int64_t m = n - k;
  int64_t R = coop_rows<T>(m);
  const size_t lds = (size_t)R * kNb * sizeof(T);
  if (scratch && lds <= 128 * 1024) {
    double* slots = static_cast<double*>(scratch);
    int32_t* bar =
        reinterpret_cast<int32_t*>(slots + (size_t)(2 * kCoopMaxG + 2) * kSlot) + k / kNb;
    const unsigned G = (unsigned)((m + R - 1) / R);
    if (G == 1) {  // one workgroup: no co-residency to guarantee
      hipLaunchKernelGGL(k_getf2_coop<T>, dim3(1), dim3(kCoopThreads), (unsigned)lds, s, n, k, jb,
                         R, A, lda, ipiv, sing, slots, bar);
      return hipGetLastError();
    }
    void* args[] = {&n, &k, &jb, &R, &A, &lda, &ipiv, &sing, &slots, &bar};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_getf2_coop<T>), dim3(G),
                                      dim3(kCoopThreads), args, (unsigned)lds, s);
  }
  hipLaunchKernelGGL(k_getf2<T>, dim3(1), dim3(kPanelThreads), 0, s, n, k, jb, 0, A, lda, ipiv,
                     sing);
  return hipGetLastError();
}

}  // namespace

// Blocked LU with partial pivoting over whole columns (GEPP).  scratch: NULL
// or gepp_scratch_bytes(n) bytes (candidate rows and barrier counters of the
// multi-workgroup panel; cleared here).
template <class T>
hipError_t launch_lu_factor(int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* perm,
                            int32_t* sing, hipStream_t s, void* scratch) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, grid1(n, 256), dim3(256), 0, s, perm, n);
  if (scratch) {
    const int64_t words = (int64_t)(gepp_scratch_bytes(n) / sizeof(int32_t));
    hipError_t e = launch_fill_i32(static_cast<int32_t*>(scratch), 0, words - 64, s);
    if (e != hipSuccess) return e;
  }
  for (int64_t k = 0; k < n; k += kNb) {
    const int jb = (int)std::min<int64_t>(kNb, n - k);
    hipError_t e = launch_panel<T>(n, k, jb, A, lda, ipiv, sing, scratch, s);
    if (e != hipSuccess) return e;
    const int64_t ncols = (n - jb) + 1;
    hipLaunchKernelGGL(k_laswp_trsm<T>, dim3((unsigned)((ncols + 3) / 4)), dim3(256), 0, s, n, k,
                       jb, A, lda, ipiv, perm);
    const int64_t rest = n - k - jb;
    if (rest > 0) {
      dim3 g((unsigned)((rest + kGT - 1) / kGT), (unsigned)((rest + kGT - 1) / kGT));
      // global-to-LDS panel loads need 16-byte aligned panels
      const int E = 16 / (int)sizeof(T);
      const int dma = ((uintptr_t)A % 16 == 0 && lda % E == 0 && (k + jb) % E == 0 && k % E == 0);
      hipLaunchKernelGGL(k_gemm_update<T>, g, dim3(256), 0, s, rest, rest, jb,
                         A + (k + jb) + k * lda, A + k + (k + jb) * lda,
                         A + (k + jb) + (k + jb) * lda, lda, dma);
    }
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_trsv_batch(const TrsvBatch<T>& bt, int32_t scope, int32_t* ctl, int32_t* err,
                             hipStream_t s) {
  if (bt.total <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    const dim3 g2(2u * (unsigned)bt.total);  // lower and upper pass in one launch
    if (scope)
      hipLaunchKernelGGL((k_trsv32<true>), g2, dim3(kTrsvThreads), 0, s, bt, ctl, err);
    else
      hipLaunchKernelGGL((k_trsv32<false>), g2, dim3(kTrsvThreads), 0, s, bt, ctl, err);
  } else {
    const dim3 g((unsigned)bt.total);
    if (scope)
      hipLaunchKernelGGL((k_trsv<T, false, true>), g, dim3(kTrsvThreads), 0, s, bt, ctl, err);
    else
      hipLaunchKernelGGL((k_trsv<T, false, false>), g, dim3(kTrsvThreads), 0, s, bt, ctl, err);
    hipLaunchKernelGGL((k_trsv<T, true, false>), g, dim3(kTrsvThreads), 0, s, bt, ctl, err);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_lu_solve(int64_t n, int32_t scope, const T* LU, int64_t lda,
                           const int32_t* perm, const T* b, T* x, int32_t* sync, int32_t* err,
                           const int32_t* stop, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  TrsvBatch<T> bt;
  bt.one.LU = LU;
  bt.one.lda = lda;
  bt.one.n = n;
  bt.one.x = x;
  bt.one.rhs = b;
  bt.one.perm = perm;
  bt.one.flags = sync + 2;
  bt.one.epoch = trsv_epoch(sync, n);
  bt.one.xp = trsv_xp(sync, n);
  bt.one.stop = stop;
  bt.sys = nullptr;
  bt.pref = nullptr;
  bt.B = 1;
  bt.nsteps = (int32_t)((n + kTb - 1) / kTb);
  bt.total = bt.nsteps;
  hipError_t e = launch_trsv_batch<T>(bt, scope, sync, err, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_ipiv_to_perm(int64_t n, const int32_t* ipiv, int32_t* perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ipiv_to_perm, dim3(1), dim3(64), 0, s, n, ipiv, perm);
  return hipGetLastError();
}

template hipError_t launch_lu_factor<float>(int64_t, float*, int64_t, int32_t*, int32_t*,
                                            int32_t*, hipStream_t, void*);
template hipError_t launch_lu_factor<double>(int64_t, double*, int64_t, int32_t*, int32_t*,
                                             int32_t*, hipStream_t, void*);
template hipError_t launch_trsv_batch<float>(const TrsvBatch<float>&, int32_t, int32_t*,
                                             int32_t*, hipStream_t);
template hipError_t launch_trsv_batch<double>(const TrsvBatch<double>&, int32_t, int32_t*,
                                              int32_t*, hipStream_t);
template hipError_t launch_lu_solve<float>(int64_t, int32_t, const float*, int64_t,
                                           const int32_t*, const float*, float*, int32_t*,
                                           int32_t*, const int32_t*, hipStream_t);
template hipError_t launch_lu_solve<double>(int64_t, int32_t, const double*, int64_t,
                                            const int32_t*, const double*, double*, int32_t*,
                                            int32_t*, const int32_t*, hipStream_t);

}  // namespace nrs
