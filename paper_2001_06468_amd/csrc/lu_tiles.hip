// Persistent tile LU with static block pivoting (the dense solve of Sec. 4,
// step 3), for one system or a batch of independent systems of different
// sizes in a single launch.
//
// The matrix is cut into 64 x 64 tiles.  Tile (i, j) is finished by exactly
// one task, in "band" m = min(i, j):
//   update : C = A_ij - sum_{k<m} L_ik U_kj   (matrix cores, 16x16x4 MFMA),
//            each rank-64 term folded in as soon as its two tiles are final;
//            in the FP32 forms the two tiles of a term go from memory
//            straight into LDS (global-to-LDS loads), one term ahead;
//   then    i == j : partial pivoting inside the tile (one wavefront, rows in
//                    registers, pivot rows relabelled instead of moved);
//           i <  j : U_mj = L_mm^-1 P_m C   (one lane per column);
//           i >  j : L_im = C U_mm^-1       (one lane per row).
// Tasks are numbered band by band; inside a band of a batch, first the
// diagonal tasks of all systems, then the off-diagonal tasks system by
// system, so that a system's row and column tasks are taken after its
// diagonal task has had the others' time to finish.  That is a topological
// order; each workgroup of the single launch takes its task number from an
// atomic ticket, so a task only waits for tasks whose owners already run.  Every wait is bounded (a timeout raises ctl[2] and the kernel
// still completes), and the last workgroup to finish clears the ticket and
// all completion flags.
//
// Because interchanges stay inside a diagonal tile, L tiles left of the
// diagonal keep the unpermuted row order: block row m satisfies
//   P_m (A_m - sum_{k<m} L_mk U_k) = L_mm U_m   (columns >= m),
// and the forward substitution applies P_m after the block-row update.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "nrs_internal.h"

namespace nrs {

namespace {

constexpr int TB = 64;
constexpr int kLuThreads = 256;
constexpr int kLS = 80;  // LDS row stride of the MFMA staging tiles
constexpr int kCS = 65;  // LDS column stride of the working tile
constexpr int64_t kLuSpin = 1 << 22;
// A single FP32 system of at most kLuSoloTiles tile rows runs one workgroup
// per CU: its launch reserves kLuSoloPad bytes of dynamic LDS (the row tile
// a diagonal task solves itself, 64 x 65 floats), so a workgroup needs more
// than half of the CU's 160 KB.  Its time is the latency
// of the diagonal chain, and a second workgroup on the chain task's CU slows
// the pivot steps; at larger orders the update throughput of two workgroups
// per CU wins (measured, two per CU -> one: n = 3150 1.83 -> 1.73 ms, n = 6300
// 4.10 -> 3.67 ms, n = 8000 5.69 -> 5.65 ms, n = 10,000 8.78 -> 10.0 ms,
// n = 14,244 21.6 -> 25.4 ms).
constexpr unsigned kLuSoloPad = 17 * 1024;
// s_waitcnt operand that waits for vmcnt = 0 and leaves expcnt and lgkmcnt at
// their maxima (gfx9 layout: vmcnt in bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8).
constexpr int kWaitVmem = 0x0F70;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <class T>
struct Mf;
template <>
struct Mf<float> {
  typedef floatx4 acc_t;
  static __device__ inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mf<double> {
  typedef doublex4 acc_t;
  static __device__ inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Bounded wait for a completion flag.  After any timeout (err set) every
// later wait returns at once, so a broken dependency cannot stall the launch.
__device__ inline void wait_flag(const int32_t* f, int32_t* err) {
  int64_t spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > kLuSpin) {
      atomicExch(err, 1);
      break;
    }
    if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
}

template <class T>
__device__ inline T ld_pad(const T* A, int64_t lda, int64_t n, int64_t r, int64_t c) {
  if (r < n && c < n) return A[r + c * lda];
  return r == c ? T(1) : T(0);
}

// 32-bit pivot key: |v| rounded to FP32, its low 6 mantissa bits replaced by
// (63 - lane), so the maximum is unique and ties go to the lowest lane.
template <class T>
__device__ inline uint32_t pivot_key(T v, int lane) {
  const float a = fabsf((float)v);
  return (__float_as_uint(a) & ~63u) | (uint32_t)(63 - lane);
}

// Maximum of a 32-bit value over the 64 lanes of the wave (DPP row
// operations, then the two row broadcasts); the result is uniform.
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, 0x141, 0xF, 0xF, false)); // row_half_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, 0x140, 0xF, 0xF, false)); // row_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, 0x142, 0xA, 0xF, false)); // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, 0x143, 0xC, 0xF, false)); // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

template <class T>
__device__ inline T lane_value(T v, int lane);
template <>
__device__ inline float lane_value<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <>
__device__ inline double lane_value<double>(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders the LDS accesses of a wavefront's lanes around a hand-over between
// lanes (one lane stores what another loads): without it the compiler may
// move a load above a store that, per thread, did not happen.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// LDS of a task.  Cs is the working tile and Ws the staging tile of the
// diagonal factors (L_mm for the column solves and the diagonal panels, U_mm
// for the row solves: never both in one task).  During the update loop they
// are the two stages that hold the operand tiles of consecutive rank-64
// terms (L part first, then U part).  Two separate fields, so that the
// compiler can tell their accesses apart.
// The small fields come first, so that they stay within the 64 KB reach of
// an LDS instruction's immediate offset.
template <class T>
struct Shared {
  T row[TB];
  int32_t perm[TB];
  int32_t pos[TB];
  int32_t task[4];
  uint64_t live[2];  // diagonal tile, per panel parity: bit r set while row r is no pivot
  alignas(16) T Cs[2 * TB * TB];
  alignas(16) T Ws[2 * TB * TB];
};
static_assert(TB * kCS <= 2 * TB * TB && TB * kLS + 4 * 272 <= 2 * TB * TB,
              "working tiles (and the diagonal-block inverses) fit a stage");

template <class T>
__device__ inline T* stage_of(Shared<T>& S, int stage) { return stage ? S.Ws : S.Cs; }

// Dynamic LDS of the one-workgroup-per-CU launches: the row tile that the
// diagonal task of the next band solves itself (64 columns of kCS floats).
extern __shared__ __align__(16) float lu_xtile[];

template <class T>
__device__ inline T pivot_inverse(T piv) {
  return T(1) / piv;
}
template <>
__device__ inline float pivot_inverse<float>(float piv) {
  return __builtin_amdgcn_rcpf(piv);   // hardware reciprocal (1 ulp)
}

// x <- L^-1 x for a unit lower 16 x 16 block whose row k (entries k2 > k)
// starts at L + k * rs, in arithmetic C; the rows are read as 16-byte
// vectors (L and rs keep them 16-byte aligned), all of them independent of
// x, so the loads run ahead of the substitution.
template <class T, class C = T>
__device__ inline void unit_lower_subst16(C (&x)[16], const T* L, int rs) {
  constexpr int VW = 16 / sizeof(T);
  typedef T vq __attribute__((ext_vector_type(VW)));
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    const vq* r = reinterpret_cast<const vq*>(L + k * rs);
    C q[16];
#pragma unroll
    for (int h = (k + 1) / VW; h < 16 / VW; ++h) {
      const vq v = r[h];
#pragma unroll
      for (int e = 0; e < VW; ++e) q[h * VW + e] = (C)v[e];
    }
#pragma unroll
    for (int k2 = k + 1; k2 < 16; ++k2) x[k2] -= q[k2] * x[k];
  }
}

// Partial pivoting inside the diagonal tile held in S.Cs, blocked by panels of
// kPW columns; called by all four waves.  Rows stay at their physical place
// (S.pos[r] = logical index of physical row r once it has been the pivot, TB
// before).  Per panel:
//   wave 0 factors the panel (lane = row, the panel row in registers, DPP
//          wave maximum for the pivot, pivot values by readlane);
//   then each wave takes one column tile right of the panel: the panel's
//          pivot rows are finished there by a unit-lower substitution
//          (U12 = L11^-1 C, one lane per column) and every row that is not
//          yet a pivot gets C -= L21 U12 on the matrix cores (the live-row
//          mask comes from a ballot of wave 0).
// Wave 0 owns the column tile next to the panel, so the next panel's
// factorisation starts as soon as that tile is done; the other waves finish
// the remaining tiles meanwhile (one barrier per panel).  Afterwards the rows
// stay in physical order; the caller stores physical row r at logical row
// S.pos[r].
constexpr int kPW = 16;

template <class T>
__device__ __attribute__((noinline)) void diag_factor(Shared<T>& S, const LuSys<T>& sy, int64_t m,
                                                      int32_t* sing) {
  typedef typename Mf<T>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  bool used = false, zero = false;  // wave 0 only
  int myj = 0;
#pragma unroll
  for (int b = 0; b < TB / kPW; ++b) {
    const int c0 = b * kPW;
    T* Lp = S.Ws + (b & 1) * kPW * kPW;  // [k][k2]: multiplier of pivot k2 at panel column k
    if (w == 0) {
      wave_sync();  // this panel's columns were last written in MFMA layout
      T v[kPW];
#pragma unroll
      for (int k = 0; k < kPW; ++k) v[k] = S.Cs[(c0 + k) * kCS + lane];
      uint32_t key = used ? 0u : pivot_key(v[0], lane) + 1u;
#pragma unroll
      for (int k = 0; k < kPW; ++k) {
        const uint32_t best = wave_max_u32(key);
        const int p = __builtin_amdgcn_readfirstlane(63 - (int)((best - 1u) & 63u));
        const T piv = lane_value<T>(v[k], p);
        if (lane == p) {
          used = true;
          myj = c0 + k;
        }
        // rows already used (and the pivot row) get l = 0 and stay unchanged
        const bool upd = !used && piv != T(0);
        zero = zero || piv == T(0);
        const T l = upd ? v[k] * pivot_inverse<T>(piv) : T(0);
        v[k] = upd ? l : v[k];
        if (k + 1 < kPW) {
          v[k + 1] -= l * lane_value<T>(v[k + 1], p);
          key = used ? 0u : pivot_key(v[k + 1], lane) + 1u;
        }
#pragma unroll
        for (int c = k + 2; c < kPW; ++c) v[c] -= l * lane_value<T>(v[c], p);
        if (lane == 0) S.perm[c0 + k] = p;
      }
#pragma unroll
      for (int k = 0; k < kPW; ++k) S.Cs[(c0 + k) * kCS + lane] = v[k];
      S.pos[lane] = used ? myj : TB;
      const uint64_t um = __ballot(used);
      if (lane == 0) S.live[b & 1] = ~um;
      if (used && myj >= c0) {
        const int kp = myj - c0;
#pragma unroll
        for (int k = 0; k < kPW; ++k) Lp[k * kPW + kp] = k < kp ? v[k] : T(0);
      }
    }
    __syncthreads();
    const int ct = b + 1 + w;  // this wave's column tile
    if (ct < TB / kPW) {
      const int c = ct * kPW + (lane & 15), g = lane >> 4;
      if (lane < kPW) {  // U12 = L11^-1 C on the panel's pivot rows, column c
        int pr[kPW];
#pragma unroll
        for (int k = 0; k < kPW; ++k) pr[k] = c * kCS + S.perm[c0 + k];
        T x[kPW];
#pragma unroll
        for (int k = 0; k < kPW; ++k) x[k] = S.Cs[pr[k]];
        unit_lower_subst16<T>(x, Lp, kPW);
#pragma unroll
        for (int k = 0; k < kPW; ++k) S.Cs[pr[k]] = x[k];
      }
      wave_sync();
      // C -= L21 U12 on rows that are not yet pivots (others: L = 0); every
      // operand is read before the first product
      const uint64_t live = S.live[b & 1];
      acc_t acc[TB / 16];
#pragma unroll
      for (int rt = 0; rt < TB / 16; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[rt][r] = S.Cs[c * kCS + rt * 16 + Mf<T>::row(lane, r)];
      T bu[kPW / 4], av[kPW / 4][TB / 16];
#pragma unroll
      for (int ks = 0; ks < kPW / 4; ++ks) {
        const int kk = c0 + ks * 4 + g;
        bu[ks] = S.Cs[c * kCS + S.perm[kk]];
#pragma unroll
        for (int rt = 0; rt < TB / 16; ++rt) {
          const int row = rt * 16 + (lane & 15);
          const T v = S.Cs[kk * kCS + row];
          av[ks][rt] = (live >> row) & 1 ? -v : T(0);
        }
      }
#pragma unroll
      for (int ks = 0; ks < kPW / 4; ++ks) {
#pragma unroll
        for (int rt = 0; rt < TB / 16; ++rt) acc[rt] = Mf<T>::run(av[ks][rt], bu[ks], acc[rt]);
      }
#pragma unroll
      for (int rt = 0; rt < TB / 16; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) S.Cs[c * kCS + rt * 16 + Mf<T>::row(lane, r)] = acc[rt][r];
    }
  }
  if (w == 0 && zero && lane == 0) atomicExch(sing, 1);
  // permutation of this block row: logical row j <- original row perm[j]
  if (tid < TB) {
    const int64_t r0 = m * TB;
    const int64_t gj = r0 + tid;
    if (gj < sy.n) sy.lperm[gj] = (int32_t)(r0 + S.perm[tid]);
  }
}

// U_mj = L_mm^-1 P_m C, in place in the working tile S.Cs; L_mm (unit lower)
// is staged column-major in S.Ws, the permutation in S.perm.  Called by all
// four waves.  First wave w inverts diagonal block w of L_mm (a substitution
// on the identity in FP64, one lane per column, rounded once) into S.Ws past
// the staged tile, so that multiplying by the inverse is as accurate as the
// substitution it replaces (with the inverse formed in FP32 the refinement
// of a small channel system stopped one sweep early at a 4e-8 force error);
// then
// wave w owns columns 16w..16w+15: per block of 16 rows, X_b = D_b^-1 R_b
// and the update of the rows below, both on the matrix cores, so the
// sequential part of the solve is one 16-step substitution instead of four.
template <class T>
__device__ __attribute__((noinline)) void col_solve(Shared<T>& S) {
  typedef typename Mf<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
  T* col = S.Cs + (w * 16 + li) * kCS;
  T* DI = S.Ws + TB * kLS;  // inverses of the diagonal blocks: block b, (i, k) at b*272 + i*17 + k
  {  // rows to logical order in this wave's columns (all loads before stores)
    T t[TB / 4];
#pragma unroll
    for (int q = 0; q < TB / 4; ++q) t[q] = col[S.perm[g + 4 * q]];
    wave_sync();
#pragma unroll
    for (int q = 0; q < TB / 4; ++q) col[g + 4 * q] = t[q];
  }
  if (lane < 16) {  // wave w: column `lane` of the inverse of diagonal block w (in FP64)
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = k == lane ? 1.0 : 0.0;
    unit_lower_subst16<T, double>(x, S.Ws + w * 16 * kLS + w * 16, kLS);
#pragma unroll
    for (int k = 0; k < 16; ++k) DI[w * 272 + k * 17 + lane] = (T)x[k];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < TB / 16; ++b) {
    const int rb = b * 16;
    wave_sync();
    {  // X_b = D_b^-1 (rows rb.. of the right-hand side) on the matrix cores
      T av[4], bv[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        av[ks] = DI[b * 272 + li * 17 + ks * 4 + g];
        bv[ks] = col[rb + ks * 4 + g];
      }
      acc_t x;
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = T(0);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) x = Mf<T>::run(av[ks], bv[ks], x);
      wave_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) col[rb + Mf<T>::row(lane, r)] = x[r];
    }
    wave_sync();
    // the row blocks below (q < nr), every operand read before the first product
    const int nr = TB / 16 - 1 - b;
    acc_t acc[TB / 16 - 1];
    T av[4][TB / 16 - 1], bv[4];
#pragma unroll
    for (int q = 0; q < TB / 16 - 1; ++q)
      if (q < nr)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][r] = col[(b + 1 + q) * 16 + Mf<T>::row(lane, r)];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k = rb + ks * 4 + g;
      bv[ks] = col[k];
#pragma unroll
      for (int q = 0; q < TB / 16 - 1; ++q)
        if (q < nr) av[ks][q] = -S.Ws[k * kLS + (b + 1 + q) * 16 + li];
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < TB / 16 - 1; ++q)
        if (q < nr) acc[q] = Mf<T>::run(av[ks][q], bv[ks], acc[q]);
#pragma unroll
    for (int q = 0; q < TB / 16 - 1; ++q)
      if (q < nr)
#pragma unroll
        for (int r = 0; r < 4; ++r) col[(b + 1 + q) * 16 + Mf<T>::row(lane, r)] = acc[q][r];
  }
}

// L_im = C U_mm^-1, in place in S.Cs.  With U = D Uh (D its diagonal, Uh unit
// upper), Y = C Uh^-1 and L = Y D^-1.  S.Ws holds Uh row-major, S.row the
// reciprocals of D.  Called by all four waves.  First wave w inverts
// diagonal block w of Uh (one lane per row, in FP64 and rounded once, as in
// col_solve) into S.Ws past the staged tile;
// then wave w owns rows 16w..16w+15: per block of 16 columns, Y_b = R_b
// Uh_b^-1 and the update of the columns to the right on the matrix cores.
template <class T, bool XT = false>
__device__ __attribute__((noinline)) void row_solve(Shared<T>& S) {
  typedef typename Mf<T>::acc_t acc_t;
  // XT: the tile is the hand-over tile in dynamic LDS instead of S.Cs
  T* const Ct = XT ? reinterpret_cast<T*>(lu_xtile) : S.Cs;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
  const int r0 = w * 16;
  T* UI = S.Ws + TB * kLS;  // inverses of Uh's diagonal blocks: block b, (k, j) at b*272 + k*17 + j
  if (lane < 16) {  // wave w: row `lane` of the inverse of diagonal block w (in FP64)
    double y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) y[k] = k == lane ? 1.0 : 0.0;
    unit_lower_subst16<T, double>(y, S.Ws + w * 16 * kLS + w * 16, kLS);
#pragma unroll
    for (int k = 0; k < 16; ++k) UI[w * 272 + lane * 17 + k] = (T)y[k];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < TB / 16; ++b) {
    const int cb = b * 16;
    wave_sync();
    {  // Y_b = (columns cb.. of the right-hand side) Uh_b^-1 on the matrix cores
      T av[4], bv[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        av[ks] = Ct[(cb + ks * 4 + g) * kCS + r0 + li];
        bv[ks] = UI[b * 272 + (ks * 4 + g) * 17 + li];
      }
      acc_t y;
#pragma unroll
      for (int r = 0; r < 4; ++r) y[r] = T(0);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) y = Mf<T>::run(av[ks], bv[ks], y);
      wave_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) Ct[(cb + li) * kCS + r0 + Mf<T>::row(lane, r)] = y[r];
    }
    wave_sync();
    // the column blocks to the right (q < nc), every operand read before the
    // first product
    const int nc = TB / 16 - 1 - b;
    acc_t acc[TB / 16 - 1];
    T av[4], bv[4][TB / 16 - 1];
#pragma unroll
    for (int q = 0; q < TB / 16 - 1; ++q)
      if (q < nc)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[q][r] = Ct[((b + 1 + q) * 16 + li) * kCS + r0 + Mf<T>::row(lane, r)];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k = cb + ks * 4 + g;
      av[ks] = -Ct[k * kCS + r0 + li];
#pragma unroll
      for (int q = 0; q < TB / 16 - 1; ++q)
        if (q < nc) bv[ks][q] = S.Ws[k * kLS + (b + 1 + q) * 16 + li];
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < TB / 16 - 1; ++q)
        if (q < nc) acc[q] = Mf<T>::run(av[ks], bv[ks][q], acc[q]);
#pragma unroll
    for (int q = 0; q < TB / 16 - 1; ++q)
      if (q < nc)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Ct[((b + 1 + q) * 16 + li) * kCS + r0 + Mf<T>::row(lane, r)] = acc[q][r];
  }
  wave_sync();
#pragma unroll
  for (int q = 0; q < TB / 4; ++q) {
    const int c = g + 4 * q;
    T* e = &Ct[c * kCS + r0 + li];
    *e = *e * S.row[c];
  }
}

// LAPACK-style interchange sequence of one diagonal tile (lane 0).
template <class T>
__device__ void diag_ipiv(Shared<T>& S, const LuSys<T>& sy, int64_t m) {
  if (threadIdx.x != 0 || !sy.ipiv) return;
  int pos[TB], at[TB];  // pos[orig] = current position, at[position] = orig row
  for (int r = 0; r < TB; ++r) pos[r] = at[r] = r;
  const int64_t r0 = m * TB;
  for (int j = 0; j < TB; ++j) {
    const int orig = S.perm[j];
    const int q = pos[orig];
    if (r0 + j < sy.n) sy.ipiv[r0 + j] = (int32_t)(r0 + q);
    const int oj = at[j];
    at[j] = orig;
    pos[orig] = j;
    at[q] = oj;
    pos[oj] = q;
  }
}

// Wave 0 of a task: wait until term k of tile (i, j) is published (its L and
// U tiles), then return the end e of the run [k, e) of terms whose tiles are
// all published, the 64 lanes testing 64 terms at a time; the acquire (and
// the completion of its L1 invalidation) orders every later tile load of the
// workgroup after the flags.
template <class T>
__device__ inline int64_t published_run(const LuSys<T>& sy, int64_t i, int64_t j, int64_t k,
                                        int64_t m, int32_t* err, int lane) {
  const int64_t nt = sy.nt;
  if (lane == 0) {
    wait_flag(&sy.done[i * nt + k], err);
    wait_flag(&sy.done[k * nt + j], err);
  }
  int64_t e = k + 1;
  for (;;) {
    const int64_t q = e + lane;
    bool ok = false;
    if (q < m) {
      const int32_t a = __hip_atomic_load(&sy.done[i * nt + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int32_t b = __hip_atomic_load(&sy.done[q * nt + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = a != 0 && b != 0;
    }
    const uint64_t bal = __ballot(ok);
    const int run = bal == ~0ull ? 64 : __builtin_ctzll(~bal);
    e += run;
    if (run < 64) break;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __builtin_amdgcn_s_waitcnt(kWaitVmem);
  return e;
}

// Slot of U(k, c) in the register-staged update loop's U tile (S.Ws): rows of 64, the
// column XOR-swizzled by a rotation of the row index, so that the
// transposing stores (one row per lane) and the matrix-core reads (16
// columns of 4 rows) each touch 64 different banks.
__device__ inline int us_at(int k, int c) { return k * TB + (c ^ (((k & 3) << 4) | (k >> 2))); }

// U(k, j) into the U part of an FP32 update stage Lb, in the layout the
// update loop's issue() gives it (the L part untouched).
__device__ inline void dma_u_part(float* Lb, const float* A, int64_t lda, int64_t n, int64_t k,
                                  int64_t j, int w, int lane) {
  const int pl = lane & 15, sub = lane >> 4;
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const int q = w * 4 + q4, kc = 4 * q + sub;
    const int64_t cg = min(j * TB + kc, n - 1);
    const float* gu = A + (k * TB + 4 * (pl ^ (kc & 15))) + cg * lda;
    __builtin_amdgcn_global_load_lds(gu, Lb + TB * TB + q * 256, 16, 0, 0);
  }
}

// Uh = D^-1 U of the finished diagonal tile of band mb, row-major in S.Ws,
// and the reciprocals of D in S.row, for row_solve.
template <class T>
__device__ inline void stage_uh(Shared<T>& S, const LuSys<T>& sy, int64_t mb) {
  const int tid = threadIdx.x;
  T ua[TB * TB / kLuThreads];
#pragma unroll
  for (int q = 0; q < TB * TB / kLuThreads; ++q) {
    const int e = tid + q * kLuThreads, r = e % TB, c = e / TB;
    ua[q] = ld_pad(sy.A, sy.lda, sy.n, mb * TB + r, mb * TB + c);
  }
  if (tid < TB) S.row[tid] = ld_pad(sy.A, sy.lda, sy.n, mb * TB + tid, mb * TB + tid);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TB * TB / kLuThreads; ++q) {
    const int e = tid + q * kLuThreads, r = e % TB, c = e / TB;
    S.Ws[r * kLS + c] = ua[q] / S.row[r];
  }
  __syncthreads();
  if (tid < TB) S.row[tid] = T(1) / S.row[tid];
}

// One tile task: update, then factor / solve, store, publish.  XO: the
// launch runs one workgroup per CU and may hand row tiles over (LuSys::pre).
template <class T, bool B16, bool XO>
__device__ inline void run_task(Shared<T>& S, const LuSys<T>& sy, int64_t i,
                                                   int64_t j, int64_t m, int32_t* err) {
  typedef typename Mf<T>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // tasks on the diagonal chain issue ahead of other waves on their SIMDs
    const bool chain = i == j || i == j + 1 || j == i + 1;
    if (chain) __builtin_amdgcn_s_setprio(2);
    const int64_t nt = sy.nt, n = sy.n, lda = sy.lda;
    T* A = sy.A;
    const int qi = (w >> 1) * 32, qj = (w & 1) * 32;
    // one-workgroup-per-CU FP32 system: the diagonal task of band m >= 1
    // solves the row tile (m, m - 1) itself and applies its last term from LDS
    const bool xover = XO && std::is_same<T, float>::value && !B16 && sy.pre && i == j && m >= 1;
    const int64_t kmax = xover ? m - 1 : m;  // update terms taken from memory
    // this task's tile of A (only this task ever writes it), loaded up front
    // so that the subtraction after the last update does not wait on memory
    T a_ij[16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = qi + a * 16 + Mf<T>::row(lane, r);
          const int cc = qj + b * 16 + (lane & 15);
          a_ij[(a * 2 + b) * 4 + r] = ld_pad(A, lda, n, i * TB + rr, j * TB + cc);
        }
    // ---- update: acc = sum_{k<m} L_ik U_kj ----
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[a][b][r] = T(0);
    // The rank-64 terms are folded in as their tiles appear: one wait covers
    // every term whose two tiles are already published ([k, kend)), and inside
    // such a run the tiles of term k+1 are loaded while term k runs on the
    // matrix cores.
    if constexpr (std::is_same<T, float>::value) {
      // FP32 A: each term's two operand tiles go from memory straight into
      // LDS (16-byte global-to-LDS loads, no registers), the next term's into
      // the other stage while the current one runs on the matrix cores; one
      // barrier per term.  Term k uses stage (k + m) % 2, so the last term
      // reads stage 1 (Ws) and the working tile (stage 0, Cs) is free once it
      // ends.
      // In both layouts the 16-byte chunks are XOR-swizzled so that each
      // matrix-core operand read touches every LDS bank once.
      //   FP32 operands (A's columns), 64 floats per k or per column:
      //     L part: (k, row) at k*64 + 4*((row/4) ^ 4*(k%4)) + row%4
      //     U part: (k, col) at 4096 + col*64 + 4*((k/4) ^ (col%16)) + k%4
      //     L rows past the order read the padding rows of A's columns (lda
      //     is a multiple of 64) and U columns past the order repeat column
      //     n-1; both only reach entries of the product outside the matrix,
      //     which C below does not take.  k < m <= nt-1, so the term's L
      //     columns and U rows lie inside the matrix.
      //   BF16 operands (the tiles' copies: L_ik as [row][k], U_kj as
      //     [column][k], 64 values per row, zero past the order):
      //     row r, chunk c (8 values) at r*64 + 8*(c ^ ((r/2) % 8)),
      //     U part 4096 values further.
      const int sub = lane >> 4, li = lane & 15;
      const __bf16* sh = reinterpret_cast<const __bf16*>(sy.sh);
      auto issue = [&](int64_t k, int stage) {
        if constexpr (B16) {
          const __bf16* Lt = sh + (i * nt + k) * (TB * TB);
          const __bf16* Ut = sh + (k * nt + j) * (TB * TB);
          __bf16* Lb = reinterpret_cast<__bf16*>(stage_of(S, stage));
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int q = w * 2 + h, r = 8 * q + (lane >> 3);
            const int c = (lane & 7) ^ ((r >> 1) & 7);
            __builtin_amdgcn_global_load_lds(Lt + r * TB + 8 * c, Lb + q * 512, 16, 0, 0);
            __builtin_amdgcn_global_load_lds(Ut + r * TB + 8 * c, Lb + TB * TB + q * 512, 16, 0, 0);
          }
        } else {
          float* Lb = stage_of(S, stage);
          const int p = lane & 15;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            const int q = w * 4 + q4, kc = 4 * q + sub;
            const float* gl = A + (i * TB + 4 * (p ^ (4 * sub))) + (k * TB + kc) * lda;
            __builtin_amdgcn_global_load_lds(gl, Lb + q * 256, 16, 0, 0);
            const int64_t cg = min(j * TB + kc, n - 1);
            const float* gu = A + (k * TB + 4 * (p ^ (kc & 15))) + cg * lda;
            __builtin_amdgcn_global_load_lds(gu, Lb + TB * TB + q * 256, 16, 0, 0);
          }
        }
      };
      // per-lane parts of the operand addresses
      int la0, la1, lb0, lb1;
      if constexpr (B16) {  // rows qi + li, qi + 16 + li (L) and qj + li, qj + 16 + li (U)
        la0 = (qi + li) * TB;
        la1 = (qi + 16 + li) * TB;
        lb0 = TB * TB + (qj + li) * TB;
        lb1 = TB * TB + (qj + 16 + li) * TB;
      } else {  // L rows qi + li, qi + 16 + li at k = kk + sub; U columns qj + li, qj + 16 + li
        la0 = sub * TB + 4 * (((qi + li) >> 2) ^ (4 * sub)) + (li & 3);
        la1 = sub * TB + 4 * (((qi + 16 + li) >> 2) ^ (4 * sub)) + (li & 3);
        lb0 = TB * TB + (qj + li) * TB + sub;
        lb1 = TB * TB + (qj + 16 + li) * TB + sub;
      }
      int64_t kend = 0;
      for (int64_t k = 0; k < kmax; ++k) {
        const int stage = (int)((k + m) & 1);
        if (k >= kend) {
          if (w == 0) {
            const int64_t e = published_run(sy, i, j, k, kmax, err, lane);
            if (lane == 0) S.task[2] = (int32_t)e;
          }
          __syncthreads();
          kend = S.task[2];
          issue(k, stage);
        }
        __builtin_amdgcn_s_waitcnt(kWaitVmem);  // this wave's share of term k has landed
        __syncthreads();  // all shares landed; term k-1's reads of the other stage are done
        if (k + 1 < kend) issue(k + 1, stage ^ 1);
        if constexpr (B16) {
          const __bf16* Sb = reinterpret_cast<const __bf16*>(stage_of(S, stage));
          const int key = (li >> 1) & 7;
#pragma unroll
          for (int kk = 0; kk < TB; kk += 32) {
            const int c = 8 * ((kk / 8 + sub) ^ key);
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(Sb + la0 + c);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(Sb + la1 + c);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(Sb + lb0 + c);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(Sb + lb1 + c);
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
          }
        } else {
          // operands read two matrix-core steps ahead (the scheduling groups
          // keep each step's reads in front of the products two steps back),
          // so the LDS latency overlaps the matrix-core work
          const float* Sb = stage_of(S, stage);
          float a0[TB / 4], a1[TB / 4], b0[TB / 4], b1[TB / 4];
          auto rd = [&](int t) {
            const int ub = 4 * (t ^ li);
            a0[t] = Sb[la0 + 4 * t * TB];
            a1[t] = Sb[la1 + 4 * t * TB];
            b0[t] = Sb[lb0 + ub];
            b1[t] = Sb[lb1 + ub];
          };
          rd(0);
          rd(1);
          __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
          for (int t = 0; t < TB / 4; ++t) {
            if (t + 2 < TB / 4) {
              rd(t + 2);
              __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
            }
            acc[0][0] = Mf<T>::run(a0[t], b0[t], acc[0][0]);
            acc[0][1] = Mf<T>::run(a0[t], b1[t], acc[0][1]);
            acc[1][0] = Mf<T>::run(a1[t], b0[t], acc[1][0]);
            acc[1][1] = Mf<T>::run(a1[t], b1[t], acc[1][1]);
            __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
          }
        }
      }
      if constexpr (XO && !B16) {
        if (xover) {
          // The last term L(m, p) U(p, m), p = m - 1: L(m, p) is solved here
          // from the row task's tile before its solve (handed over long
          // before it is needed), so the solved tile's store, flag and load
          // leave the diagonal chain; U(p, m) comes from its column task.
          const int64_t p = m - 1;
          __syncthreads();  // the last term taken from memory has been read
          if (tid == 0) {
            wait_flag(&sy.preflag[p], err);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(kWaitVmem);
          }
          __syncthreads();
          {
            const float* src = sy.pre + p * (TB * TB);
            for (int c = w; c < TB; c += kLuThreads / TB) lu_xtile[c * kCS + lane] = src[c * TB + lane];
          }
          if (tid == 0) {
            wait_flag(&sy.done[p * nt + p], err);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(kWaitVmem);
          }
          __syncthreads();
          stage_uh<T>(S, sy, p);
          __syncthreads();
          row_solve<T, true>(S);  // lu_xtile <- L(m, p)
          if (tid == 0) {
            wait_flag(&sy.done[p * nt + m], err);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(kWaitVmem);
          }
          __syncthreads();  // also: the solve's reads of S.Ws are done
          dma_u_part(S.Ws, A, lda, n, p, j, w, lane);  // U(p, m) into the U part of stage 1
          __builtin_amdgcn_s_waitcnt(kWaitVmem);
          __syncthreads();
#pragma unroll
          for (int t = 0; t < TB / 4; ++t) {
            const int kk = 4 * t + sub, ub = 4 * (t ^ li);
            const float a0 = lu_xtile[kk * kCS + qi + li], a1 = lu_xtile[kk * kCS + qi + 16 + li];
            const float b0 = S.Ws[lb0 + ub], b1 = S.Ws[lb1 + ub];
            acc[0][0] = Mf<T>::run(a0, b0, acc[0][0]);
            acc[0][1] = Mf<T>::run(a0, b1, acc[0][1]);
            acc[1][0] = Mf<T>::run(a1, b0, acc[1][0]);
            acc[1][1] = Mf<T>::run(a1, b1, acc[1][1]);
          }
        }
      }
    } else {
    // FP64: the tiles pass through registers (loaded one term ahead) into
    // the staging tiles, L in Cs (kLS layout) and U in Ws
    T* Ls = S.Cs;
    T* Us = S.Ws;
    const int r = tid & 63, c0 = tid >> 6;
    T la[16], ua[16];
    int64_t kend = 0;
    for (int64_t k = 0; k < m; ++k) {
      if (k >= kend) {
        if (w == 0) {
          const int64_t e = published_run(sy, i, j, k, m, err, lane);
          if (lane == 0) S.task[2] = (int32_t)e;
        }
        __syncthreads();
        kend = S.task[2];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = c0 + 4 * q;
          la[q] = ld_pad(A, lda, n, i * TB + r, k * TB + c);
          ua[q] = ld_pad(A, lda, n, k * TB + r, j * TB + c);
        }
      }
      __syncthreads();  // the previous term's reads of the staging tiles are done
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = c0 + 4 * q;
        Ls[c * kLS + r] = la[q];
        Us[us_at(r, c)] = ua[q];
      }
      __syncthreads();
      if (k + 1 < kend) {  // next term's tiles, in flight during this one
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = c0 + 4 * q;
          la[q] = ld_pad(A, lda, n, i * TB + r, (k + 1) * TB + c);
          ua[q] = ld_pad(A, lda, n, (k + 1) * TB + r, j * TB + c);
        }
      }
#pragma unroll 4
      for (int kk = 0; kk < TB; kk += 4) {
        const int kr = kk + (lane >> 4), li = lane & 15;
        const T a0 = Ls[kr * kLS + qi + li], a1 = Ls[kr * kLS + qi + 16 + li];
        const T b0 = Us[us_at(kr, qj + li)], b1 = Us[us_at(kr, qj + 16 + li)];
        acc[0][0] = Mf<T>::run(a0, b0, acc[0][0]);
        acc[0][1] = Mf<T>::run(a0, b1, acc[0][1]);
        acc[1][0] = Mf<T>::run(a1, b0, acc[1][0]);
        acc[1][1] = Mf<T>::run(a1, b1, acc[1][1]);
      }
    }
    __syncthreads();  // the last term's reads of the stages are done: Cs is stage 0
    }
    // ---- C = A_ij - acc into the working tile (entries outside the matrix
    // keep the padding of A: the products there are not used) ----
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = qi + a * 16 + Mf<T>::row(lane, r);
          const int cc = qj + b * 16 + (lane & 15);
          const T v = a_ij[(a * 2 + b) * 4 + r];
          S.Cs[cc * kCS + rr] =
              (i * TB + rr < n && j * TB + cc < n) ? v - acc[a][b][r] : v;
        }
    if constexpr (XO && std::is_same<T, float>::value && !B16) {
      if (sy.pre && i == j + 1) {
        // the tile before its solve, for the diagonal task of band i
        __syncthreads();
        float* dst = sy.pre + j * (TB * TB);
        for (int c = w; c < TB; c += kLuThreads / TB) dst[c * TB + lane] = S.Cs[c * kCS + lane];
        __builtin_amdgcn_s_waitcnt(kWaitVmem);  // this wave's stores have landed
        __syncthreads();
        if (tid == 0) __hip_atomic_store(&sy.preflag[j], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (i != j) {
      if (tid == 0) {
        wait_flag(&sy.done[m * nt + m], err);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
      }
    }
    __syncthreads();
    if (i == j) {
      diag_factor<T>(S, sy, m, sy.sing);
    } else if (i < j) {
      // U_mj = L_mm^-1 P_m C; L_mm staged column-major
      {
        T la[TB * TB / kLuThreads];
#pragma unroll
        for (int q = 0; q < TB * TB / kLuThreads; ++q) {
          const int e = tid + q * kLuThreads, r = e % TB, c = e / TB;
          la[q] = ld_pad(A, lda, n, m * TB + r, m * TB + c);
        }
#pragma unroll
        for (int q = 0; q < TB * TB / kLuThreads; ++q) {
          const int e = tid + q * kLuThreads, r = e % TB, c = e / TB;
          S.Ws[c * kLS + r] = la[q];
        }
      }
      if (tid < TB) {
        const int64_t g = m * TB + tid;
        S.perm[tid] = g < n ? (int)(sy.lperm[g] - m * TB) : tid;
      }
      __syncthreads();
      col_solve<T>(S);
    } else {
      // L_im = C U_mm^-1; Uh = D^-1 U staged row-major, 1 / diag in S.row
      stage_uh<T>(S, sy, m);
      __syncthreads();
      row_solve<T>(S);
    }
    __syncthreads();
    {  // store the finished tile, one column per 64 threads (coalesced); the
       // diagonal tile's rows go to their logical places
      const int64_t rr = i * TB + (i == j ? S.pos[lane] : lane);
      if (rr < n) {
        for (int c = w; c < TB; c += kLuThreads / TB) {
          const int64_t cc = j * TB + c;
          if (cc < n) A[rr + cc * lda] = S.Cs[c * kCS + lane];
        }
      }
    }
    if constexpr (B16) {
      // the BF16 copy of an off-diagonal tile for the updates that read it:
      // L tile [row][k] = C(row, k), U tile [column][k] = C(k, column); entries
      // past the order are zero, as ld_pad reads them
      if (i != j) {
        __bf16* dst = reinterpret_cast<__bf16*>(sy.sh) + (i * nt + j) * (TB * TB);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int q = tid + h * kLuThreads, a = q >> 3, b0 = (q & 7) * 8;
          bf16x8 v;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            v[e] = (__bf16)(i > j ? S.Cs[(b0 + e) * kCS + a] : S.Cs[a * kCS + b0 + e]);
          *reinterpret_cast<bf16x8*>(dst + a * TB + b0) = v;
        }
      }
    }
    // Every wave waits until its own stores (tile, BF16 copy, pivot order)
    // are acknowledged before the barrier.  The barrier does not wait for
    // other waves' global stores, and thread 0's release writes back only
    // what has already reached its XCD's L2, so without this wait a consumer
    // on another XCD can, rarely, read part of the tile before it lands.
    __builtin_amdgcn_s_waitcnt(kWaitVmem);
    __syncthreads();
    if (tid == 0) {
      __hip_atomic_store(&sy.done[i * nt + j], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (chain) __builtin_amdgcn_s_setprio(0);
}

// One workgroup per task.  The ticket, not blockIdx, decides the task, so a
// workgroup only waits for tasks taken by workgroups that already run.
// MINB = workgroups per CU the register budget must allow: 1 for a single
// system (the diagonal chain runs alone on its CU), 2 for batches (more
// independent tasks in flight).
template <class T, int MINB, bool B16>
__global__ __launch_bounds__(kLuThreads, MINB) void k_lu_tiles(LuBatch<T> bt, int32_t* ctl) {
  __shared__ Shared<T> S;
  const int tid = threadIdx.x;
  const int32_t B = bt.B;
  int32_t* err = ctl + 2;
  if (tid == 0) S.task[0] = atomicAdd(&ctl[0], 1);
  __syncthreads();
  const int32_t t = S.task[0];
  if (t < bt.total) {
    // (band, part, system) of the ticket: last prefix entry <= t; the
    // off-diagonal part starts at p = 1.  One system: band m starts at
    // m (2 nt - m).
    int m, s, p;
    if (bt.sys == nullptr) {
      const int64_t ntt = bt.one.nt;
      int lo = 0, hi = (int)ntt;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)mid * (2 * ntt - mid) <= t) lo = mid; else hi = mid;
      }
      m = lo;
      s = 0;
      p = (int)(t - (int64_t)lo * (2 * ntt - lo));
    } else {
      int lo = 0, hi = 2 * bt.nbands * B;  // pref[lo] <= t < pref[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bt.pref[mid] <= t) lo = mid; else hi = mid;
      }
      const int half = lo / B;
      m = half >> 1;
      s = lo % B;
      p = t - bt.pref[lo] + (half & 1);
    }
    int64_t i, j;
    if (p == 0) {
      i = j = m;
    } else if (p & 1) {
      i = m;
      j = m + (p + 1) / 2;
    } else {
      i = m + p / 2;
      j = m;
    }
    const LuSys<T> sy = bt.sys ? bt.sys[s] : bt.one;
    run_task<T, B16, MINB == 1>(S, sy, i, j, m, err);
    if (i == j) diag_ipiv<T>(S, sy, m);
  }
  // the last workgroup to finish clears the ticket and every flag
  __syncthreads();
  if (tid == 0) S.task[1] = atomicAdd(&ctl[1], 1);
  __syncthreads();
  if (S.task[1] == (int)gridDim.x - 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int q = 0; q < B; ++q) {
      const LuSys<T> sy = bt.sys ? bt.sys[q] : bt.one;
      const int64_t nf = (int64_t)sy.nt * sy.nt;
      for (int64_t e = tid; e < nf; e += kLuThreads) sy.done[e] = 0;
      if (sy.preflag)
        for (int64_t e = tid; e < sy.nt; e += kLuThreads) sy.preflag[e] = 0;
    }
    __syncthreads();
    if (tid == 0) {
      ctl[0] = 0;
      ctl[1] = 0;
    }
  }
}

}  // namespace

// Ticket prefix over (band, part, system): pref[(2b)*B + s] = ticket of the
// diagonal task of band b of system s, pref[(2b+1)*B + s] = first ticket of
// its 2(nt-b)-2 off-diagonal tasks (empty entries once b >= nt).
void lu_task_prefix(const int32_t* nts, int32_t B, std::vector<int32_t>& pref, int32_t& nbands) {
  nbands = 0;
  for (int s = 0; s < B; ++s) nbands = std::max(nbands, nts[s]);
  pref.assign((size_t)2 * nbands * B + 1, 0);
  int32_t acc = 0;
  for (int b = 0; b < nbands; ++b) {
    for (int s = 0; s < B; ++s) {
      pref[(size_t)(2 * b) * B + s] = acc;
      if (b < nts[s]) acc += 1;
    }
    for (int s = 0; s < B; ++s) {
      pref[(size_t)(2 * b + 1) * B + s] = acc;
      if (b < nts[s]) acc += 2 * (nts[s] - b) - 2;
    }
  }
  pref[(size_t)2 * nbands * B] = acc;
}

template <class T>
hipError_t launch_lu_tiles(const LuBatch<T>& bt, int32_t* ctl, hipStream_t s) {
  if (bt.total <= 0) return hipSuccess;
  const dim3 grid((unsigned)bt.total), block(kLuThreads);
  if (bt.sys) {
    hipLaunchKernelGGL((k_lu_tiles<T, 2, false>), grid, block, 0, s, bt, ctl);
    return hipGetLastError();
  }
  const unsigned pad = (std::is_same<T, float>::value && bt.one.nt <= kLuSoloTiles) ? kLuSoloPad : 0;
  if constexpr (std::is_same<T, float>::value) {
    if (bt.one.sh) {
      hipLaunchKernelGGL((k_lu_tiles<float, 1, true>), grid, block, pad, s, bt, ctl);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_lu_tiles<T, 1, false>), grid, block, pad, s, bt, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t lu_factor_any(int64_t n, int32_t scope, T* A, int64_t lda, int32_t* ipiv,
                         int32_t* perm, int32_t* sing, int32_t* done, int32_t* ctl,
                         hipStream_t s, uint16_t* sh, void* gepp) {
  if (scope == 0) return launch_lu_factor<T>(n, A, lda, ipiv, perm, sing, s, gepp);
  LuBatch<T> bt;
  const int64_t nt = lu_tiles_nt(n);
  bt.one.A = A;
  bt.one.lda = lda;
  bt.one.n = n;
  bt.one.nt = nt;
  bt.one.lperm = perm;
  bt.one.ipiv = ipiv;
  bt.one.done = done;
  bt.one.sing = sing;
  bt.one.sh = std::is_same<T, float>::value ? sh : nullptr;
  if (std::is_same<T, float>::value && sh == nullptr && nt >= 2 && nt <= kLuHandoverTiles) {
    // the row-tile hand-over area after the flags (lu_done_ints)
    bt.one.preflag = done + nt * nt;
    bt.one.pre = reinterpret_cast<T*>(done + (lu_done_flag_ints(n) + 63) / 64 * 64);
  }
  bt.sys = nullptr;
  bt.pref = nullptr;
  bt.B = 1;
  bt.nbands = (int32_t)nt;
  bt.total = (int32_t)(nt * nt);
  return launch_lu_tiles<T>(bt, ctl, s);
}

template hipError_t lu_factor_any<float>(int64_t, int32_t, float*, int64_t, int32_t*, int32_t*,
                                         int32_t*, int32_t*, int32_t*, hipStream_t, uint16_t*,
                                         void*);
template hipError_t lu_factor_any<double>(int64_t, int32_t, double*, int64_t, int32_t*, int32_t*,
                                          int32_t*, int32_t*, int32_t*, hipStream_t, uint16_t*,
                                          void*);
template hipError_t launch_lu_tiles<float>(const LuBatch<float>&, int32_t*, hipStream_t);
template hipError_t launch_lu_tiles<double>(const LuBatch<double>&, int32_t*, hipStream_t);

}  // namespace nrs
