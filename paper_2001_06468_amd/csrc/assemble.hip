// Fused NEAREST operator assembly (Sec. 3 eqs. 18, 21-23 and the matrix view
// after them), rigid-body blocks of the swimming problem (Sec. 2, Sec. 4),
// right-hand side, and the matrix-free FP64 product used by refinement.
//
// Mapping: one lane per collocation row m, lanes of a wave take consecutive m
// so that every store of A (column-major) is a contiguous 64-element run.  A
// workgroup owns a strip of kTN force points n; the quadrature points of each
// n are contiguous in the nu-sorted layout, so the inner loop walks one
// segment with wave-uniform (scalar) loads and sums the segment in registers:
// the segmented reduction over nu needs no cross-lane traffic and the dense
// 3N x 3Q stokeslet matrix is never formed.
#include "nrs_internal.h"

namespace nrs {

namespace {

// Launch shapes (rows per workgroup, force points per strip); every shape
// computes each entry with the same operations, so the choice (made by the
// autotuner) never changes a result.
constexpr int kShapeBlk[kAsmShapes] = {64, 64, 64, 128, 128, 128, 256, 256, 256};
constexpr int kShapeTN[kAsmShapes] = {4, 8, 16, 4, 8, 16, 4, 8, 16};

// Component j of e_i x r.
__device__ inline double cross_unit(int i, int j, const double r[3]) {
  // (e_i x r)_j = eps_{j i k} r_k
  if (i == j) return 0.0;
  const int k = 3 - i - j;
  // eps_{j i k} = +1 for cyclic (j,i,k)
  const bool cyc = (j == 0 && i == 1) || (j == 1 && i == 2) || (j == 2 && i == 0);
  return cyc ? r[k] : -r[k];
}

// The rigid-body rows and columns of the swimming problem, written by extra
// workgroups of the assembly launch.  Task t < 3N M: row `row` of the
// velocity equations and body s = t / 3N, its six entries in columns
// 3N + 6s .. 3N + 6s + 5 (-1 for U_j on its own component, -(e_i x r_m)_j
// for Omega_i, zero for other bodies).  Task 3N M + t', t' < n M: column
// col = t' / M and body s = t' % M, the six entries of rows 3N + 6s ..
// (force rows W_m delta_jk, moment rows W_m (r_m x e_k)_i for the body's
// points, zero elsewhere and in the rigid-rigid block).  r_m = x_m - x0.
struct RigidArgs {
  int64_t N;
  int32_t M;
  const int32_t* body;
  const double* x;
  const double* Y;
  const double* W;
};

template <class T>
__device__ inline void rigid_task(int64_t t, const RigidArgs& g, T* __restrict__ A, int64_t lda) {
  const int64_t N = g.N, M = g.M, n = 3 * N + 6 * M;
  const int64_t ta = 3 * N * M;
  if (t < ta) {
    const int s = (int)(t / (3 * N));
    const int64_t row = t - (int64_t)s * 3 * N;
    const int j = (int)(row / N);
    const int64_t m = row - j * N;
    const bool own = g.body[m] == s;
    double r[3] = {0.0, 0.0, 0.0};
    if (own) {
      r[0] = g.x[m] - g.Y[12 * s + 0];
      r[1] = g.x[N + m] - g.Y[12 * s + 1];
      r[2] = g.x[2 * N + m] - g.Y[12 * s + 2];
    }
    T* col = A + (3 * N + 6 * (int64_t)s) * lda + row;
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
      if (own) v = c < 3 ? (c == j ? -1.0 : 0.0) : -cross_unit(c - 3, j, r);
      col[c * lda] = (T)v;
    }
    return;
  }
  t -= ta;
  if (t >= n * M) return;
  const int64_t col = t / M;
  const int s = (int)(t - col * M);
  T* out = A + col * lda + 3 * N + 6 * (int64_t)s;
  if (col < 3 * N) {
    const int k = (int)(col / N);
    const int64_t m = col - k * N;
    if (g.body[m] == s) {
      const double r[3] = {g.x[m] - g.Y[12 * s], g.x[N + m] - g.Y[12 * s + 1],
                           g.x[2 * N + m] - g.Y[12 * s + 2]};
      const double wm = g.W[m];
      for (int c = 0; c < 6; ++c)
        // (r x e_k)_i = -(e_k x r)_i
        out[c] = (T)(c < 3 ? (c == k ? wm : 0.0) : -wm * cross_unit(k, c - 3, r));
      return;
    }
  }
  for (int c = 0; c < 6; ++c) out[c] = (T)0.0;
}

// Workgroups past the force-point strips (blockIdx.y >= strips) take the
// rigid-body tasks, kAsmBlock consecutive tasks each.
template <class T, int kAsmBlock, int kTN>
__device__ inline bool rigid_part(const RigidArgs& g, T* __restrict__ A, int64_t lda) {
  const int64_t strips = (g.N + kTN - 1) / kTN;
  if ((int64_t)blockIdx.y < strips) return false;
  const int64_t t = (((int64_t)blockIdx.y - strips) * gridDim.x + blockIdx.x) * kAsmBlock +
                    threadIdx.x;
  if (g.M > 0) rigid_task<T>(t, g, A, lda);
  return true;
}

// FP32 form: coordinates carried as hi + lo floats so that r = x_m - X_q keeps
// FP32 relative accuracy even when |r| << |x|.
template <int kAsmBlock, int kTN>
__global__ __launch_bounds__(kAsmBlock) void k_assemble32(
    int64_t N, const double* __restrict__ x, const int32_t* __restrict__ seg,
    const float4* __restrict__ Xhi, const float4* __restrict__ Xlo, float eps2, float scale,
    float* __restrict__ A, int64_t lda, RigidArgs rg) {
  if (rigid_part<float, kAsmBlock, kTN>(rg, A, lda)) return;
  const int64_t m = blockIdx.x * (int64_t)kAsmBlock + threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.y * kTN;
  const bool live = m < N;
  float xh = 0, yh = 0, zh = 0, xl = 0, yl = 0, zl = 0;
  if (live) {
    const double px = x[m], py = x[N + m], pz = x[2 * N + m];
    xh = (float)px;
    yh = (float)py;
    zh = (float)pz;
    xl = (float)(px - (double)xh);
    yl = (float)(py - (double)yh);
    zl = (float)(pz - (double)zh);
  }
  const int64_t nend = min<int64_t>(N, n0 + kTN);
  for (int64_t n = n0; n < nend; ++n) {
    const int a = seg[n], b = seg[n + 1];
    float a00 = 0, a11 = 0, a22 = 0, a01 = 0, a02 = 0, a12 = 0;
    for (int p = a; p < b; ++p) {
      const float4 h = Xhi[p];
      const float4 l = Xlo[p];
      const float rx = (xh - h.x) + (xl - l.x);
      const float ry = (yh - h.y) + (yl - l.y);
      const float rz = (zh - h.z) + (zl - l.z);
      const float d = rx * rx + ry * ry + rz * rz + eps2;
      const float rho = __builtin_amdgcn_rsqf(d);
      const float t = h.w * (rho * rho * rho);
      const float s = (d + eps2) * t;
      const float tx = t * rx, ty = t * ry, tz = t * rz;
      a00 += s + tx * rx;
      a11 += s + ty * ry;
      a22 += s + tz * rz;
      a01 += tx * ry;
      a02 += tx * rz;
      a12 += ty * rz;
    }
    if (live) {
      float* c0 = A + n * lda;
      float* c1 = A + (N + n) * lda;
      float* c2 = A + (2 * N + n) * lda;
      c0[m] = scale * a00;
      c0[N + m] = scale * a01;
      c0[2 * N + m] = scale * a02;
      c1[m] = scale * a01;
      c1[N + m] = scale * a11;
      c1[2 * N + m] = scale * a12;
      c2[m] = scale * a02;
      c2[N + m] = scale * a12;
      c2[2 * N + m] = scale * a22;
    }
  }
}

template <int kAsmBlock, int kTN>
__global__ __launch_bounds__(kAsmBlock) void k_assemble64(
    int64_t N, const double* __restrict__ x, const int32_t* __restrict__ seg,
    const double4* __restrict__ X64, double eps2, double scale, double* __restrict__ A,
    int64_t lda, RigidArgs rg) {
  if (rigid_part<double, kAsmBlock, kTN>(rg, A, lda)) return;
  const int64_t m = blockIdx.x * (int64_t)kAsmBlock + threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.y * kTN;
  const bool live = m < N;
  double px = 0, py = 0, pz = 0;
  if (live) {
    px = x[m];
    py = x[N + m];
    pz = x[2 * N + m];
  }
  const int64_t nend = min<int64_t>(N, n0 + kTN);
  for (int64_t n = n0; n < nend; ++n) {
    const int a = seg[n], b = seg[n + 1];
    double a00 = 0, a11 = 0, a22 = 0, a01 = 0, a02 = 0, a12 = 0;
    for (int p = a; p < b; ++p) {
      const double4 q = X64[p];
      const double rx = px - q.x, ry = py - q.y, rz = pz - q.z;
      const double d = rx * rx + ry * ry + rz * rz + eps2;
      const double rho = 1.0 / sqrt(d);
      const double t = q.w * (rho * rho * rho);
      const double s = (d + eps2) * t;
      const double tx = t * rx, ty = t * ry, tz = t * rz;
      a00 += s + tx * rx;
      a11 += s + ty * ry;
      a22 += s + tz * rz;
      a01 += tx * ry;
      a02 += tx * rz;
      a12 += ty * rz;
    }
    if (live) {
      double* c0 = A + n * lda;
      double* c1 = A + (N + n) * lda;
      double* c2 = A + (2 * N + n) * lda;
      c0[m] = scale * a00;
      c0[N + m] = scale * a01;
      c0[2 * N + m] = scale * a02;
      c1[m] = scale * a01;
      c1[N + m] = scale * a11;
      c1[2 * N + m] = scale * a12;
      c2[m] = scale * a02;
      c2[N + m] = scale * a12;
      c2[2 * N + m] = scale * a22;
    }
  }
}

// b = [u; f_ext or 0]; with b32 != NULL also its FP32 copy; with st != NULL
// also the body-index check (body[m] in [-1, M), else an argument error).
__global__ void k_rhs(int64_t N, int32_t M, const double* __restrict__ u,
                      const double* __restrict__ ft, double* __restrict__ b,
                      float* __restrict__ b32, const int32_t* __restrict__ body, SolveState* st) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = 3 * N + 6 * (int64_t)M;
  if (st && i < N && (body[i] < -1 || body[i] >= M)) {
    st->nonfinite = 2;
    st->failed = 1;
    st->stop = 1;
  }
  if (i >= n) return;
  const double v = i < 3 * N ? u[i] : (ft ? ft[i - 3 * N] : 0.0);
  b[i] = v;
  if (b32) b32[i] = (float)v;
}

constexpr int kApplyThreads = 256;

// Stage 2 for the 3N velocity rows: sum the chunks in a fixed order (wave w
// takes a contiguous quarter of them with four running sums), scale,
// subtract the rigid-body motion U + Omega x r_m of free-body points.
__device__ inline void apply_velocity_rows(int64_t N, int32_t M, int32_t chunks,
                                           const double* __restrict__ part, double scale,
                                           const double* __restrict__ x,
                                           const int32_t* __restrict__ body,
                                           const double* __restrict__ Y,
                                           const double* __restrict__ v, double* __restrict__ y) {
  __shared__ double red[kApplyThreads / 64][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t row = blockIdx.x * (int64_t)64 + lane;
  const int per = (chunks + kApplyThreads / 64 - 1) / (kApplyThreads / 64);
  const int c0 = w * per, c1 = min(chunks, c0 + per);
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (row < 3 * N) {
    int c = c0;
    for (; c + 3 < c1; c += 4) {
      a0 += part[(int64_t)c * 3 * N + row];
      a1 += part[(int64_t)(c + 1) * 3 * N + row];
      a2 += part[(int64_t)(c + 2) * 3 * N + row];
      a3 += part[(int64_t)(c + 3) * 3 * N + row];
    }
    for (; c < c1; ++c) a0 += part[(int64_t)c * 3 * N + row];
  }
  red[w][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (w != 0 || row >= 3 * N) return;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kApplyThreads / 64; ++q) acc += red[q][lane];
  acc *= scale;
  const int j = (int)(row / N);
  const int64_t m = row - j * N;
  const int b = (body[m] >= 0 && body[m] < M) ? body[m] : -1;
  if (b >= 0) {
    const double r[3] = {x[m] - Y[12 * b], x[N + m] - Y[12 * b + 1], x[2 * N + m] - Y[12 * b + 2]};
    const double* uw = v + 3 * N + 6 * b;
    acc -= uw[j];
    for (int i = 0; i < 3; ++i) acc -= uw[3 + i] * cross_unit(i, j, r);
  }
  y[row] = acc;
}

// Stage 2 for the 6M rigid rows of body s: one workgroup, fixed-order
// reduction of W_m f_m and W_m r_m x f_m.
constexpr int kBodyBlock = 256;
__device__ inline void apply_body_rows(int s, int64_t N, const int32_t* __restrict__ body,
                                       const double* __restrict__ x,
                                       const double* __restrict__ Y,
                                       const double* __restrict__ W,
                                       const double* __restrict__ v, double* __restrict__ y) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t m = threadIdx.x; m < N; m += kBodyBlock) {
    if (body[m] != s) continue;
    const double f[3] = {W[m] * v[m], W[m] * v[N + m], W[m] * v[2 * N + m]};
    const double r[3] = {x[m] - Y[12 * s], x[N + m] - Y[12 * s + 1], x[2 * N + m] - Y[12 * s + 2]};
    acc[0] += f[0];
    acc[1] += f[1];
    acc[2] += f[2];
    acc[3] += r[1] * f[2] - r[2] * f[1];
    acc[4] += r[2] * f[0] - r[0] * f[2];
    acc[5] += r[0] * f[1] - r[1] * f[0];
  }
  __shared__ double red[6][kBodyBlock];
  for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int off = kBodyBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 6) y[3 * N + 6 * s + threadIdx.x] = red[threadIdx.x][0];
}

// Stage 2 of the product in one launch: workgroups [0, rowblocks) take the
// velocity rows, workgroup rowblocks + s the rigid rows of body s.
__global__ __launch_bounds__(kApplyThreads) void k_apply_stage2(
    int64_t N, int32_t M, int32_t chunks, const double* __restrict__ part, double scale,
    const double* __restrict__ x, const int32_t* __restrict__ body,
    const double* __restrict__ Y, const double* __restrict__ W, const double* __restrict__ v,
    double* __restrict__ y, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t rowblocks = (3 * N + 63) / 64;
  if ((int64_t)blockIdx.x >= rowblocks) {
    apply_body_rows((int)(blockIdx.x - rowblocks), N, body, x, Y, W, v, y);
    return;
  }
  apply_velocity_rows(N, M, chunks, part, scale, x, body, Y, v, y);
}

inline dim3 grid1(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

// Grid: x = row blocks of BLK, y = strips of TN force points, then enough
// extra y rows of workgroups for the rigid-body tasks.
template <int BLK, int TN>
dim3 asm_grid(const nrs_problem& pb) {
  const int64_t N = pb.N, M = pb.M, n = 3 * N + 6 * M;
  const int64_t gx = (N + BLK - 1) / BLK, strips = (N + TN - 1) / TN;
  const int64_t tasks = 3 * N * M + n * M;
  const int64_t extra = (tasks + gx * BLK - 1) / (gx * BLK);
  return dim3((unsigned)gx, (unsigned)(strips + extra));
}
inline RigidArgs rigid_args(const nrs_problem& pb, const Sorted& srt) {
  return RigidArgs{pb.N, pb.M, pb.body, pb.x, pb.Y, srt.W};
}
template <int BLK, int TN>
void asm32(const nrs_problem& pb, const Sorted& srt, float* A, int64_t lda, float scale,
           hipStream_t s) {
  const dim3 g = asm_grid<BLK, TN>(pb);
  hipLaunchKernelGGL((k_assemble32<BLK, TN>), g, dim3(BLK), 0, s, pb.N, pb.x,
                     srt.seg, srt.X32hi, srt.X32lo, (float)(pb.eps * pb.eps), scale, A, lda,
                     rigid_args(pb, srt));
}
template <int BLK, int TN>
void asm64(const nrs_problem& pb, const Sorted& srt, double* A, int64_t lda, double scale,
           hipStream_t s) {
  const dim3 g = asm_grid<BLK, TN>(pb);
  hipLaunchKernelGGL((k_assemble64<BLK, TN>), g, dim3(BLK), 0, s, pb.N, pb.x,
                     srt.seg, srt.X64, pb.eps * pb.eps, scale, A, lda, rigid_args(pb, srt));
}

template <class T>
void asm_dispatch(int shape, const nrs_problem& pb, const Sorted& srt, T* A, int64_t lda, T scale,
                  hipStream_t s);
#define NRS_ASM_CASES(F)                                                                        \
  switch (shape) {                                                                             \
    case 0: F<64, 4>(pb, srt, A, lda, scale, s); break;                                        \
    case 1: F<64, 8>(pb, srt, A, lda, scale, s); break;                                        \
    case 2: F<64, 16>(pb, srt, A, lda, scale, s); break;                                       \
    case 3: F<128, 4>(pb, srt, A, lda, scale, s); break;                                       \
    case 5: F<128, 16>(pb, srt, A, lda, scale, s); break;                                      \
    case 6: F<256, 4>(pb, srt, A, lda, scale, s); break;                                       \
    case 7: F<256, 8>(pb, srt, A, lda, scale, s); break;                                       \
    case 8: F<256, 16>(pb, srt, A, lda, scale, s); break;                                      \
    default: F<128, 8>(pb, srt, A, lda, scale, s); break;                                      \
  }
template <>
void asm_dispatch<float>(int shape, const nrs_problem& pb, const Sorted& srt, float* A,
                         int64_t lda, float scale, hipStream_t s) {
  NRS_ASM_CASES(asm32)
}
template <>
void asm_dispatch<double>(int shape, const nrs_problem& pb, const Sorted& srt, double* A,
                          int64_t lda, double scale, hipStream_t s) {
  NRS_ASM_CASES(asm64)
}
#undef NRS_ASM_CASES

}  // namespace

void asm_shape_dims(int32_t shape, int32_t* blk, int32_t* tn) {
  if (shape < 0 || shape >= kAsmShapes) shape = kAsmDefaultShape;
  *blk = kShapeBlk[shape];
  *tn = kShapeTN[shape];
}

template <class T>
hipError_t launch_assemble(const nrs_problem& pb, const Sorted& srt, T* A, int64_t lda,
                           hipStream_t s, int32_t shape) {
  const int64_t N = pb.N;
  const int64_t n = 3 * N + 6 * (int64_t)pb.M;
  const T scale = (T)(1.0 / (8.0 * kPi * pb.mu));
  // one launch: the fused operator and, in extra workgroups, the rigid-body
  // rows and columns
  if (N > 0) asm_dispatch<T>(shape, pb, srt, A, lda, scale, s);
  (void)n;
  return hipGetLastError();
}
template hipError_t launch_assemble<float>(const nrs_problem&, const Sorted&, float*, int64_t,
                                           hipStream_t, int32_t);
template hipError_t launch_assemble<double>(const nrs_problem&, const Sorted&, double*, int64_t,
                                            hipStream_t, int32_t);

hipError_t launch_rhs(int64_t N, int32_t M, const double* u, const double* ftext, double* b,
                      hipStream_t s, float* b32, const int32_t* body, SolveState* st) {
  const int64_t n = 3 * N + 6 * (int64_t)M;
  hipLaunchKernelGGL(k_rhs, grid1(std::max(n, st ? N : 0), 256), dim3(256), 0, s, N, M, u, ftext,
                     b, b32, body, st);
  return hipGetLastError();
}

// Matrix-free FP64 product: the velocity rows are the flow of the force
// densities v at the force points (the field pair sum of field.hip with the
// N force points as field points: sources w_q v[nu(q)] gathered once, chunk
// partial sums), then the fixed-order chunk sum with the rigid-body motion
// and the balance rows in one launch (k_apply_stage2).  `chunks` bounds the
// partial buffer (at least field_plan(N, Q).cap).
hipError_t launch_apply(const nrs_problem& pb, const Sorted& srt, const double* v, double* y,
                        double* part, int32_t chunks, const int32_t* stop, hipStream_t s) {
  const int64_t N = pb.N, Q = pb.Q;
  if (N > 0) {
    const FieldPlan fp = field_plan(N, Q);
    if (fp.chunks > chunks) return hipErrorInvalidValue;
    hipError_t e = launch_field_sources(N, Q, pb.X, pb.w, pb.nu, v, srt.fsrc, s, stop);
    if (e != hipSuccess) return e;
    e = launch_field_part(fp, N, Q, pb.x, nullptr, 0.0, srt.fsrc, pb.eps, part, s, stop);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((3 * N + 63) / 64 + pb.M);
    hipLaunchKernelGGL(k_apply_stage2, dim3(blocks), dim3(kApplyThreads), 0, s, N, pb.M,
                       fp.chunks, part, 1.0 / (8.0 * kPi * pb.mu), pb.x, pb.body, pb.Y, srt.W, v,
                       y, stop);
  }
  return hipGetLastError();
}

}  // namespace nrs
