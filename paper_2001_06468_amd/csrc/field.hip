// Flow at field points and passive tracers.
//
// The regularized single-layer equation (Sec. 3, eq. 19) holds at any point
// of the fluid, so the nearest-neighbour sum of eq. 23 with the collocation
// point replaced by a field point y gives the velocity there:
//   u(y) = (8 pi mu)^-1 sum_q S^eps(y - X_q) w_q f[nu(q)].
// It is the flow the particle-tracking experiments (Sec. 4.3, Sec. 5.2)
// integrate for their tracers.
//
// Layout: a pre-pass gathers every quadrature point into one 64-byte record
// (position and g_q = w_q f[nu(q)]), so the pair loop reads a record with a
// single wave-uniform scalar load and keeps all 64 lanes on distinct field
// points; the q range is cut into chunks so that even a few hundred tracers
// fill the chip, and the chunk sums are added in a fixed order.
#include <algorithm>

#include "nrs_internal.h"

namespace nrs {

namespace {

constexpr int kFieldThreads = 256;  // four waves, one field point per lane
constexpr int kFieldWaves = kFieldThreads / 64;

// 1/sqrt(d) for d > 0: the hardware estimate r0 (relative error about
// 2^-23) corrected by the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3)
// with e = 1 - d r0^2, i.e. one third-order step; the neglected terms are
// about 2^-69, so the result is within rounding of the correctly rounded value.
__device__ inline double rsqrt_refined(double d) {
  const double r0 = __builtin_amdgcn_rsq(d);
  const double e = fma(-(d * r0), r0, 1.0);
  return fma(r0 * e, fma(e, 0.375, 0.5), r0);
}

// Eight lanes per record, one double each, so that consecutive lanes store
// consecutive doubles.
__global__ void k_field_sources(int64_t N, int64_t Q, const double* __restrict__ X,
                                const double* __restrict__ w, const int32_t* __restrict__ nu,
                                const double* __restrict__ f, double* __restrict__ src,
                                const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t q = i >> 3;
  const int k = (int)(i & 7);
  if (q >= Q) return;
  double v = 0.0;
  if (k < 3) {
    v = X[k * Q + q];
  } else if (k < 6) {
    const int32_t n = nu[q];
    if (n >= 0 && n < N) v = (w ? w[q] : 1.0) * f[(k - 3) * N + n];
  }
  src[i] = v;
}

// Workgroups are dealt to the eight XCDs in turn (XCD = b mod 8).  With at
// least eight chunks, workgroup b = 8 (pb + pblocks k) + x takes field-point
// block pb and chunk 8k + x, so every workgroup that reads chunk ch runs on
// XCD ch mod 8 and each XCD's L2 holds only its eighth of the records
// (workgroups past the last chunk exit at once).  With fewer chunks,
// workgroup b takes chunk b mod chunks of block b div chunks.  Wave w sums a
// contiguous quarter of the chunk; the four wave sums are added in a fixed
// order.  With K != NULL the field points are the RK stage positions y + c K.
__global__ __launch_bounds__(kFieldThreads) void k_field_part(
    int64_t P, int64_t Q, int64_t pblocks, int32_t chunks, int64_t chunk,
    const double* __restrict__ y, const double* __restrict__ K, double c,
    const FieldSrc* __restrict__ src, double eps2, double* __restrict__ part,
    const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double red[3][kFieldWaves][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int32_t ch;
  int64_t pb;
  if (chunks >= 8) {
    const int64_t j = blockIdx.x >> 3;
    pb = j % pblocks;
    ch = 8 * (int32_t)(j / pblocks) + (int32_t)(blockIdx.x & 7);
    if (ch >= chunks) return;
  } else {
    ch = blockIdx.x % chunks;
    pb = blockIdx.x / chunks;
  }
  const int64_t p = pb * 64 + lane;
  double px = 0.0, py = 0.0, pz = 0.0;
  if (p < P) {
    px = y[p];
    py = y[P + p];
    pz = y[2 * P + p];
    if (K) {
      px += c * K[p];
      py += c * K[P + p];
      pz += c * K[2 * P + p];
    }
  }
  // this wave's records [a, a + cnt) (Q < 2^31), kept wave-uniform
  const int64_t q0 = (int64_t)ch * chunk;
  const int64_t q1 = min<int64_t>(Q, q0 + chunk);
  const int64_t per = (q1 - q0 + kFieldWaves - 1) / kFieldWaves;
  const int64_t a64 = min<int64_t>(q1, q0 + w * per);
  const int a = __builtin_amdgcn_readfirstlane((int)a64);
  const int cnt = __builtin_amdgcn_readfirstlane((int)(min<int64_t>(q1, a64 + per) - a64));
  const FieldSrc* __restrict__ sw = src + a;
  double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll 2
  for (int k = 0; k < cnt; ++k) {
    const FieldSrc s = sw[k];
    const double rx = px - s.X, ry = py - s.Y, rz = pz - s.Z;
    const double d = fma(rz, rz, fma(ry, ry, fma(rx, rx, eps2)));
    const double r = rsqrt_refined(d);                           // (|r|^2 + eps^2)^(-1/2)
    const double t = r * r * r;                                  // (|r|^2 + eps^2)^(-3/2)
    const double rg = fma(rz, s.gz, fma(ry, s.gy, rx * s.gx));  // r . g
    const double al = fma(t, eps2, r);                           // (|r|^2 + 2 eps^2) t
    const double be = t * rg;
    ux = fma(al, s.gx, fma(be, rx, ux));
    uy = fma(al, s.gy, fma(be, ry, uy));
    uz = fma(al, s.gz, fma(be, rz, uz));
  }
  red[0][w][lane] = ux;
  red[1][w][lane] = uy;
  red[2][w][lane] = uz;
  __syncthreads();
  if (w < 3 && p < P) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kFieldWaves; ++k) acc += red[w][k][lane];
    part[(int64_t)ch * 3 * P + w * P + p] = acc;
  }
}

// u[i] = scale * sum over chunks of part[c][i], i < 3P, chunks added in a
// fixed order: wave w of kSumWaves takes a contiguous share of the chunks
// with four running sums (all four loads of a step in flight together), then
// the wave sums are added in wave order.
constexpr int kSumWaves = 16;
__global__ __launch_bounds__(kSumWaves * 64) void k_field_sum(int64_t n3, int32_t chunks,
                                                             const double* __restrict__ part,
                                                             double scale, double* __restrict__ u) {
  __shared__ double red[kSumWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = blockIdx.x * (int64_t)64 + lane;
  const int per = (chunks + kSumWaves - 1) / kSumWaves;
  const int c0 = min(chunks, w * per), c1 = min(chunks, c0 + per);
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (i < n3) {
    int c = c0;
    for (; c + 3 < c1; c += 4) {
      a0 += part[(int64_t)c * n3 + i];
      a1 += part[(int64_t)(c + 1) * n3 + i];
      a2 += part[(int64_t)(c + 2) * n3 + i];
      a3 += part[(int64_t)(c + 3) * n3 + i];
    }
    for (; c < c1; ++c) a0 += part[(int64_t)c * n3 + i];
  }
  red[w][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (w != 0 || i >= n3) return;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kSumWaves; ++k) acc += red[k][lane];
  u[i] = scale * acc;
}

// y += dt/6 (K1 + 2 K2 + 2 K3 + K4) over the 3P tracer coordinates.
__global__ void k_tracer_combine(int64_t n3, double* __restrict__ y, const double* __restrict__ K1,
                                 const double* __restrict__ K2, const double* __restrict__ K3,
                                 const double* __restrict__ K4, double dt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n3) y[i] = y[i] + (dt / 6.0) * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);
}

}  // namespace

// At most 2048 workgroups while there are fewer field-point blocks than that:
// eight per CU, all resident at once (a ninth workgroup on a few CUs would run
// alone after the others).
FieldPlan field_plan(int64_t P, int64_t Q) {
  FieldPlan fp;
  fp.pblocks = (P + 63) / 64;
  int64_t c = 2048 / std::max<int64_t>(fp.pblocks, 1);
  c = std::min<int64_t>(c, std::max<int64_t>(1, Q / 256));
  c = std::max<int64_t>(1, std::min<int64_t>(c, 1024));
  if (c >= 8) c -= c % 8;  // whole rounds of the eight XCDs
  fp.cap = (int32_t)c;
  fp.chunk = (Q + c - 1) / c;
  fp.chunks = (int32_t)((Q + fp.chunk - 1) / fp.chunk);
  return fp;
}

hipError_t launch_field_sources(int64_t N, int64_t Q, const double* X, const double* w,
                                const int32_t* nu, const double* f, FieldSrc* src,
                                hipStream_t s, const int32_t* stop) {
  hipLaunchKernelGGL(k_field_sources, dim3((unsigned)((8 * Q + 255) / 256)), dim3(256), 0, s, N, Q,
                     X, w, nu, f, reinterpret_cast<double*>(src), stop);
  return hipGetLastError();
}

hipError_t launch_field_part(const FieldPlan& fp, int64_t P, int64_t Q, const double* y,
                             const double* K, double c, const FieldSrc* src, double eps,
                             double* part, hipStream_t s, const int32_t* stop) {
  if (P <= 0) return hipSuccess;
  const int64_t slots = fp.chunks >= 8 ? 8 * ((fp.chunks + 7) / 8) : fp.chunks;
  const unsigned grid = (unsigned)(fp.pblocks * slots);
  hipLaunchKernelGGL(k_field_part, dim3(grid), dim3(kFieldThreads), 0, s, P, Q, fp.pblocks,
                     fp.chunks, fp.chunk, y, K, c, src, eps * eps, part, stop);
  return hipGetLastError();
}

hipError_t launch_field(const FieldPlan& fp, int64_t P, int64_t Q, const double* y,
                        const double* K, double c, const FieldSrc* src, double eps, double mu,
                        double* part, double* u, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  hipError_t e = launch_field_part(fp, P, Q, y, K, c, src, eps, part, s, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_field_sum, dim3((unsigned)((3 * P + 63) / 64)), dim3(kSumWaves * 64), 0, s,
                     3 * P, fp.chunks, part, 1.0 / (8.0 * kPi * mu), u);
  return hipGetLastError();
}

hipError_t launch_tracer_combine(int64_t P, double* y, const double* K1, const double* K2,
                                 const double* K3, const double* K4, double dt, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tracer_combine, dim3((unsigned)((3 * P + 255) / 256)), dim3(256), 0, s,
                     3 * P, y, K1, K2, K3, K4, dt);
  return hipGetLastError();
}

}  // namespace nrs
