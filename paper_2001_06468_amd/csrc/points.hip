// Geometry at time t, nearest-neighbour map and the nu-sorted (CSR) layout of
// the quadrature points.
#include "nrs_internal.h"

namespace nrs {

namespace {

// Body-frame wave displacement and derivatives of one point.
__device__ inline void wave_terms(const double* __restrict__ wave, int p, double s, double t,
                                  double d[3], double dds[3], double ddt[3]) {
  const double* wp = wave + 6 * p;
  const double beta = wp[0], A0 = wp[1], A1 = wp[2], k = wp[3], om = wp[4], phi = wp[5];
  const double th = k * s - om * t + phi;
  double sn, cs;
  sincos(th, &sn, &cs);
  const double amp = A0 + A1 * s;
  d[0] = beta * s;
  d[1] = amp * sn;
  d[2] = 0.0;
  dds[0] = beta;
  dds[1] = A1 * sn + amp * k * cs;
  dds[2] = 0.0;
  ddt[0] = 0.0;
  ddt[1] = -om * amp * cs;
  ddt[2] = 0.0;
}

// One point set of a scene for k_geometry.  mode 0: force points ->
// positions and prescribed velocities; mode 1: quadrature points ->
// positions and weights.
struct GeomSet {
  int64_t n;
  int32_t mode;
  const double* xi;
  const int32_t* body;
  const int32_t* part;
  const double* s;
  const double* aux;
  double* pos;
  double* out2;
};

__device__ inline void geometry_point(const GeomSet& g, int64_t i, int32_t M, int32_t P,
                                      const double* __restrict__ wave,
                                      const double* __restrict__ Y, double t) {
  const int64_t n = g.n;
  const int mode = g.mode;
  const double* __restrict__ xi = g.xi;
  const int32_t* __restrict__ body = g.body;
  const int32_t* __restrict__ part = g.part;
  const double* __restrict__ s = g.s;
  const double* __restrict__ aux = g.aux;
  double* __restrict__ pos = g.pos;
  double* __restrict__ out2 = g.out2;
  double p[3] = {xi[i], xi[n + i], xi[2 * n + i]};
  double d[3] = {0, 0, 0}, dds[3] = {0, 0, 0}, ddt[3] = {0, 0, 0};
  // out-of-range indices are treated as "none" (no wave / fixed point)
  const int pi = (part[i] >= 0 && part[i] < P) ? part[i] : -1;
  if (pi >= 0) {
    wave_terms(wave, pi, s[i], t, d, dds, ddt);
    p[0] += d[0];
    p[1] += d[1];
    p[2] += d[2];
  }
  const int b = (body[i] >= 0 && body[i] < M) ? body[i] : -1;
  double q[3], v[3];
  if (b >= 0) {
    const double* Yb = Y + 12 * b;
    for (int r = 0; r < 3; ++r) {
      q[r] = Yb[r] + (Yb[3 + 3 * r] * p[0] + Yb[4 + 3 * r] * p[1] + Yb[5 + 3 * r] * p[2]);
      v[r] = Yb[3 + 3 * r] * ddt[0] + Yb[4 + 3 * r] * ddt[1] + Yb[5 + 3 * r] * ddt[2];
    }
  } else {
    q[0] = p[0];
    q[1] = p[1];
    q[2] = p[2];
    v[0] = v[1] = v[2] = 0.0;
  }
  if (pos) {
    pos[i] = q[0];
    pos[n + i] = q[1];
    pos[2 * n + i] = q[2];
  }
  if (out2) {
    if (mode == 0) {
      if (b < 0) {
        v[0] = aux[i];
        v[1] = aux[n + i];
        v[2] = aux[2 * n + i];
      }
      out2[i] = v[0];
      out2[n + i] = v[1];
      out2[2 * n + i] = v[2];
    } else {
      double w = aux[i];
      if (pi >= 0) w *= sqrt(dds[0] * dds[0] + dds[1] * dds[1] + dds[2] * dds[2]);
      out2[i] = w;
    }
  }
}

// Both point sets of a scene in one launch: the first nb0 workgroups take
// set 0 (force points), the rest set 1 (quadrature points).
__global__ void k_geometry(GeomSet g0, GeomSet g1, int64_t nb0, int32_t M, int32_t P,
                           const double* __restrict__ wave, const double* __restrict__ Y,
                           double t) {
  const bool first = blockIdx.x < nb0;
  const GeomSet& g = first ? g0 : g1;
  const int64_t i = (blockIdx.x - (first ? 0 : nb0)) * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  geometry_point(g, i, M, P, wave, Y, t);
}

// One thread per quadrature point; force points of the block's groups are
// staged through LDS.  Squared distance without contraction so that the
// result equals the (dx*dx + dy*dy) + dz*dz of a plain FP64 evaluation.
constexpr int kNnBlock = 256;
__global__ __launch_bounds__(kNnBlock) void k_nearest(int64_t N, const double* __restrict__ x,
                                                      GroupTable gt, int64_t Q,
                                                      const double* __restrict__ X,
                                                      const int32_t* __restrict__ groupX,
                                                      int32_t* __restrict__ nu) {
#pragma clang fp contract(off)
  __shared__ double sx[kNnBlock], sy[kNnBlock], sz[kNnBlock];
  __shared__ int s_lo, s_hi;
  const int64_t q = blockIdx.x * (int64_t)kNnBlock + threadIdx.x;
  const bool active = q < Q;
  int lo = 0, hi = 0;
  double qx = 0, qy = 0, qz = 0;
  if (active) {
    const int g = groupX[q];
    if (g >= 0 && g < gt.G) {
      lo = gt.off[g];
      hi = gt.off[g + 1];
    }
    qx = X[q];
    qy = X[Q + q];
    qz = X[2 * Q + q];
  }
  if (threadIdx.x == 0) {
    s_lo = 0x7fffffff;
    s_hi = -1;
  }
  __syncthreads();
  if (active && hi > lo) {
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
  }
  __syncthreads();
  const int blo = s_lo, bhi = s_hi;
  double best = __builtin_huge_val();
  int arg = -1;
  for (int base = blo; base < bhi; base += kNnBlock) {
    const int j = base + threadIdx.x;
    if (j < bhi) {
      sx[threadIdx.x] = x[j];
      sy[threadIdx.x] = x[N + j];
      sz[threadIdx.x] = x[2 * N + j];
    }
    __syncthreads();
    const int cnt = min(kNnBlock, bhi - base);
    for (int c = 0; c < cnt; ++c) {
      const int nidx = base + c;
      if (nidx >= lo && nidx < hi) {
        const double dx = sx[c] - qx;
        const double dy = sy[c] - qy;
        const double dz = sz[c] - qz;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < best || arg < 0) {
          best = d2;
          arg = nidx;
        }
      }
    }
    __syncthreads();
  }
  if (active) nu[q] = arg;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Quadrature points whose nu is outside [0, N) are left out of the layout and
// counted in cnt[N + 1] (reported as an argument error by the caller).
__global__ void k_csr_count(int64_t N, int64_t Q, const int32_t* __restrict__ nu, int32_t* cnt) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < Q) {
    const int32_t v = nu[q];
    if (v >= 0 && v < N)
      atomicAdd(&cnt[v], 1);
    else
      atomicAdd(&cnt[N + 1], 1);
  }
}

// Exclusive scan of cnt[0..N) into seg[0..N]; cnt becomes the scatter cursor.
// st (may be NULL): argument error when some nu was outside [0, N) (counted
// in cnt[N + 1]).
constexpr int kScanBlock = 1024;

// Exclusive scan of one value per thread over a kScanBlock workgroup: a
// shuffle scan inside each wavefront, then the wavefronts' totals scanned by
// wavefront 0 (two barriers); *total receives the sum over the workgroup.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* wtot, int32_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wtot[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int32_t t = lane < kScanBlock / 64 ? wtot[lane] : 0;
#pragma unroll
    for (int off = 1; off < kScanBlock / 64; off <<= 1) {
      const int32_t y = __shfl_up(t, off, 64);
      if (lane >= off) t += y;
    }
    if (lane < kScanBlock / 64) wtot[lane] = t;
  }
  __syncthreads();
  *total = wtot[kScanBlock / 64 - 1];
  return x - v + (wv ? wtot[wv - 1] : 0);
}

__global__ __launch_bounds__(kScanBlock) void k_csr_scan(int64_t N, int32_t* cnt, int32_t* seg,
                                                         SolveState* st) {
  if (threadIdx.x == 0 && st && cnt[N + 1] > 0) {
    st->nonfinite = 2;
    st->failed = 1;
    st->stop = 1;
  }
  __shared__ int32_t wtot[kScanBlock / 64];
  const int tid = threadIdx.x;
  const int64_t per = (N + kScanBlock - 1) / kScanBlock;
  const int64_t a = tid * per, b = min<int64_t>(N, a + per);
  int32_t sum = 0;
  for (int64_t i = a; i < b; ++i) sum += cnt[i];
  int32_t total;
  int32_t run = block_exclusive_scan(sum, wtot, &total);
  for (int64_t i = a; i < b; ++i) {
    const int32_t c = cnt[i];
    seg[i] = run;
    cnt[i] = run;
    run += c;
  }
  if (tid == kScanBlock - 1) seg[N] = total;
}

// Count, scan and scatter in one workgroup with the counters in LDS, for
// N <= kCsrSmallN and Q <= kCsrSmallQ (the single-system workloads): the
// same segments (seg) as the three-kernel path; the order inside a segment
// is arbitrary until k_csr_finish sorts it.
constexpr int64_t kCsrSmallN = 8192;
constexpr int64_t kCsrSmallQ = 1 << 17;
__global__ __launch_bounds__(kScanBlock) void k_csr_small(int64_t N, int64_t Q,
                                                          const int32_t* __restrict__ nu,
                                                          int32_t* __restrict__ seg,
                                                          int32_t* __restrict__ perm,
                                                          SolveState* st) {
  __shared__ int32_t c[kCsrSmallN + 2];
  __shared__ int32_t wtot[kScanBlock / 64];
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < N + 2; i += kScanBlock) c[i] = 0;
  __syncthreads();
  for (int64_t q = tid; q < Q; q += kScanBlock) {
    const int32_t v = nu[q];
    atomicAdd(&c[(v >= 0 && v < N) ? v : N + 1], 1);
  }
  __syncthreads();
  if (tid == 0 && st && c[N + 1] > 0) {
    st->nonfinite = 2;
    st->failed = 1;
    st->stop = 1;
  }
  const int64_t per = (N + kScanBlock - 1) / kScanBlock;
  const int64_t a = tid * per, b = min<int64_t>(N, a + per);
  int32_t sum = 0;
  for (int64_t i = a; i < b; ++i) sum += c[i];
  int32_t total;
  int32_t run = block_exclusive_scan(sum, wtot, &total);
  for (int64_t i = a; i < b; ++i) {
    const int32_t k = c[i];
    seg[i] = run;
    c[i] = run;
    run += k;
  }
  if (tid == kScanBlock - 1) seg[N] = total;
  __syncthreads();
  for (int64_t q = tid; q < Q; q += kScanBlock) {
    const int32_t v = nu[q];
    if (v >= 0 && v < N) perm[atomicAdd(&c[v], 1)] = (int32_t)q;
  }
}

__global__ void k_csr_scatter(int64_t N, int64_t Q, const int32_t* __restrict__ nu,
                              int32_t* cursor, int32_t* perm) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < Q) {
    const int32_t v = nu[q];
    if (v >= 0 && v < N) {
      const int pos = atomicAdd(&cursor[v], 1);
      perm[pos] = (int32_t)q;
    }
  }
}

// Per segment (one wavefront each): order the members by original index
// (deterministic layout), pack the sorted coordinates and sum the patch
// weight.  A member's place is the number of members with a smaller index
// (the indices are distinct), found by comparing against every member
// broadcast from its lane; segments longer than 256 members (not met by
// the workloads) are sorted by insertion in lane 0.
constexpr int kFinishWaves = 4;
__device__ inline double csr_store(int64_t Q, int64_t n, int pos, int q, const double* __restrict__ X,
                                   const double* __restrict__ w, int32_t* __restrict__ perm,
                                   int32_t* __restrict__ nus, double4* __restrict__ X64,
                                   float4* __restrict__ X32hi, float4* __restrict__ X32lo) {
  const double px = X[q], py = X[Q + q], pz = X[2 * Q + q];
  const double wq = w ? w[q] : 1.0;
  perm[pos] = q;
  nus[pos] = (int32_t)n;
  X64[pos] = make_double4(px, py, pz, wq);
  const float hx = (float)px, hy = (float)py, hz = (float)pz;
  X32hi[pos] = make_float4(hx, hy, hz, (float)wq);
  X32lo[pos] = make_float4((float)(px - (double)hx), (float)(py - (double)hy),
                           (float)(pz - (double)hz), 0.0f);
  return wq;
}

__global__ __launch_bounds__(kFinishWaves * 64) void k_csr_finish(
    int64_t N, int64_t Q, const int32_t* __restrict__ seg, int32_t* __restrict__ perm,
    const double* __restrict__ X, const double* __restrict__ w, int32_t* __restrict__ nus,
    double4* __restrict__ X64, float4* __restrict__ X32hi, float4* __restrict__ X32lo,
    double* __restrict__ W) {
  // weights by sorted position, so that the patch weight is summed in an
  // order that does not depend on the (atomic, unordered) scatter
  __shared__ double s_w[kFinishWaves][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * kFinishWaves + wv;
  if (n >= N) return;
  const int a = seg[n], len = seg[n + 1] - a;
  double wsum = 0.0;
  if (len <= 256) {
    int key[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) key[c] = c * 64 + lane < len ? perm[a + c * 64 + lane] : 0x7fffffff;
    int rank[4] = {0, 0, 0, 0};
#pragma unroll
    for (int cj = 0; cj < 4; ++cj) {
      if (cj * 64 < len) {   // wave-uniform
        const int top = min(64, len - cj * 64);
        for (int jj = 0; jj < top; ++jj) {
          const int kj = __shfl(key[cj], jj, 64);
#pragma unroll
          for (int c = 0; c < 4; ++c) rank[c] += kj < key[c] ? 1 : 0;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c * 64 + lane < len)
        s_w[wv][rank[c]] = csr_store(Q, n, a + rank[c], key[c], X, w, perm, nus, X64, X32hi, X32lo);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // lane l adds sorted places l, l + 64, ...; then a fixed tree over lanes
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c * 64 + lane < len) wsum += s_w[wv][c * 64 + lane];
  } else if (lane == 0) {
    for (int i = a + 1; i < a + len; ++i) {
      const int32_t k = perm[i];
      int j = i - 1;
      while (j >= a && perm[j] > k) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = k;
    }
    for (int i = a; i < a + len; ++i) wsum += csr_store(Q, n, i, perm[i], X, w, perm, nus, X64, X32hi, X32lo);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wsum += __shfl_xor(wsum, o, 64);
  if (lane == 0) W[n] = wsum;
}

inline dim3 grid1(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_geometry(const nrs_scene& sc, double t, const double* Y, double* x, double* X,
                           double* w, double* u, hipStream_t s) {
  GeomSet g0 = {(sc.N > 0 && (x || u)) ? sc.N : 0, 0, sc.xi, sc.body, sc.part, sc.s, sc.ufix, x, u};
  GeomSet g1 = {(sc.Q > 0 && (X || w)) ? sc.Q : 0, 1, sc.Xi, sc.bodyX, sc.partX, sc.sX, sc.w0, X, w};
  const int64_t nb0 = (g0.n + 255) / 256, nb1 = (g1.n + 255) / 256;
  if (nb0 + nb1 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geometry, dim3((unsigned)(nb0 + nb1)), dim3(256), 0, s, g0, g1, nb0, sc.M,
                     sc.P, sc.wave, Y, t);
  return hipGetLastError();
}

hipError_t launch_nearest(int64_t N, const double* x, const GroupTable& gt, int64_t Q,
                          const double* X, const int32_t* groupX, int32_t* nu, hipStream_t s) {
  if (Q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nearest, grid1(Q, kNnBlock), dim3(kNnBlock), 0, s, N, x, gt, Q, X, groupX,
                     nu);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, grid1(n, 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, grid1(n, 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_build_csr(int64_t N, int64_t Q, const double* X, const double* w,
                            const int32_t* nu, Sorted& srt, SolveState* st, hipStream_t s) {
  if (N <= kCsrSmallN && Q <= kCsrSmallQ) {
    hipLaunchKernelGGL(k_csr_small, dim3(1), dim3(kScanBlock), 0, s, N, Q, nu, srt.seg, srt.perm,
                       st);
  } else {
    hipError_t e = launch_fill_i32(srt.cnt, 0, N + 2, s);
    if (e != hipSuccess) return e;
    if (Q > 0) {
      hipLaunchKernelGGL(k_csr_count, grid1(Q, 256), dim3(256), 0, s, N, Q, nu, srt.cnt);
    }
    hipLaunchKernelGGL(k_csr_scan, dim3(1), dim3(kScanBlock), 0, s, N, srt.cnt, srt.seg, st);
    if (Q > 0) {
      hipLaunchKernelGGL(k_csr_scatter, grid1(Q, 256), dim3(256), 0, s, N, Q, nu, srt.cnt,
                         srt.perm);
    }
  }
  hipLaunchKernelGGL(k_csr_finish, dim3((unsigned)((N + kFinishWaves - 1) / kFinishWaves)),
                     dim3(kFinishWaves * 64), 0, s, N, Q, srt.seg, srt.perm, X, w, srt.nus, srt.X64,
                     srt.X32hi, srt.X32lo, srt.W);
  return hipGetLastError();
}

}  // namespace nrs
