// Learned warm start: a per-point network with pooled body context that
// predicts, in each free body's own frame, the force density at its force
// points and the body's (U, Omega).  One workgroup handles one body: its
// points' features and hidden states live in LDS, lane j of every wave owns
// hidden unit j (H = 64 = one wavefront), waves take points round-robin.
//
//   h1_m = tanh(W1 phi_m + b1),          c = mean_m h1_m
//   h2_m = tanh(W2 h1_m + V2 c + b2),    d = mean_m h2_m
//   y_m  = W3 h2_m + b3,                 z = W4 d + b4
//
// Training: one workgroup per selected body runs the forward pass, the loss
// (mean over bodies of the point MSE + body MSE) and the reverse pass, and
// writes its gradient row; a second kernel sums the rows in a fixed order
// (deterministic), then Adam updates the parameters.
#include <cmath>

#include "nrs_internal.h"

namespace nrs {
namespace {

constexpr int kH = kMlpHidden;    // hidden width (one wavefront)
constexpr int kF = 7;             // input features
constexpr int kO = 3;             // point outputs
constexpr int kP = 6;             // body outputs
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// offsets of the parameter groups in the flat vector
constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kH * kF;
constexpr int oW2 = ob1 + kH;
constexpr int oV2 = oW2 + kH * kH;
constexpr int ob2 = oV2 + kH * kH;
constexpr int oW3 = ob2 + kH;
constexpr int ob3 = oW3 + kO * kH;
constexpr int oW4 = ob3 + kO;
constexpr int ob4 = oW4 + kP * kH;
constexpr int kCount = ob4 + kP;
static_assert(kCount == kMlpParams, "parameter layout");

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct MlpShared {
  float phi[kMlpMaxPts][8];
  float h1[kMlpMaxPts][kH];
  float h2[kMlpMaxPts][kH];
  float y[kMlpMaxPts][4];      // outputs, then their gradients
  float c[kH], d[kH], vc[kH], sa2[kH], vs2[kH];
  float part[kWaves][kH];
  float z[8], dz[8];
  float red[kWaves];
};

// Forward pass of one body (points p0 .. p0+n-1 of phi).  Leaves h1, h2, c,
// d, y and z in LDS.
__device__ void body_forward(MlpShared& S, const float* __restrict__ th,
                             const float* __restrict__ phi, int64_t p0, int n) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < n * kF; e += kThreads) {
    const int p = e / kF, f = e - p * kF;
    S.phi[p][f] = phi[(p0 + p) * kF + f];
  }
  __syncthreads();
  float w1[kF];
#pragma unroll
  for (int f = 0; f < kF; ++f) w1[f] = th[oW1 + lane * kF + f];
  const float b1 = th[ob1 + lane];
  float acc = 0.f;
  for (int p = w; p < n; p += kWaves) {
    float a = b1;
#pragma unroll
    for (int f = 0; f < kF; ++f) a = fmaf(w1[f], S.phi[p][f], a);
    const float h = tanhf(a);
    S.h1[p][lane] = h;
    acc += h;
  }
  S.part[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) s += S.part[q][lane];
    S.c[lane] = s / (float)n;
  }
  __syncthreads();
  // V2 c + b2, then the second layer with W2's row `lane` in registers
  if (w == 0) {
    float a = th[ob2 + lane];
    for (int i = 0; i < kH; ++i) a = fmaf(th[oV2 + lane * kH + i], S.c[i], a);
    S.vc[lane] = a;
  }
  float w2[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) w2[i] = th[oW2 + lane * kH + i];
  __syncthreads();
  const float vcl = S.vc[lane];
  acc = 0.f;
  for (int p = w; p < n; p += kWaves) {
    float a = vcl;
#pragma unroll
    for (int i = 0; i < kH; ++i) a = fmaf(w2[i], S.h1[p][i], a);
    const float h = tanhf(a);
    S.h2[p][lane] = h;
    acc += h;
  }
  S.part[w][lane] = acc;
  const float w30 = th[oW3 + lane], w31 = th[oW3 + kH + lane], w32 = th[oW3 + 2 * kH + lane];
  for (int p = w; p < n; p += kWaves) {
    const float h = S.h2[p][lane];
    const float y0 = wave_sum(w30 * h), y1 = wave_sum(w31 * h), y2 = wave_sum(w32 * h);
    if (lane == 0) {
      S.y[p][0] = y0 + th[ob3];
      S.y[p][1] = y1 + th[ob3 + 1];
      S.y[p][2] = y2 + th[ob3 + 2];
    }
  }
  __syncthreads();
  if (w == 0) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) s += S.part[q][lane];
    const float dl = s / (float)n;
    S.d[lane] = dl;
#pragma unroll
    for (int o = 0; o < kP; ++o) {
      const float v = wave_sum(th[oW4 + o * kH + lane] * dl);
      if (lane == 0) S.z[o] = v + th[ob4 + o];
    }
  }
  __syncthreads();
}

// Point range of body b; false (and err bit 1) if b or its range is invalid.
__device__ inline bool body_range(const int32_t* __restrict__ body_off, int b, int32_t nbodies,
                                  int64_t npts, int64_t& p0, int& n, int32_t* err) {
  if (b < 0 || b >= nbodies) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return false;
  }
  const int64_t lo = body_off[b], hi = body_off[b + 1];
  if (lo < 0 || hi > npts || hi - lo > kMlpMaxPts || hi < lo) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return false;
  }
  p0 = lo;
  n = (int)(hi - lo);
  return n > 0;
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(
    const float* __restrict__ th, int32_t nbodies, int64_t npts,
    const int32_t* __restrict__ body_off, const int32_t* __restrict__ sel,
    const float* __restrict__ phi, float* __restrict__ y, float* __restrict__ z,
    int32_t* __restrict__ err) {
  __shared__ MlpShared S;
  const int b = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  int64_t p0;
  int n;
  if (!body_range(body_off, b, nbodies, npts, p0, n, err)) return;
  body_forward(S, th, phi, p0, n);
  for (int e = threadIdx.x; e < n * kO; e += kThreads) {
    const int p = e / kO, o = e - p * kO;
    y[(p0 + p) * kO + o] = S.y[p][o];
  }
  if (threadIdx.x < kP) z[(int64_t)b * kP + threadIdx.x] = S.z[threadIdx.x];
}

// Forward + loss + reverse pass of selected body blockIdx.x; writes the row
// grad_rows[blockIdx.x][0 .. kCount] (last entry: the body's loss share).
__global__ __launch_bounds__(kThreads) void k_mlp_grad(
    const float* __restrict__ th, int32_t nbodies, int64_t npts,
    const int32_t* __restrict__ body_off,
    const int32_t* __restrict__ sel, int32_t nsel, const float* __restrict__ phi,
    const float* __restrict__ t_pt, const float* __restrict__ t_body,
    float* __restrict__ grad_rows, int32_t* __restrict__ err) {
  __shared__ MlpShared S;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int b = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  float* __restrict__ g = grad_rows + (int64_t)blockIdx.x * (kCount + 1);
  int64_t p0;
  int n;
  if (!body_range(body_off, b, nbodies, npts, p0, n, err)) {
    for (int e = tid; e <= kCount; e += kThreads) g[e] = 0.f;
    return;
  }
  body_forward(S, th, phi, p0, n);
  const float invM = 1.f / (float)nsel;
  // output gradients and the loss share
  float lsum = 0.f;
  for (int e = tid; e < n * kO; e += kThreads) {
    const int p = e / kO, o = e - p * kO;
    const float r = S.y[p][o] - t_pt[(p0 + p) * kO + o];
    lsum += r * r;
    S.y[p][o] = 2.f * r * invM / (float)(n * kO);
  }
  lsum = wave_sum(lsum) / (float)(n * kO);
  float zs = 0.f;
  if (w == 0 && lane < kP) {
    const float r = S.z[lane] - t_body[(int64_t)b * kP + lane];
    zs = r * r;
    S.dz[lane] = 2.f * r * invM / (float)kP;
  }
  zs = wave_sum(zs) / (float)kP;
  if (lane == 0) S.red[w] = lsum + (w == 0 ? zs : 0.f);
  __syncthreads();
  if (tid == 0) g[kCount] = (S.red[0] + S.red[1] + S.red[2] + S.red[3]) * invM;
  // dW4, db4 (outer products with d)
  for (int e = tid; e < kP * kH; e += kThreads) g[oW4 + e] = S.dz[e / kH] * S.d[e % kH];
  if (tid < kP) g[ob4 + tid] = S.dz[tid];
  // dW3, db3; then da2 = (W3^T dy + W4^T dz / n) (1 - h2^2) in place of h2
  {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    const float w30 = th[oW3 + lane], w31 = th[oW3 + kH + lane], w32 = th[oW3 + 2 * kH + lane];
    float bz = 0.f;
#pragma unroll
    for (int o = 0; o < kP; ++o) bz = fmaf(th[oW4 + o * kH + lane], S.dz[o], bz);
    bz /= (float)n;
    float s2 = 0.f;
    for (int p = w; p < n; p += kWaves) {
      const float h = S.h2[p][lane];
      const float d0 = S.y[p][0], d1 = S.y[p][1], d2 = S.y[p][2];
      a0 = fmaf(d0, h, a0);
      a1 = fmaf(d1, h, a1);
      a2 = fmaf(d2, h, a2);
      const float dh = fmaf(w30, d0, fmaf(w31, d1, fmaf(w32, d2, bz)));
      const float da = dh * (1.f - h * h);
      S.h2[p][lane] = da;
      s2 += da;
    }
    // fixed-order cross-wave sums through LDS
    __shared__ float cw[kWaves][4][kH];
    cw[w][0][lane] = a0;
    cw[w][1][lane] = a1;
    cw[w][2][lane] = a2;
    cw[w][3][lane] = s2;
    __syncthreads();
    if (w == 0) {
      float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) {
        r0 += cw[q][0][lane];
        r1 += cw[q][1][lane];
        r2 += cw[q][2][lane];
        r3 += cw[q][3][lane];
      }
      g[oW3 + lane] = r0;
      g[oW3 + kH + lane] = r1;
      g[oW3 + 2 * kH + lane] = r2;
      S.sa2[lane] = r3;
      g[ob2 + lane] = r3;
    }
    __syncthreads();
  }
  if (tid < kO) {
    float s = 0.f;
    for (int p = 0; p < n; ++p) s += S.y[p][tid];
    g[ob3 + tid] = s;
  }
  // dW2[j][i] = sum_p da2[p][j] h1[p][i];  dV2[j][i] = sa2[j] c[i]
  for (int e = tid; e < kH * kH; e += kThreads) {
    const int j = e / kH, i = e - j * kH;
    float s = 0.f;
    for (int p = 0; p < n; ++p) s = fmaf(S.h2[p][j], S.h1[p][i], s);
    g[oW2 + e] = s;
    g[oV2 + e] = S.sa2[j] * S.c[i];
  }
  // V2^T sa2 / n (lane = i)
  if (w == 0) {
    float s = 0.f;
    for (int j = 0; j < kH; ++j) s = fmaf(th[oV2 + j * kH + lane], S.sa2[j], s);
    S.vs2[lane] = s / (float)n;
  }
  float w2c[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) w2c[j] = th[oW2 + j * kH + lane];
  __syncthreads();
  // da1 = (W2^T da2 + V2^T sa2 / n) (1 - h1^2) in place of h1
  const float vs = S.vs2[lane];
  for (int p = w; p < n; p += kWaves) {
    float a = vs;
#pragma unroll
    for (int j = 0; j < kH; ++j) a = fmaf(w2c[j], S.h2[p][j], a);
    const float h = S.h1[p][lane];
    S.h1[p][lane] = a * (1.f - h * h);
  }
  __syncthreads();
  // dW1[i][f] = sum_p da1[p][i] phi[p][f];  db1[i] = sum_p da1[p][i]
  for (int e = tid; e < kH * (kF + 1); e += kThreads) {
    const int i = e / (kF + 1), f = e - i * (kF + 1);
    float s = 0.f;
    if (f < kF) {
      for (int p = 0; p < n; ++p) s = fmaf(S.h1[p][i], S.phi[p][f], s);
      g[oW1 + i * kF + f] = s;
    } else {
      for (int p = 0; p < n; ++p) s += S.h1[p][i];
      g[ob1 + i] = s;
    }
  }
}

// out[k] = sum over rows r (in order) of rows[r][k], k <= kCount
__global__ void k_mlp_reduce(const float* __restrict__ rows, int32_t nrows,
                             float* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > kCount) return;
  float s = 0.f;
  for (int r = 0; r < nrows; ++r) s += rows[(int64_t)r * (kCount + 1) + k];
  out[k] = s;
}

__global__ void k_adam(int64_t count, float* __restrict__ th, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float beta1,
                       float beta2, float eps, float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const float gk = g[k];
  const float mk = beta1 * m[k] + (1.f - beta1) * gk;
  const float vk = beta2 * v[k] + (1.f - beta2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  th[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ---- frames: body_off from the point-to-body map, features, targets, warm start

// start[b] / end[b] of body b's points; bad[0] set when a body's points are not
// contiguous (counted against the number of points labelled b).
// Body offsets from the point-to-body map.  The points of bodies 0..M-1
// must form one block in which the body index starts at 0, steps up by one
// at each change and ends at M-1 (every other point has body < 0 or >= M).
// Each point checks the changes on its two sides; starts[0] counts the
// block's beginnings (exactly one is allowed), and each run's first point
// writes its offset.
__device__ inline int32_t body_or_none(const int32_t* body, int64_t m, int64_t N, int32_t M) {
  if (m < 0 || m >= N) return -1;
  const int32_t b = body[m];
  return (b >= 0 && b < M) ? b : -1;
}

__global__ void k_body_runs(int64_t N, int32_t M, const int32_t* __restrict__ body,
                            int32_t* __restrict__ off, int32_t* __restrict__ starts,
                            int32_t* __restrict__ err) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int32_t b = body_or_none(body, m, N, M);
  if (b < 0) return;
  const int32_t prev = body_or_none(body, m - 1, N, M);
  const int32_t next = body_or_none(body, m + 1, N, M);
  if (prev != b) {
    if (!(prev == b - 1 || (b == 0 && prev < 0))) atomicOr(err, 2);
    if (b == 0 && prev < 0) atomicAdd(starts, 1);
    off[b] = (int32_t)m;
  }
  if (next != b) {
    if (!(next == b + 1 || (b == M - 1 && next < 0))) atomicOr(err, 2);
    if (b == M - 1) off[M] = (int32_t)(m + 1);
  }
}

__global__ void k_body_sizes(int32_t M, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ starts, int32_t* __restrict__ err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= M) return;
  const int32_t n = off[b + 1] - off[b];
  if (n <= 0 || n > kMlpMaxPts || (b == 0 && starts[0] != 1)) atomicOr(err, 2);
}

// phi[m] = (B^T (x_m - x0), B^T u_m, s_m) for points of bodies 0..M-1
__global__ void k_features(int64_t N, const double* __restrict__ x, const double* __restrict__ u,
                           const double* __restrict__ s, const int32_t* __restrict__ body,
                           int32_t M, const double* __restrict__ Y, float* __restrict__ phi) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int32_t b = body[m];
  float* out = phi + m * kF;
  if (b < 0 || b >= M) {
    for (int f = 0; f < kF; ++f) out[f] = 0.f;
    return;
  }
  const double* y = Y + (int64_t)b * 12;
  const double r[3] = {x[m] - y[0], x[N + m] - y[1], x[2 * N + m] - y[2]};
  const double v[3] = {u[m], u[N + m], u[2 * N + m]};
  for (int k = 0; k < 3; ++k) {
    // column k of B (row-major B[i][k] at y[3 + 3 i + k])
    const double bk0 = y[3 + k], bk1 = y[6 + k], bk2 = y[9 + k];
    out[k] = (float)(bk0 * r[0] + bk1 * r[1] + bk2 * r[2]);
    out[3 + k] = (float)(bk0 * v[0] + bk1 * v[1] + bk2 * v[2]);
  }
  out[6] = (float)s[m];
}

// Training targets from a solution sol = [f (3 x N component-major); (U, Omega) per body]
__global__ void k_targets(int64_t N, int32_t M, const int32_t* __restrict__ body,
                          const double* __restrict__ Y, const double* __restrict__ sol,
                          double sf, double su, double so, float* __restrict__ t_pt,
                          float* __restrict__ t_body) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) {
    const int32_t b = body[m];
    if (b >= 0 && b < M) {
      const double* y = Y + (int64_t)b * 12;
      const double f[3] = {sol[m], sol[N + m], sol[2 * N + m]};
      for (int k = 0; k < 3; ++k)
        t_pt[m * kO + k] = (float)((y[3 + k] * f[0] + y[6 + k] * f[1] + y[9 + k] * f[2]) / sf);
    } else {
      for (int k = 0; k < 3; ++k) t_pt[m * kO + k] = 0.f;
    }
  }
  if (m < M) {
    const double* y = Y + m * 12;
    const double* uw = sol + 3 * N + 6 * m;
    for (int k = 0; k < 3; ++k) {
      t_body[m * kP + k] =
          (float)((y[3 + k] * uw[0] + y[6 + k] * uw[1] + y[9 + k] * uw[2]) / su);
      t_body[m * kP + 3 + k] =
          (float)((y[3 + k] * uw[3] + y[6 + k] * uw[4] + y[9 + k] * uw[5]) / so);
    }
  }
}

// Lab-frame initial guess from the network outputs (inverse of k_targets);
// points outside the bodies get zero force density.
__global__ void k_to_lab(int64_t N, int32_t M, const int32_t* __restrict__ body,
                         const double* __restrict__ Y, const float* __restrict__ y,
                         const float* __restrict__ z, double sf, double su, double so,
                         double* __restrict__ x0) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) {
    const int32_t b = body[m];
    if (b >= 0 && b < M) {
      const double* B = Y + (int64_t)b * 12 + 3;
      const double q[3] = {y[m * kO], y[m * kO + 1], y[m * kO + 2]};
      for (int i = 0; i < 3; ++i)
        x0[i * N + m] = sf * (B[3 * i] * q[0] + B[3 * i + 1] * q[1] + B[3 * i + 2] * q[2]);
    } else {
      x0[m] = 0.0;
      x0[N + m] = 0.0;
      x0[2 * N + m] = 0.0;
    }
  }
  if (m < M) {
    const double* B = Y + m * 12 + 3;
    const float* zz = z + m * kP;
    double* o = x0 + 3 * N + 6 * m;
    for (int i = 0; i < 3; ++i) {
      o[i] = su * (B[3 * i] * zz[0] + B[3 * i + 1] * zz[1] + B[3 * i + 2] * zz[2]);
      o[3 + i] = so * (B[3 * i] * zz[3] + B[3 * i + 1] * zz[4] + B[3 * i + 2] * zz[5]);
    }
  }
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_mlp_forward(const float* th, int32_t nb, int32_t nbodies, int64_t npts,
                              const int32_t* body_off, const int32_t* sel, const float* phi,
                              float* y, float* z, int32_t* err, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)nb), dim3(kThreads), 0, s, th, nbodies, npts,
                     body_off, sel, phi, y, z, err);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* th, int32_t nbodies, int64_t npts,
                           const int32_t* body_off, const int32_t* sel, int32_t nsel,
                           const float* phi, const float* t_pt, const float* t_body, float* rows,
                           float* grad, int32_t* err, hipStream_t s) {
  if (nsel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)nsel), dim3(kThreads), 0, s, th, nbodies, npts,
                     body_off, sel, nsel, phi, t_pt, t_body, rows, err);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_for(kCount + 1, 256)), dim3(256), 0, s, rows, nsel,
                     grad);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* th, const float* g, float* m, float* v, int32_t t,
                       float lr, float beta1, float beta2, float eps, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(count, 256)), dim3(256), 0, s, count, th, g, m, v,
                     lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_body_off(int64_t N, int32_t M, const int32_t* body, int32_t* off,
                           int32_t* starts, int32_t* err, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipError_t e = launch_fill_i32(starts, 0, 1, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_i32(off, 0, (int64_t)M + 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_body_runs, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, M, body, off,
                     starts, err);
  hipLaunchKernelGGL(k_body_sizes, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, off, starts, err);
  return hipGetLastError();
}

hipError_t launch_features(int64_t N, const double* x, const double* u, const double* sarc,
                           const int32_t* body, int32_t M, const double* Y, float* phi,
                           hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, x, u, sarc, body, M,
                     Y, phi);
  return hipGetLastError();
}

hipError_t launch_targets(int64_t N, int32_t M, const int32_t* body, const double* Y,
                          const double* sol, const double* sc, float* t_pt, float* t_body,
                          hipStream_t s) {
  const int64_t n = N > M ? N : M;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_targets, dim3(blocks_for(n, 256)), dim3(256), 0, s, N, M, body, Y, sol,
                     sc[0], sc[1], sc[2], t_pt, t_body);
  return hipGetLastError();
}

hipError_t launch_to_lab(int64_t N, int32_t M, const int32_t* body, const double* Y,
                         const float* y, const float* z, const double* sc, double* x0,
                         hipStream_t s) {
  const int64_t n = N > M ? N : M;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_lab, dim3(blocks_for(n, 256)), dim3(256), 0, s, N, M, body, Y, y, z,
                     sc[0], sc[1], sc[2], x0);
  return hipGetLastError();
}

}  // namespace nrs
