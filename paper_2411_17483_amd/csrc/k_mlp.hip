// k_mlp.hip -- the learned-radius network: forward, backward and Adam
// kernels, feature standardisation and radius calibration.
//
// y = W3 g(W2 g(W1 xs + b1) + b2) + b3, g(z) = z Phi(z), xs = (x - mu) / sd.
// The products use the BF16-rounded weights (kept as FP32 values of the BF16
// grid, `wr`), all sums accumulate in FP32; Adam updates the FP32 master
// (`p`) and re-rounds.  Every reduction runs in a fixed order, so a step is
// deterministic.
#include <math.h>

#include <algorithm>
#include <vector>

#include "mlp.h"

namespace sofa {

static inline unsigned nblk(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}
__device__ __forceinline__ float round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011) for the initial weights
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; r++) {
    uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__global__ void k_mlp_init(float* __restrict__ p, MlpDims d, uint64_t seed) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.total()) return;
  float scale = 0.0f;
  if (i < d.oW1 + (int64_t)d.H1 * d.D) scale = sqrtf(2.0f / d.D);
  else if (i >= d.oW2 && i < d.oW2 + (int64_t)d.H2 * d.H1) scale = sqrtf(2.0f / d.H1);
  else if (i >= d.oW3 && i < d.oW3 + d.H2) scale = sqrtf(1.0f / d.H2);
  float v = 0.0f;
  if (scale > 0.0f) {
    uint4 r = philox(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0x4D4C5031u, 0u), (uint32_t)seed,
                     (uint32_t)(seed >> 32));
    double u1 = 1.0 - ((double)(r.x >> 5) * 67108864.0 + (double)(r.y >> 6)) * (1.0 / 9007199254740992.0);
    double u2 = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * (1.0 / 9007199254740992.0);
    v = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2)) * scale;
  }
  p[i] = v;
}

// rounded copy: BF16 grid for weights, unchanged biases
__global__ void k_mlp_round(const float* __restrict__ p, float* __restrict__ wr, MlpDims d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.total()) return;
  wr[i] = d.is_weight(i) ? round_bf16(p[i]) : p[i];
}

// ----------------------------------------------------------------------------
// C[m][n] = sum_k A(m,k) B(k,n) with A(m,k) = A[m*sam + k*sak] and
// B(k,n) = B[k*sbk + n*sbn]; k runs in increasing order.  Epilogues:
//  0: C = acc (+ bias[n])
//  1: C = acc + bias[n] (pre-activation), H = g(C)
//  2: C = acc * g'(Zin[m][n])
constexpr int kTm = 64, kTn = 64, kTk = 16;
constexpr int kSplitK = 8;  // batch slices of the weight-gradient products

// With gridDim.z = S > 1 (epilogue 0 only), slice z sums k in
// [z*ceil(K/S), (z+1)*ceil(K/S)) and writes C + z*M*ldc.

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              int64_t sam, int64_t sak, const float* __restrict__ Bm,
                                              int64_t sbk, int64_t sbn, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, float* __restrict__ H,
                                              const float* __restrict__ Zin) {
  __shared__ float As[kTk][kTm + 1];
  __shared__ float Bs[kTk][kTn + 1];
  const int t = threadIdx.x, tm = t / 16, tn = t % 16;
  const int m0 = blockIdx.y * kTm, n0 = blockIdx.x * kTn;
  const int per = (K + (int)gridDim.z - 1) / (int)gridDim.z;
  const int kb = (int)blockIdx.z * per, ke = kb + per < K ? kb + per : K;
  C += (int64_t)blockIdx.z * M * ldc;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += kTk) {
    for (int e = t; e < kTk * kTm; e += 256) {
      int kk = e / kTm, mm = e % kTm;
      int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < ke) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.0f;
    }
    for (int e = t; e < kTk * kTn; e += 256) {
      int kk = e / kTn, nn = e % kTn;
      int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < N && k < ke) ? Bm[(int64_t)k * sbk + (int64_t)n * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTk; kk++) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk][tm * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk][tn * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int m = m0 + tm * 4 + i, n = n0 + tn * 4 + j;
      if (m >= M || n >= N) continue;
      float z = acc[i][j];
      if (EPI == 0) {
        if (bias) z += bias[n];
        C[(int64_t)m * ldc + n] = z;
      } else if (EPI == 1) {
        z += bias[n];
        C[(int64_t)m * ldc + n] = z;
        H[(int64_t)m * ldc + n] = gelu(z);
      } else {
        C[(int64_t)m * ldc + n] = z * gelu_grad(Zin[(int64_t)m * ldc + n]);
      }
    }
}

template <int EPI>
static void gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
                 int64_t sbk, int64_t sbn, float* C, int ldc, const float* bias, float* H,
                 const float* Zin, hipStream_t st) {
  dim3 g((unsigned)((N + kTn - 1) / kTn), (unsigned)((M + kTm - 1) / kTm));
  k_gemm<EPI><<<g, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, H, Zin);
}

// forward layer Z = A W^T + bias, H = g(Z) with A: M x K (row stride lda)
// and W: N x K (row n contiguous): 32 x 32 output tiles and K steps of 64,
// so that a batch of a thousand rows fills the chip in a few steps.  Every
// output is the same FMA chain as k_gemm's (k increasing from a zero
// accumulator, then + bias), so both give identical values.
constexpr int kFt = 32, kFk = 64;

__global__ __launch_bounds__(256) void k_fwd(int M, int N, int K, const float* __restrict__ A, int64_t lda,
                                             const float* __restrict__ W, const float* __restrict__ bias,
                                             float* __restrict__ Z, float* __restrict__ H) {
  __shared__ float As[kFk][kFt + 1];
  __shared__ float Ws[kFk][kFt + 1];
  const int t = threadIdx.x, tm = t / 16, tn = t % 16;  // rows 2tm, 2tm+1; columns 2tn, 2tn+1
  const int m0 = blockIdx.y * kFt, n0 = blockIdx.x * kFt;
  float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
  for (int k0 = 0; k0 < K; k0 += kFk) {
    // 64 x 32 values of each operand, 8 per thread, consecutive threads on consecutive k
    float av[8], wv[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int idx = t + 256 * e, kk = idx % kFk, r = idx / kFk;
      const int k = k0 + kk, m = m0 + r, n = n0 + r;
      av[e] = (m < M && k < K) ? A[(int64_t)m * lda + k] : 0.0f;
      wv[e] = (n < N && k < K) ? W[(int64_t)n * K + k] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int idx = t + 256 * e, kk = idx % kFk, r = idx / kFk;
      As[kk][r] = av[e];
      Ws[kk][r] = wv[e];
    }
    __syncthreads();
    const int kn = K - k0 < kFk ? K - k0 : kFk;
    for (int kk = 0; kk < kn; kk++) {
      const float a0 = As[kk][2 * tm], a1 = As[kk][2 * tm + 1];
      const float w0 = Ws[kk][2 * tn], w1 = Ws[kk][2 * tn + 1];
      acc[0][0] = fmaf(a0, w0, acc[0][0]);
      acc[0][1] = fmaf(a0, w1, acc[0][1]);
      acc[1][0] = fmaf(a1, w0, acc[1][0]);
      acc[1][1] = fmaf(a1, w1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const int m = m0 + 2 * tm + i, n = n0 + 2 * tn + j;
      if (m >= M || n >= N) continue;
      const float z = acc[i][j] + bias[n];
      Z[(int64_t)m * N + n] = z;
      H[(int64_t)m * N + n] = gelu(z);
    }
}

// split-K: partial products over K slices into P[s][M][N], then a fixed-order sum
__global__ void k_sum_slices(const float* __restrict__ P, int S, int64_t MN, float* __restrict__ C) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float s = 0.0f;
  for (int j = 0; j < S; j++) s += P[(int64_t)j * MN + i];
  C[i] = s;
}

// C[M][N] = sum over the batch (K) of A(m,k) B(k,n): S slices in one launch
// into part[S][M][N], then their sum in slice order
static void gemm_splitk(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
                        int64_t sbk, int64_t sbn, float* C, float* part, int S, hipStream_t st) {
  dim3 g((unsigned)((N + kTn - 1) / kTn), (unsigned)((M + kTm - 1) / kTm), (unsigned)S);
  k_gemm<0><<<g, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, part, N, nullptr, nullptr, nullptr);
  k_sum_slices<<<nblk((int64_t)M * N, 256), 256, 0, st>>>(part, S, (int64_t)M * N, C);
}

// xs[b][d] = (x[b*ld + d] - mu[d]) / sd[d]
__global__ void k_standardize(const float* __restrict__ x, int64_t ld, int64_t B, int D,
                              const float* __restrict__ mu, const float* __restrict__ sd,
                              float* __restrict__ xs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * D) return;
  int64_t b = i / D;
  int d = (int)(i % D);
  xs[i] = (x[b * ld + d] - mu[d]) / sd[d];
}

// y[b] = sum_i w3[i] h2[b][i] + b3 (one wave per row, fixed tree order)
__global__ __launch_bounds__(256) void k_out(const float* __restrict__ h2, int64_t B, int H2,
                                             const float* __restrict__ w3, const float* __restrict__ b3,
                                             float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  float s = 0.0f;
  for (int i = lane; i < H2; i += 64) s = fmaf(w3[i], h2[b * H2 + i], s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) y[b] = s + b3[0];
}

// loss = mean (y - t)^2 and dy = 2 (y - t) / B (one block, fixed order)
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              int64_t B, float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    float r = y[b] - t[b];
    dy[b] = 2.0f * r / (float)B;
    s = fmaf(r, r, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = red[0] / (float)B;
}

// column sums over the batch: out[i] = sum_b scale_b * X[b][i]  (scale nullable)
// column sums over the batch, sum_b scale[b] X[b][i] (scale may be null):
// part[s][i] over the rows b = 4s + r (mod 4 kColSlices), r = wave, the four
// waves added in order, then the kColSlices partials added in slice order
constexpr int kColSlices = 16;

__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ X, int64_t B, int W,
                                                    const float* __restrict__ scale,
                                                    float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = threadIdx.x >> 6;
  float acc = 0.0f;
  if (c < W)
    for (int64_t b = (int64_t)blockIdx.y * 4 + r; b < B; b += 4 * kColSlices)
      acc = fmaf(scale ? scale[b] : 1.0f, X[b * W + c], acc);
  red[r][threadIdx.x & 63] = acc;
  __syncthreads();
  if (r == 0 && c < W) {
    const int j = threadIdx.x & 63;
    part[(int64_t)blockIdx.y * W + c] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
  }
}

__global__ void k_colsum_fin(const float* __restrict__ part, int W, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W) return;
  float s = 0.0f;
  for (int j = 0; j < kColSlices; j++) s += part[(int64_t)j * W + i];
  out[i] = s;
}

// part holds at least kColSlices * W floats
static void colsum(const float* X, int64_t B, int W, const float* scale, float* part, float* out,
                   hipStream_t st) {
  dim3 g(nblk(W, 64), kColSlices);
  k_colsum_part<<<g, 256, 0, st>>>(X, B, W, scale, part);
  k_colsum_fin<<<nblk(W, 256), 256, 0, st>>>(part, W, out);
}

// dz2[b][i] = dy[b] * w3[i] * g'(z2[b][i])
__global__ void k_dz2(const float* __restrict__ dy, const float* __restrict__ w3,
                      const float* __restrict__ z2, int64_t B, int H2, float* __restrict__ dz2) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * H2) return;
  int64_t b = e / H2;
  int i = (int)(e % H2);
  dz2[e] = dy[b] * w3[i] * gelu_grad(z2[e]);
}

// Adam on the master, then the rounded copy
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float* __restrict__ wr, MlpDims d, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.total()) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  wr[i] = d.is_weight(i) ? round_bf16(pi) : pi;
}

// feature mean and population standard deviation, one block per feature (FP64)
__global__ __launch_bounds__(256) void k_feat_stats(const float* __restrict__ x, int64_t n, int D,
                                                    float* __restrict__ mu, float* __restrict__ sd) {
  __shared__ double red[256];
  const int d = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i * D + d];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double m = red[0] / (double)n;
  __syncthreads();
  s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double e = x[i * D + d] - m;
    s += e * e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double v = sqrt(red[0] / (double)n);
    mu[d] = (float)m;
    sd[d] = v > 0.0 ? (float)v : 1.0f;
  }
}

__global__ void k_residual(const float* __restrict__ t, const float* __restrict__ y, int64_t n,
                           int64_t npad, float* __restrict__ r) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  r[i] = i < n ? t[i] - y[i] : INFINITY;
}

__global__ void k_bitonic_f32(float* __restrict__ a, int64_t npad, int64_t j, int64_t k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  int64_t ixj = i ^ j;
  if (ixj <= i) return;
  float x = a[i], y = a[ixj];
  bool up = (i & k) == 0;
  if ((x > y) == up) {
    a[i] = y;
    a[ixj] = x;
  }
}

// radius = exp(y + margin); U0 = radius^2 rounded up
__global__ void k_radius(const float* __restrict__ y, int64_t B, float margin, float* __restrict__ r,
                         float* __restrict__ u0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  double R = exp((double)y[i] + (double)margin);
  if (r) r[i] = (float)R;
  if (u0) u0[i] = __double2float_ru(R * R * (1.0 + 1e-12));
}

// The forward pass and radius of a batch in one launch, for inference (the
// radii of a search, sofa_radius_predict): the operations of k_standardize,
// k_fwd (each output's FMA chain over k from a zero accumulator, then the
// bias and the GELU), k_out (its per-lane sums and shuffle tree) and
// k_radius, in the same order, so the radii equal those of the separate
// kernels bit for bit.  Workgroup: kInferQ queries, activations in LDS;
// thread j computes neuron j (and j + 256, ...) of each layer for them.
constexpr int kInferQ = 4;

__host__ __device__ inline size_t infer_lds_bytes(const MlpDims& d) {
  return (size_t)kInferQ * (d.D + d.H1 + d.H2) * 4;
}

__global__ __launch_bounds__(256) void k_infer(const float* __restrict__ feat, int64_t ld, int64_t B, MlpDims d,
                                               const float* __restrict__ wr, const float* __restrict__ mu,
                                               const float* __restrict__ sd, float margin,
                                               float* __restrict__ r, float* __restrict__ u0) {
  extern __shared__ float act[];
  float* xs = act;                   // kInferQ x D
  float* h1 = xs + kInferQ * d.D;    // kInferQ x H1
  float* h2 = h1 + kInferQ * d.H1;   // kInferQ x H2
  const int64_t q0 = (int64_t)blockIdx.x * kInferQ;
  const int nq = (int)(B - q0 < kInferQ ? B - q0 : kInferQ);
  const int t = threadIdx.x;
  for (int i = t; i < nq * d.D; i += 256) {
    const int q = i / d.D, k = i % d.D;
    xs[i] = (feat[(q0 + q) * ld + k] - mu[k]) / sd[k];
  }
  __syncthreads();
  const float* W1 = wr + d.oW1;
  for (int j = t; j < d.H1; j += 256) {
    float acc[kInferQ];
#pragma unroll
    for (int q = 0; q < kInferQ; q++) acc[q] = 0.0f;
    for (int k = 0; k < d.D; k++) {
      const float w = W1[(int64_t)j * d.D + k];
#pragma unroll
      for (int q = 0; q < kInferQ; q++) acc[q] = fmaf(xs[q * d.D + k], w, acc[q]);
    }
    const float bj = wr[d.ob1 + j];
#pragma unroll
    for (int q = 0; q < kInferQ; q++)
      if (q < nq) h1[q * d.H1 + j] = gelu(acc[q] + bj);
  }
  __syncthreads();
  const float* W2 = wr + d.oW2;
  for (int j = t; j < d.H2; j += 256) {
    float acc[kInferQ];
#pragma unroll
    for (int q = 0; q < kInferQ; q++) acc[q] = 0.0f;
    for (int k = 0; k < d.H1; k++) {
      const float w = W2[(int64_t)j * d.H1 + k];
#pragma unroll
      for (int q = 0; q < kInferQ; q++) acc[q] = fmaf(h1[q * d.H1 + k], w, acc[q]);
    }
    const float bj = wr[d.ob2 + j];
#pragma unroll
    for (int q = 0; q < kInferQ; q++)
      if (q < nq) h2[q * d.H2 + j] = gelu(acc[q] + bj);
  }
  __syncthreads();
  const int lane = t & 63, q = t >> 6;  // one wave per query (kInferQ = 4 waves)
  if (q < nq) {
    const float* w3 = wr + d.oW3;
    float s = 0.0f;
    for (int i = lane; i < d.H2; i += 64) s = fmaf(w3[i], h2[q * d.H2 + i], s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
      const float y = s + wr[d.ob3];
      const double R = exp((double)y + (double)margin);
      if (r) r[q0 + q] = (float)R;
      if (u0) u0[q0 + q] = __double2float_ru(R * R * (1.0 + 1e-12));
    }
  }
}
static_assert(kInferQ * 64 <= 256, "one wave per query of a workgroup");

// the fused launch holds a workgroup's activations in at most 64 KB of LDS
// (the default dimensions take 8.5 KB)
bool infer_fits(const MlpDims& d) { return infer_lds_bytes(d) <= 65536; }
size_t model_radius_scratch_floats(const MlpDims& d, int64_t B) {
  return infer_fits(d) ? 0 : mlp_act_floats(d, B);
}

sofa_status launch_infer(const sofa_radius* m, const float* feat, int64_t ld, int64_t B, float* r, float* u0,
                         hipStream_t st) {
  if (B <= 0) return SOFA_OK;
  const MlpDims& d = m->dims;
  k_infer<<<nblk(B, kInferQ), 256, infer_lds_bytes(d), st>>>(feat, ld, B, d, m->wr.as<float>(), m->mu.as<float>(),
                                                             m->sd.as<float>(), m->margin, r, u0);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// ----------------------------------------------------------------------------
// host side
static sofa_status ensure_act(sofa_radius* m, int64_t B) {
  const MlpDims& d = m->dims;
  if (!m->part.p) {
    const int64_t mn = std::max<int64_t>((int64_t)d.H2 * d.H1, (int64_t)d.H1 * d.D);
    // split-K partials, and the column-sum partials (kColSlices per column)
    const int64_t need = std::max<int64_t>((int64_t)kSplitK * mn,
                                           (int64_t)kColSlices * std::max(d.H1, d.H2));
    SOFA_TRY(m->part.alloc((size_t)need * 4));
  }
  if (B <= m->act_rows) return SOFA_OK;
  const size_t per = (size_t)d.D + 2 * d.H1 + 3 * d.H2 + 4;
  SOFA_TRY(m->act.alloc(per * (size_t)B * 4));
  m->act_rows = B;
  return SOFA_OK;
}

MlpAct act_views(float* base, const MlpDims& d, int64_t B) {
  MlpAct a;
  a.xs = base;
  a.z1 = a.xs + (size_t)B * d.D;
  a.h1 = a.z1 + (size_t)B * d.H1;
  a.z2 = a.h1 + (size_t)B * d.H1;
  a.h2 = a.z2 + (size_t)B * d.H2;
  a.dz2 = a.h2 + (size_t)B * d.H2;
  a.y = a.dz2 + (size_t)B * d.H2;
  a.dy = a.y + B;
  return a;
}

size_t mlp_act_floats(const MlpDims& d, int64_t B) {
  return ((size_t)d.D + 2 * d.H1 + 3 * d.H2 + 4) * (size_t)B;
}

void mlp_forward(const sofa_radius* m, const float* feat, int64_t ld, int64_t B, const MlpAct& a,
                 hipStream_t st) {
  const MlpDims& d = m->dims;
  const float* wr = m->wr.as<float>();
  k_standardize<<<nblk(B * d.D, 256), 256, 0, st>>>(feat, ld, B, d.D, m->mu.as<float>(),
                                                    m->sd.as<float>(), a.xs);
  const dim3 g1((unsigned)((d.H1 + kFt - 1) / kFt), (unsigned)((B + kFt - 1) / kFt));
  k_fwd<<<g1, 256, 0, st>>>((int)B, d.H1, d.D, a.xs, d.D, wr + d.oW1, wr + d.ob1, a.z1, a.h1);
  const dim3 g2((unsigned)((d.H2 + kFt - 1) / kFt), (unsigned)((B + kFt - 1) / kFt));
  k_fwd<<<g2, 256, 0, st>>>((int)B, d.H2, d.H1, a.h1, d.H1, wr + d.oW2, wr + d.ob2, a.z2, a.h2);
  k_out<<<nblk(B, 4), 256, 0, st>>>(a.h2, B, d.H2, wr + d.oW3, wr + d.ob3, a.y);
}

static void mlp_backward(const sofa_radius* m, const float* target, int64_t B, const MlpAct& a,
                         float* grad, float* loss, float* part, hipStream_t st) {
  const MlpDims& d = m->dims;
  const float* wr = m->wr.as<float>();
  k_loss<<<1, 256, 0, st>>>(a.y, target, B, a.dy, loss);
  // output layer
  colsum(a.h2, B, d.H2, a.dy, part, grad + d.oW3, st);
  colsum(a.dy, B, 1, nullptr, part, grad + d.ob3, st);
  // second layer: dz2, dW2 = dz2^T h1, db2
  k_dz2<<<nblk(B * d.H2, 256), 256, 0, st>>>(a.dy, wr + d.oW3, a.z2, B, d.H2, a.dz2);
  gemm_splitk(d.H2, d.H1, (int)B, a.dz2, 1, d.H2, a.h1, d.H1, 1, grad + d.oW2, part, kSplitK, st);
  colsum(a.dz2, B, d.H2, nullptr, part, grad + d.ob2, st);
  // first layer: dz1 = (dz2 W2) * g'(z1) (written over h1), dW1 = dz1^T xs, db1
  gemm<2>((int)B, d.H1, d.H2, a.dz2, d.H2, 1, wr + d.oW2, d.H1, 1, a.h1, d.H1, nullptr, nullptr, a.z1, st);
  gemm_splitk(d.H1, d.D, (int)B, a.h1, 1, d.H1, a.xs, d.D, 1, grad + d.oW1, part, kSplitK, st);
  colsum(a.h1, B, d.H1, nullptr, part, grad + d.ob1, st);
}

}  // namespace sofa

using namespace sofa;

extern "C" sofa_status sofa_radius_create(const sofa_radius_params* p, sofa_radius** out) {
  if (!p || !out) return set_error(SOFA_EINVAL, "null argument");
  *out = nullptr;
  MlpDims d;
  d.D = p->in_dim ? p->in_dim : 32;
  d.H1 = p->hidden1 ? p->hidden1 : 256;
  d.H2 = p->hidden2 ? p->hidden2 : 256;
  if (d.D < 1 || d.D > 64 || d.H1 < 1 || d.H1 > 4096 || d.H2 < 1 || d.H2 > 4096)
    return set_error(SOFA_EINVAL, "network dimensions out of range");
  if (p->k < 1 || p->k > kMaxK) return set_error(SOFA_EINVAL, "k=%d out of range", p->k);
  d.layout();
  sofa_radius* m = new sofa_radius();
  m->dims = d;
  m->k = p->k;
  m->lr = p->lr > 0 ? p->lr : 1e-3f;
  m->beta1 = p->beta1 > 0 ? p->beta1 : 0.9f;
  m->beta2 = p->beta2 > 0 ? p->beta2 : 0.999f;
  m->eps = p->eps > 0 ? p->eps : 1e-8f;
  const int64_t P = d.total();
  sofa_status s = m->p.alloc(P * 4);
  if (s == SOFA_OK) s = m->wr.alloc(P * 4);
  if (s == SOFA_OK) s = m->g.alloc(P * 4);
  if (s == SOFA_OK) s = m->m1.alloc(P * 4);
  if (s == SOFA_OK) s = m->m2.alloc(P * 4);
  if (s == SOFA_OK) s = m->mu.alloc(d.D * 4);
  if (s == SOFA_OK) s = m->sd.alloc(d.D * 4);
  if (s == SOFA_OK) s = m->loss.alloc(64);
  if (s != SOFA_OK) {
    delete m;
    return s;
  }
  k_mlp_init<<<nblk(P, 256), 256>>>(m->p.as<float>(), d, p->seed);
  k_mlp_round<<<nblk(P, 256), 256>>>(m->p.as<float>(), m->wr.as<float>(), d);
  std::vector<float> zeros(d.D, 0.0f), ones(d.D, 1.0f);
  if (hipMemset(m->m1.p, 0, P * 4) != hipSuccess || hipMemset(m->m2.p, 0, P * 4) != hipSuccess ||
      hipMemcpy(m->mu.p, zeros.data(), d.D * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->sd.p, ones.data(), d.D * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    delete m;
    return set_error(SOFA_EDEVICE, "initialising the network failed: %s", hipGetErrorString(hipGetLastError()));
  }
  *out = m;
  return SOFA_OK;
}

extern "C" void sofa_radius_free(sofa_radius* m) { delete m; }

extern "C" int64_t sofa_radius_num_params(const sofa_radius* m) { return m ? m->dims.total() : 0; }

extern "C" sofa_status sofa_radius_get(const sofa_radius* m, float* params, float* mu, float* sd,
                                       float* margin, int64_t* step) {
  if (!m) return set_error(SOFA_EINVAL, "null model");
  if (params) SOFA_HIP(hipMemcpy(params, m->p.p, m->dims.total() * 4, hipMemcpyDeviceToHost));
  if (mu) SOFA_HIP(hipMemcpy(mu, m->mu.p, m->dims.D * 4, hipMemcpyDeviceToHost));
  if (sd) SOFA_HIP(hipMemcpy(sd, m->sd.p, m->dims.D * 4, hipMemcpyDeviceToHost));
  if (margin) *margin = m->margin;
  if (step) *step = m->step;
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_set(sofa_radius* m, const float* params, const float* mu,
                                       const float* sd, const float* margin, const int64_t* step) {
  if (!m) return set_error(SOFA_EINVAL, "null model");
  const int64_t P = m->dims.total();
  if (params) {
    SOFA_HIP(hipMemcpy(m->p.p, params, P * 4, hipMemcpyHostToDevice));
    k_mlp_round<<<nblk(P, 256), 256>>>(m->p.as<float>(), m->wr.as<float>(), m->dims);
    SOFA_HIP(hipMemset(m->m1.p, 0, P * 4));
    SOFA_HIP(hipMemset(m->m2.p, 0, P * 4));
    m->step = 0;
  }
  if (mu) SOFA_HIP(hipMemcpy(m->mu.p, mu, m->dims.D * 4, hipMemcpyHostToDevice));
  if (sd) {
    for (int d = 0; d < m->dims.D; d++)
      if (!(sd[d] > 0.0f)) return set_error(SOFA_EINVAL, "sd[%d] must be positive", d);
    SOFA_HIP(hipMemcpy(m->sd.p, sd, m->dims.D * 4, hipMemcpyHostToDevice));
  }
  if (margin) m->margin = *margin;
  if (step) m->step = *step;
  SOFA_HIP(hipDeviceSynchronize());
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_standardize(sofa_radius* m, const float* d_feat, int64_t n,
                                               void* stream) {
  if (!m || !d_feat || n < 1) return set_error(SOFA_EINVAL, "bad arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  k_feat_stats<<<m->dims.D, 256, 0, st>>>(d_feat, n, m->dims.D, m->mu.as<float>(), m->sd.as<float>());
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

static sofa_status grads_impl(sofa_radius* m, const float* feat, const float* target, int64_t B,
                              float* grad, float* loss, hipStream_t st) {
  if (!m || !feat || !target || B < 1 || B > 65536) return set_error(SOFA_EINVAL, "bad arguments");
  SOFA_TRY(ensure_act(m, B));
  MlpAct a = act_views(m->act.as<float>(), m->dims, B);
  mlp_forward(m, feat, m->dims.D, B, a, st);
  mlp_backward(m, target, B, a, grad, loss, m->part.as<float>(), st);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_gradients(sofa_radius* m, const float* d_feat, const float* d_target,
                                             int64_t B, float* d_grad, float* d_loss, void* stream) {
  if (!d_grad) return set_error(SOFA_EINVAL, "null gradient array");
  return grads_impl(m, d_feat, d_target, B, d_grad, d_loss, reinterpret_cast<hipStream_t>(stream));
}

extern "C" sofa_status sofa_radius_train_step(sofa_radius* m, const float* d_feat,
                                              const float* d_target, int64_t B, float* d_loss,
                                              void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SOFA_TRY(grads_impl(m, d_feat, d_target, B, m->g.as<float>(), d_loss, st));
  m->step++;
  const float c1 = (float)(1.0 - pow((double)m->beta1, (double)m->step));
  const float c2 = (float)(1.0 - pow((double)m->beta2, (double)m->step));
  k_adam<<<nblk(m->dims.total(), 256), 256, 0, st>>>(m->p.as<float>(), m->g.as<float>(), m->m1.as<float>(),
                                                     m->m2.as<float>(), m->wr.as<float>(), m->dims, m->lr,
                                                     m->beta1, m->beta2, m->eps, c1, c2);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_fit(sofa_radius* m, const float* d_feat, const float* d_target,
                                       int64_t n, int32_t epochs, int32_t batch, float* h_epoch_loss,
                                       void* stream) {
  if (!m || !d_feat || !d_target || n < 1 || epochs < 1 || batch < 1 || batch > 65536)
    return set_error(SOFA_EINVAL, "bad arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t steps = (n + batch - 1) / batch;
  DevBuf losses;
  SOFA_TRY(losses.alloc((size_t)steps * 4));
  std::vector<float> h(steps);
  for (int e = 0; e < epochs; e++) {
    for (int64_t s = 0; s < steps; s++) {
      const int64_t b0 = s * batch, bn = std::min<int64_t>(batch, n - b0);
      SOFA_TRY(sofa_radius_train_step(m, d_feat + b0 * m->dims.D, d_target + b0, bn,
                                      losses.as<float>() + s, stream));
    }
    if (h_epoch_loss) {
      SOFA_HIP(hipMemcpyAsync(h.data(), losses.p, (size_t)steps * 4, hipMemcpyDeviceToHost, st));
      SOFA_HIP(hipStreamSynchronize(st));
      double acc = 0;
      for (float v : h) acc += v;
      h_epoch_loss[e] = (float)(acc / (double)steps);
    }
  }
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_forward(const sofa_radius* m, const float* d_feat, int64_t B,
                                           float* d_y, void* stream) {
  if (!m || !d_feat || !d_y || B < 0) return set_error(SOFA_EINVAL, "bad arguments");
  if (B == 0) return SOFA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DevBuf act;
  SOFA_TRY(act.alloc(mlp_act_floats(m->dims, B) * 4));
  MlpAct a = act_views(act.as<float>(), m->dims, B);
  mlp_forward(m, d_feat, m->dims.D, B, a, st);
  SOFA_HIP(hipMemcpyAsync(d_y, a.y, (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_calibrate(sofa_radius* m, const float* d_feat, const float* d_target,
                                             int64_t n, double quantile, void* stream) {
  if (!m || !d_feat || !d_target || n < 1 || !(quantile >= 0.0 && quantile <= 1.0))
    return set_error(SOFA_EINVAL, "bad arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int64_t npad = 1;
  while (npad < n) npad <<= 1;
  DevBuf act, r;
  SOFA_TRY(act.alloc(mlp_act_floats(m->dims, n) * 4));
  SOFA_TRY(r.alloc((size_t)npad * 4));
  MlpAct a = act_views(act.as<float>(), m->dims, n);
  mlp_forward(m, d_feat, m->dims.D, n, a, st);
  k_residual<<<nblk(npad, 256), 256, 0, st>>>(d_target, a.y, n, npad, r.as<float>());
  for (int64_t k = 2; k <= npad; k <<= 1)
    for (int64_t j = k >> 1; j > 0; j >>= 1)
      k_bitonic_f32<<<nblk(npad, 256), 256, 0, st>>>(r.as<float>(), npad, j, k);
  const int64_t idx = std::min<int64_t>(n - 1, (int64_t)floor(quantile * (double)(n - 1) + 0.5));
  float v = 0;
  SOFA_HIP(hipMemcpyAsync(&v, r.as<float>() + idx, 4, hipMemcpyDeviceToHost, st));
  SOFA_HIP(hipStreamSynchronize(st));
  m->margin = v;
  return SOFA_OK;
}

extern "C" sofa_status sofa_radius_predict(const sofa_radius* m, const float* d_feat, int64_t B,
                                           float* d_radius, void* stream) {
  if (!m || !d_feat || !d_radius || B < 0) return set_error(SOFA_EINVAL, "bad arguments");
  if (B == 0) return SOFA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (infer_fits(m->dims)) {
    SOFA_TRY(launch_infer(m, d_feat, m->dims.D, B, d_radius, nullptr, st));
    SOFA_HIP(hipStreamSynchronize(st));
    return SOFA_OK;
  }
  DevBuf act;
  SOFA_TRY(act.alloc(mlp_act_floats(m->dims, B) * 4));
  MlpAct a = act_views(act.as<float>(), m->dims, B);
  mlp_forward(m, d_feat, m->dims.D, B, a, st);
  k_radius<<<nblk(B, 256), 256, 0, st>>>(a.y, B, m->margin, d_radius, nullptr);
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

namespace sofa {
// radii of a query batch inside sofa_knn: forward on the pool values, U0
sofa_status launch_model_radius(const sofa_radius* m, const float* pool, int64_t ld, int64_t B,
                                float* scratch, float* U0, hipStream_t st) {
  if (infer_fits(m->dims)) return launch_infer(m, pool, ld, B, nullptr, U0, st);
  MlpAct a = act_views(scratch, m->dims, B);
  mlp_forward(m, pool, ld, B, a, st);
  k_radius<<<nblk(B, 256), 256, 0, st>>>(a.y, B, m->margin, nullptr, U0);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}
}  // namespace sofa
