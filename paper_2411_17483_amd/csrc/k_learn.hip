// k_learn.hip -- learned SFA quantisation on the GPU (Algorithm 1, MCB), FP64.
//
// Steps, in the order of Algorithm 1: stride sample of m rows, orthonormal DFT
// of the pool values of each sampled row, population variance of every pool
// value, the l values of largest variance (ties: lower pool index), then per
// kept value a sort of its sample and the alpha-1 breakpoints (equi-depth
// order statistics or equi-width steps, Section IV-E).
#include "kernels.h"

#include <cmath>

namespace sofa {

static constexpr double kPi = 3.14159265358979323846;

// Basis value of pool entry p at time t.
// SFA (summary 0): orthonormal DFT, p = 2(k-1) is Re X_k (cos), p = 2(k-1)+1
// is Im X_k (-sin); the angle uses (k*t mod n).
// iSAX (summary 1, Section IV-D): entry p < l is the mean of segment p of l
// equal segments, scaled to an orthonormal row: (n/l)^-1/2 on the segment,
// so that the coefficient is sqrt(n/l) times the PAA mean; entries p >= l
// are zero.
__device__ __forceinline__ double basis64(int p, int t, int n, int summary, int l) {
  if (summary == 1) {
    const int seg = n / l;
    return (p < l && t / seg == p) ? 1.0 / sqrt((double)seg) : 0.0;
  }
  int k = p / 2 + 1;
  long long kt = ((long long)k * t) % n;
  double ang = 2.0 * kPi * (double)kt / (double)n;
  double s = 1.0 / sqrt((double)n);
  return (p & 1) ? -sin(ang) * s : cos(ang) * s;
}

__global__ void k_basis64(double* __restrict__ b64, int n, int np, int summary, int l) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)np * n) return;
  int p = (int)(i / n), t = (int)(i % n);
  b64[i] = basis64(p, t, n, summary, l);
}

// Transposed FP32 basis for the MFMA projection: bt[r][t] for r < nrows,
// t < n_pad.  Row r holds pool entry cols[r] (or r when cols is null); rows
// >= nvalid and columns >= n are zero.
__global__ void k_basis32_t(float* __restrict__ bt, int nrows, int nvalid, int n, int n_pad,
                            const int* __restrict__ cols, int summary, int l) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nrows * n_pad) return;
  int r = (int)(i / n_pad), t = (int)(i % n_pad);
  float v = 0.0f;
  if (r < nvalid && t < n) v = (float)basis64(cols ? cols[r] : r, t, n, summary, l);
  bt[i] = v;
}

// DFT pool of the stride sample: F[i][p] = sum_t x[row_i][t] * b64[p][t],
// row_i = floor(i*N/m).  One wave per sampled row; lane p < np owns pool value p.
__global__ __launch_bounds__(256) void k_sample_dft(const float* __restrict__ X, int64_t N, int n,
                                                    int64_t m, const double* __restrict__ b64,
                                                    int np, double* __restrict__ F) {
#pragma clang fp contract(off)
  __shared__ float xs[4][kMaxN];
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the loop bound is uniform across the workgroup (the barriers inside)
  for (int64_t i0 = (int64_t)blockIdx.x * 4; i0 < m; i0 += (int64_t)gridDim.x * 4) {
    const int64_t i = i0 + wave;
    const bool ok = i < m;
    const int64_t row = ok ? (int64_t)((i * N) / m) : 0;
    for (int t = lane; t < n; t += 64) xs[wave][t] = ok ? X[row * n + t] : 0.0f;
    __syncthreads();
    if (ok && lane < np) {
      const double* b = b64 + (int64_t)lane * n;
      double s = 0.0;
      for (int t = 0; t < n; t++) s = s + (double)xs[wave][t] * b[t];
      F[i * np + lane] = s;
    }
    __syncthreads();
  }
}

// Mean and population variance of column p of F (m x np), one block per column.
__global__ __launch_bounds__(256) void k_col_stats(const double* __restrict__ F, int64_t m, int np,
                                                   double* __restrict__ var) {
  __shared__ double red[256];
  int p = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += F[i * np + p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double mu = red[0] / (double)m;
  __syncthreads();
  s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    double d = F[i * np + p] - mu;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) var[p] = red[0] / (double)m;
}

// Top-l pool values by variance, decreasing; equal variances keep the lower index.
__global__ void k_select(const double* __restrict__ var, int np, int l, int* __restrict__ sel) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long used = 0ull;
  for (int j = 0; j < 16; j++) {
    if (j >= l) {
      sel[j] = 0;
      continue;
    }
    int best = -1;
    for (int p = 0; p < np; p++) {
      if ((used >> p) & 1ull) continue;
      if (best < 0 || var[p] > var[best]) best = p;
    }
    sel[j] = best;
    used |= 1ull << best;
  }
}

// cols[j][i] = F[i][sel[j]] for i < m; +inf padding up to mpad (a power of two).
__global__ void k_gather_cols(const double* __restrict__ F, int64_t m, int np,
                              const int* __restrict__ sel, int l, double* __restrict__ cols,
                              int64_t mpad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)l * mpad) return;
  int j = (int)(i / mpad);
  int64_t r = i % mpad;
  cols[i] = (r < m) ? F[r * np + sel[j]] : INFINITY;
}

// One compare-exchange stage of a bitonic sort of each row of a (l x mpad).
__global__ void k_bitonic_stage(double* __restrict__ a, int64_t mpad, int l, int64_t j, int64_t k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)l * mpad) return;
  int64_t row = i / mpad, idx = i % mpad;
  int64_t ixj = idx ^ j;
  if (ixj <= idx) return;
  double* r = a + row * mpad;
  double x = r[idx], y = r[ixj];
  bool up = (idx & k) == 0;
  if ((x > y) == up) {
    r[idx] = y;
    r[ixj] = x;
  }
}

// Breakpoints from the sorted sample of each kept value.
__global__ void k_breakpoints(const double* __restrict__ cols, int64_t m, int64_t mpad, int l,
                              int alpha, int binning, double* __restrict__ beta) {
#pragma clang fp contract(off)
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l * (alpha - 1)) return;
  int j = i / (alpha - 1), a = i % (alpha - 1) + 1;
  const double* v = cols + (int64_t)j * mpad;
  if (binning == 0) {
    int64_t idx = (int64_t)(((int64_t)a * m) / alpha);
    beta[i] = v[idx];
  } else {
    beta[i] = v[0] + (double)a * (v[m - 1] - v[0]) / (double)alpha;
  }
}

// FP32 breakpoint table used by quantisation and the lower-bound tables:
// beta32[j][a] = beta_j(a+1) rounded to nearest, +inf where unused.
__global__ void k_beta32(const double* __restrict__ beta64, int l, int alpha,
                         float* __restrict__ beta32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kTable) return;
  int j = i / kAlphaMax, a = i % kAlphaMax;
  float v = INFINITY;
  if (j < l && a < alpha - 1) v = (float)beta64[j * (alpha - 1) + a];
  beta32[i] = v;
}

// ----------------------------------------------------------------------------
static inline unsigned nblk(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

// Phi^-1(p) of the standard normal: bisection on Phi(x) = erfc(-x / sqrt 2) / 2,
// which is monotone, down to adjacent doubles
static double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int i = 0; i < 2000; i++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// iSAX breakpoints (Section IV-D): the alpha - 1 equal-depth quantiles of
// N(0,1), the same for every segment, scaled by sqrt(n/l) to the orthonormal
// PAA coefficients
void isax_breakpoints(int n, int l, int alpha, double* beta) {
  const double s = std::sqrt((double)(n / l));
  for (int a = 1; a < alpha; a++) {
    const double b = normal_quantile((double)a / (double)alpha) * s;
    for (int j = 0; j < l; j++) beta[(size_t)j * (alpha - 1) + a - 1] = b;
  }
}

sofa_status launch_learn(const float* X, int64_t N, int n, int64_t m, int pool, int l, int alpha,
                         int binning, int summary, int selection, hipStream_t st, double* h_var,
                         int* h_sel, double* h_beta) {
  int np = 2 * pool;
  int64_t mpad = 1;
  while (mpad < m) mpad <<= 1;
  DevBuf b64, F, var, sel, cols, beta;
  SOFA_TRY(b64.alloc(sizeof(double) * np * n));
  SOFA_TRY(F.alloc(sizeof(double) * m * np));
  SOFA_TRY(var.alloc(sizeof(double) * np));
  SOFA_TRY(sel.alloc(sizeof(int) * 16));
  SOFA_TRY(cols.alloc(sizeof(double) * l * mpad));
  SOFA_TRY(beta.alloc(sizeof(double) * l * (alpha > 1 ? alpha - 1 : 1)));
  k_basis64<<<nblk((int64_t)np * n, 256), 256, 0, st>>>(b64.as<double>(), n, np, summary, l);
  k_sample_dft<<<grid_blocks(m, 4), 256, 0, st>>>(X, N, n, m, b64.as<double>(), np, F.as<double>());
  k_col_stats<<<np, 256, 0, st>>>(F.as<double>(), m, np, var.as<double>());
  if (summary == 1) {
    // iSAX keeps the l segments in time order and fixed breakpoints; the
    // sample only reports the variance of each PAA coefficient
    SOFA_HIP(hipGetLastError());
    SOFA_HIP(hipMemcpyAsync(h_var, var.p, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    SOFA_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < 16; j++) h_sel[j] = j < l ? j : 0;
    if (alpha > 1) isax_breakpoints(n, l, alpha, h_beta);
    return SOFA_OK;
  }
  if (selection == 1) {
    // the first l pool values, in pool order
    int first[16];
    for (int j = 0; j < 16; j++) first[j] = j < l ? j : 0;
    SOFA_HIP(hipMemcpyAsync(sel.p, first, sizeof(first), hipMemcpyHostToDevice, st));
  } else {
    k_select<<<1, 64, 0, st>>>(var.as<double>(), np, l, sel.as<int>());
  }
  if (alpha > 1) {
    k_gather_cols<<<nblk((int64_t)l * mpad, 256), 256, 0, st>>>(F.as<double>(), m, np, sel.as<int>(),
                                                                  l, cols.as<double>(), mpad);
    for (int64_t k = 2; k <= mpad; k <<= 1)
      for (int64_t j = k >> 1; j > 0; j >>= 1)
        k_bitonic_stage<<<nblk((int64_t)l * mpad, 256), 256, 0, st>>>(cols.as<double>(), mpad, l, j, k);
    k_breakpoints<<<nblk((int64_t)l * (alpha - 1), 256), 256, 0, st>>>(
        cols.as<double>(), m, mpad, l, alpha, binning, beta.as<double>());
  }
  SOFA_HIP(hipGetLastError());
  SOFA_HIP(hipMemcpyAsync(h_var, var.p, sizeof(double) * np, hipMemcpyDeviceToHost, st));
  SOFA_HIP(hipMemcpyAsync(h_sel, sel.p, sizeof(int) * 16, hipMemcpyDeviceToHost, st));
  if (alpha > 1)
    SOFA_HIP(hipMemcpyAsync(h_beta, beta.p, sizeof(double) * l * (alpha - 1), hipMemcpyDeviceToHost, st));
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

sofa_status launch_bins_tables(sofa_bins* b, hipStream_t st) {
  int n = b->n, n_pad = b->n_pad;
  SOFA_TRY(b->d_sel.alloc(sizeof(int) * 16));
  SOFA_HIP(hipMemcpyAsync(b->d_sel.p, b->sel, sizeof(int) * 16, hipMemcpyHostToDevice, st));
  SOFA_TRY(b->d_bt_sel.alloc(sizeof(float) * 16 * n_pad));
  SOFA_TRY(b->d_bt_pool.alloc(sizeof(float) * b->ncol_pool * n_pad));
  SOFA_TRY(b->d_beta32.alloc(sizeof(float) * kTable));
  k_basis32_t<<<nblk((int64_t)16 * n_pad, 256), 256, 0, st>>>(b->d_bt_sel.as<float>(), 16, b->l, n,
                                                                n_pad, b->d_sel.as<int>(), b->summary, b->l);
  k_basis32_t<<<nblk((int64_t)b->ncol_pool * n_pad, 256), 256, 0, st>>>(
      b->d_bt_pool.as<float>(), b->ncol_pool, 2 * b->pool, n, n_pad, nullptr, b->summary, b->l);
  DevBuf beta64;
  int nb = b->l * (b->alpha > 1 ? b->alpha - 1 : 1);
  SOFA_TRY(beta64.alloc(sizeof(double) * nb));
  if (b->alpha > 1)
    SOFA_HIP(hipMemcpyAsync(beta64.p, b->beta.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
  k_beta32<<<nblk(kTable, 256), 256, 0, st>>>(beta64.as<double>(), b->l, b->alpha, b->d_beta32.as<float>());
  SOFA_HIP(hipGetLastError());
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

}  // namespace sofa
