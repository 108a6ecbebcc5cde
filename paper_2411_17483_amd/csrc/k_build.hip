// k_build.hip -- SFA transform of a collection on the matrix cores and the
// leaf layout of the index.
//
// Projection (Algorithm 2, step 1): the kept Fourier values of a row are dot
// products with a partial orthonormal DFT basis (only the kept columns are
// needed, not a full FFT), so a batch of rows times the basis is a GEMM,
// [rows x n] . [n x 16], run with v_mfma_f32_16x16x4f32.  Rows are staged
// through LDS with coalesced 16-byte loads and read back in the MFMA operand
// layout.  Quantisation (Algorithm 2, step 2) is fused into the epilogue: a
// binary search over the FP32 breakpoints held in LDS.
//
// Layout: the MESSI tree of Sections IV-A and IV-B is replaced by a flat array sorted
// by a key that interleaves the leading bits of the symbols (most significant
// first, positions in word order), cut into fixed-size leaves; each leaf
// keeps a per-position [min, max] symbol envelope.
#include "kernels.h"

namespace sofa {

typedef float f4v __attribute__((ext_vector_type(4)));

static inline unsigned nblk(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

// ----------------------------------------------------------------------------
// z-normalisation (Section II): per row, the mean and the population standard
// deviation in FP64 (lane sums over t = lane, lane + 64, ..., then a
// butterfly across the wave), and (x - mean) / sd formed in FP64 and rounded
// to FP32 once; sd = 0 gives zeros.  One wave per row; rows are re-read from
// L2 for the second moment and the output.
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Output row r reads input row r, or with src_rows > m the stride-sample
// row floor(r * src_rows / m).  in and out may be the same array when
// src_rows == m (no __restrict__): each element is read and then written by
// the same lane.
__global__ __launch_bounds__(256) void k_znorm(const float* in, int64_t m, int n, float* out,
                                               int64_t src_rows) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < m; r += (int64_t)gridDim.x * 4) {
    const int64_t src = src_rows > m ? r * src_rows / m : r;
    const float* x = in + src * n;
    double s = 0.0;
    for (int t = lane; t < n; t += 64) s += (double)x[t];
    const double mu = wave_sum64(s) / (double)n;
    double q = 0.0;
    for (int t = lane; t < n; t += 64) {
      const double d = (double)x[t] - mu;
      q += d * d;
    }
    const double sd = sqrt(wave_sum64(q) / (double)n);
    float* o = out + r * n;
    for (int t = lane; t < n; t += 64) o[t] = sd > 0.0 ? (float)(((double)x[t] - mu) / sd) : 0.0f;
  }
}

sofa_status launch_znorm(const float* in, int64_t m, int n, float* out, hipStream_t st, int64_t src_rows) {
  if (m <= 0) return SOFA_OK;
  k_znorm<<<grid_blocks(m, 4), 256, 0, st>>>(in, m, n, out, src_rows);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// ----------------------------------------------------------------------------
// projection.  A wave takes 16 rows at a time and loads them straight into
// the MFMA operand layout, no LDS staging: for 16-column block m, lane
// (li, g) = (lane % 16, lane / 16) holds columns 16m + 4g .. 16m + 4g + 3 of
// row li (the four lanes of a row read 64 contiguous bytes), and the four
// v_mfma_f32_16x16x4f32 steps of the block take one component each, with
// the basis rows read in the same column order.  Each wave works on its own
// rows, so no workgroup barrier orders the waves.
template <int NG, bool QUANT>
__global__ __launch_bounds__(256) void k_project(const float* __restrict__ X, int64_t m, int n,
                                                 int64_t ldx, const float* __restrict__ BT,
                                                 int n_pad, float* __restrict__ out, int ld_out,
                                                 const float* __restrict__ beta32, int l,
                                                 uint8_t* __restrict__ words,
                                                 double* __restrict__ norm2,
                                                 unsigned* __restrict__ bad) {
  __shared__ float bq[QUANT ? kTable : 1];
  __shared__ __attribute__((aligned(16))) uint8_t Wb[4][16 * 16];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, g = lane >> 4;
  if (QUANT)
    for (int i = threadIdx.x; i < kTable; i += 256) bq[i] = beta32[i];
  __syncthreads();
  unsigned badf = 0;
  const int nblk16 = (n + 15) / 16;  // column blocks holding data
  const int64_t ntile = (m + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    const int64_t row0 = tile * 16;
    const int64_t row = row0 + li;
    const float* xr = X + (row < m ? row : m - 1) * ldx;
    f4v acc[NG];
#pragma unroll
    for (int gi = 0; gi < NG; gi++) acc[gi] = (f4v){0.f, 0.f, 0.f, 0.f};
    double nrm = 0.0;
    // column blocks in batches of four: 4 x 16 B per lane in flight
    for (int mb = 0; mb < nblk16; mb += 4) {
      float4 a[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int col = 16 * (mb + u) + 4 * g;
        a[u] = (row < m && mb + u < nblk16 && col < n) ? *reinterpret_cast<const float4*>(xr + col)
                                                        : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        if (mb + u >= nblk16) break;
        const int col = 16 * (mb + u) + 4 * g;
        nrm += (double)a[u].x * a[u].x + (double)a[u].y * a[u].y + (double)a[u].z * a[u].z +
               (double)a[u].w * a[u].w;
        if (!(isfinite(a[u].x) && isfinite(a[u].y) && isfinite(a[u].z) && isfinite(a[u].w))) badf = 1;
#pragma unroll
        for (int gi = 0; gi < NG; gi++) {
          const float4 b = *reinterpret_cast<const float4*>(BT + (int64_t)(gi * 16 + li) * n_pad + col);
          acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].x, b.x, acc[gi], 0, 0, 0);
          acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].y, b.y, acc[gi], 0, 0, 0);
          acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].z, b.z, acc[gi], 0, 0, 0);
          acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].w, b.w, acc[gi], 0, 0, 0);
        }
      }
    }
    // D[row 4g+r][col li] of each 16-column group
    if (out) {
#pragma unroll
      for (int gi = 0; gi < NG; gi++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int64_t ro = row0 + 4 * g + r;
          if (ro < m) out[ro * ld_out + gi * 16 + li] = acc[gi][r];
        }
    }
    if (norm2) {
      nrm += __shfl_xor(nrm, 16);
      nrm += __shfl_xor(nrm, 32);
      if (g == 0 && row < m) norm2[row] = nrm;
    }
    if (QUANT) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        float c = acc[0][r];
        int sy = 0;
        if (li < l) {
          const float* bj = bq + li * kAlphaMax;
#pragma unroll
          for (int step = 128; step > 0; step >>= 1)
            if (bj[sy + step - 1] <= c) sy += step;
        }
        Wb[wave][(4 * g + r) * 16 + li] = (uint8_t)sy;
      }
      // the wave's own staging bytes: order its LDS writes before its reads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < 16 && row0 + lane < m)
        *reinterpret_cast<uint4*>(words + (row0 + lane) * kWordBytes) =
            *reinterpret_cast<const uint4*>(&Wb[wave][lane * 16]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (bad && badf) atomicOr(bad, 1u);
}

template <int NG, bool QUANT>
static void launch_project_t(const float* X, int64_t m, int n, int64_t ldx, const float* bt,
                             int n_pad, float* out, int ld_out, const float* beta32, int l,
                             uint8_t* words, double* norm2, unsigned* bad, hipStream_t st) {
  // four 16-row tiles per workgroup round; enough workgroups to keep every
  // CU's waves loading
  int64_t tiles = (m + 63) / 64;
  unsigned grid = (unsigned)(tiles < 256 * 8 ? tiles : 256 * 8);
  if (grid == 0) grid = 1;
  k_project<NG, QUANT><<<grid, 256, 0, st>>>(X, m, n, ldx, bt, n_pad, out, ld_out, beta32, l,
                                             words, norm2, bad);
}

sofa_status launch_project(const float* X, int64_t m, int n, int64_t ldx, const float* bt, int ng,
                           int n_pad, float* out, int ld_out, const float* beta32, int l,
                           uint8_t* words, double* norm2, unsigned* bad, hipStream_t st) {
  if (m <= 0) return SOFA_OK;
  if ((n & 3) || (ldx & 3) || (reinterpret_cast<uintptr_t>(X) & 15))
    return set_error(SOFA_EINVAL, "projection needs n and the row stride to be multiples of 4 "
                                  "and a 16-byte aligned array");
  if (words) {
    if (ng != 1) return set_error(SOFA_EINTERNAL, "quantised projection needs one column group");
    launch_project_t<1, true>(X, m, n, ldx, bt, n_pad, out, ld_out, beta32, l, words, norm2, bad, st);
  } else {
    switch (ng) {
      case 1: launch_project_t<1, false>(X, m, n, ldx, bt, n_pad, out, ld_out, nullptr, 0, nullptr, norm2, bad, st); break;
      case 2: launch_project_t<2, false>(X, m, n, ldx, bt, n_pad, out, ld_out, nullptr, 0, nullptr, norm2, bad, st); break;
      case 3: launch_project_t<3, false>(X, m, n, ldx, bt, n_pad, out, ld_out, nullptr, 0, nullptr, norm2, bad, st); break;
      case 4: launch_project_t<4, false>(X, m, n, ldx, bt, n_pad, out, ld_out, nullptr, 0, nullptr, norm2, bad, st); break;
      default: return set_error(SOFA_EINTERNAL, "unsupported column groups %d", ng);
    }
  }
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// ----------------------------------------------------------------------------
// sort key of every row (sfa_key)
__global__ void k_keys(const uint8_t* __restrict__ words, int64_t N, int l, int alpha, int scheme,
                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint4 w = *reinterpret_cast<const uint4*>(words + i * kWordBytes);
  uint32_t wv[4] = {w.x, w.y, w.z, w.w};
  uint32_t s8[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    uint32_t s = (wv[j >> 2] >> (8 * (j & 3))) & 255u;
    s8[j] = (j < l) ? (s * 256u) / (uint32_t)alpha : 0u;
  }
  keys[i] = sfa_key(s8, scheme);
  vals[i] = (uint32_t)i;
}

// LSD radix sort of (u64 key, u32 value), 8-bit digits, stable.
constexpr int kRsItems = 16;
constexpr int kRsTile = 256 * kRsItems;

// per tile, the count of each digit (hist[digit][tile]); dsum[digit]
// accumulates the digit's total over the tiles (cleared beforehand)
__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t N,
                                                 int shift, uint32_t* __restrict__ hist,
                                                 int64_t ntiles, uint32_t* __restrict__ dsum) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; r++) {
    int64_t i = base + r * 256 + threadIdx.x;
    if (i < N) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t c = cnt[threadIdx.x];
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = c;
  if (c) atomicAdd(dsum + threadIdx.x, c);
}

// exclusive scan of hist in digit-major order, one workgroup per digit:
// the digit's start is the sum of the totals of the smaller digits, then
// its row of ntiles counts is scanned in pieces of 1024 x kScanPer
constexpr int kScanPer = 4;
__global__ __launch_bounds__(1024) void k_rs_scan(uint32_t* __restrict__ hist, int64_t ntiles,
                                                  const uint32_t* __restrict__ dsum) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t start;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int d = blockIdx.x;
  if (w == 0) {
    // sum of dsum[0..d), at most four values per lane
    uint32_t v = 0;
    for (int i = lane; i < d; i += 64) v += dsum[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) start = v;
  }
  __syncthreads();
  uint32_t carry = start;
  uint32_t* row = hist + (int64_t)d * ntiles;
  for (int64_t p0 = 0; p0 < ntiles; p0 += 1024 * kScanPer) {
    uint32_t v[kScanPer], s = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; e++) {
      const int64_t i = p0 + (int64_t)t * kScanPer + e;
      v[e] = i < ntiles ? row[i] : 0u;
      s += v[e];
    }
    uint32_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t x = wsum[i];
      wpre += i < w ? x : 0u;
      tot += x;
    }
    uint32_t ex = carry + wpre + incl - s;
#pragma unroll
    for (int e = 0; e < kScanPer; e++) {
      const int64_t i = p0 + (int64_t)t * kScanPer + e;
      if (i < ntiles) row[i] = ex;
      ex += v[e];
    }
    carry += tot;
    __syncthreads();  // wsum is rewritten by the next piece
  }
}

__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout, int64_t N,
                                                    int shift, const uint32_t* __restrict__ hist,
                                                    int64_t ntiles) {
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t wc[4][256];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  gbase[t] = hist[(int64_t)t * ntiles + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kRsItems; r++) {
    int64_t i = base + r * 256 + t;
    bool valid = i < N;
    uint64_t k = valid ? kin[i] : ~0ull;
    uint32_t v = valid ? vin[i] : 0u;
    uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t peers = ~0ull;
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
      uint64_t bal = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bal : ~bal;
    }
    uint32_t rank = (uint32_t)__popcll(peers & lt);
    wc[0][t] = 0u;
    wc[1][t] = 0u;
    wc[2][t] = 0u;
    wc[3][t] = 0u;
    __syncthreads();
    if (rank == 0) wc[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t run = gbase[t];
      for (int w = 0; w < 4; w++) {
        uint32_t c = wc[w][t];
        wc[w][t] = run;
        run += c;
      }
      gbase[t] = run;
    }
    __syncthreads();
    if (valid) {
      uint32_t dst = wc[wave][d] + rank;
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
  }
}

// permuted copy: leaf-order position p holds row src = perm[p].  A wave
// moves kPermRows rows per step, all their loads issued before any store.
constexpr int kPermRows = 4;
__global__ __launch_bounds__(256) void k_permute(const float* __restrict__ X, int n,
                                                 const uint32_t* __restrict__ perm, int64_t N,
                                                 int n_pad, float* __restrict__ Xo,
                                                 const uint8_t* __restrict__ win,
                                                 uint8_t* __restrict__ wout,
                                                 const double* __restrict__ nin,
                                                 double* __restrict__ nout,
                                                 int32_t* __restrict__ ids) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * kPermRows; p0 < N; p0 += nw * kPermRows) {
    for (int c0 = 0; c0 < n_pad; c0 += 256) {
      const int c = c0 + lane * 4;
      if (c >= n_pad) break;  // rows shorter than 256 values: lanes past the row idle
      float4 v[kPermRows];
#pragma unroll
      for (int r = 0; r < kPermRows; r++) {
        const int64_t p = p0 + r;
        v[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < N && c < n) v[r] = *reinterpret_cast<const float4*>(X + (int64_t)perm[p] * n + c);
      }
#pragma unroll
      for (int r = 0; r < kPermRows; r++)
        if (p0 + r < N) *reinterpret_cast<float4*>(Xo + (p0 + r) * n_pad + c) = v[r];
    }
    if (lane < kPermRows && p0 + lane < N) {
      const int64_t p = p0 + lane, src = perm[p];
      *reinterpret_cast<uint4*>(wout + p * kWordBytes) = *reinterpret_cast<const uint4*>(win + src * kWordBytes);
      nout[p] = nin[src];
      ids[p] = (int32_t)src;
    }
  }
}

// per-leaf envelope: lo[16] then hi[16] symbols; one wave per leaf
__global__ __launch_bounds__(256) void k_envelope(const uint8_t* __restrict__ words, int64_t N,
                                                  int L, int64_t n_leaves,
                                                  uint8_t* __restrict__ env) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t leaf = (int64_t)blockIdx.x * 4 + wave;
  if (leaf >= n_leaves) return;
  int64_t s = leaf * L, e = s + L < N ? s + L : N;
  uint32_t lo[16], hi[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    lo[j] = 255u;
    hi[j] = 0u;
  }
  for (int64_t p = s + lane; p < e; p += 64) {
    uint4 w = *reinterpret_cast<const uint4*>(words + p * kWordBytes);
    uint32_t wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 16; j++) {
      uint32_t b = (wv[j >> 2] >> (8 * (j & 3))) & 255u;
      lo[j] = b < lo[j] ? b : lo[j];
      hi[j] = b > hi[j] ? b : hi[j];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int j = 0; j < 16; j++) {
      uint32_t a = __shfl_xor(lo[j], off), b = __shfl_xor(hi[j], off);
      lo[j] = a < lo[j] ? a : lo[j];
      hi[j] = b > hi[j] ? b : hi[j];
    }
  if (lane < 32) {
    uint32_t v = lane < 16 ? lo[0] : hi[0];
#pragma unroll
    for (int j = 1; j < 16; j++)
      if ((lane & 15) == j) v = lane < 16 ? lo[j] : hi[j];
    env[leaf * 32 + lane] = (uint8_t)v;
  }
}

// maximum of FP64 squared norms (non-negative, so the bit patterns order like the values)
__global__ __launch_bounds__(256) void k_max_norm(const double* __restrict__ nrm, int64_t N,
                                                  unsigned long long* __restrict__ out) {
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256)
    mx = nrm[i] > mx ? nrm[i] : mx;
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(mx));
}

sofa_status launch_layout(sofa_index* ix, const float* X, const uint8_t* words_in,
                          const double* norm2_in, hipStream_t st) {
  const int64_t N = ix->N;
  const int n = ix->n, n_pad = ix->n_pad;
  DevBuf k0, k1, v0, v1, hist, dsum, mx;
  SOFA_TRY(k0.alloc(8 * N));
  SOFA_TRY(k1.alloc(8 * N));
  SOFA_TRY(v0.alloc(4 * N));
  SOFA_TRY(v1.alloc(4 * N));
  const int64_t ntiles = (N + kRsTile - 1) / kRsTile;
  SOFA_TRY(hist.alloc(4 * 256 * ntiles));
  SOFA_TRY(dsum.alloc(4 * 256 * 8));  // digit totals of each of the 8 passes
  SOFA_TRY(mx.alloc(8));
  SOFA_TRY(launch_fill_u32(dsum.as<uint32_t>(), 0u, 256 * 8, st));
  k_keys<<<nblk(N, 256), 256, 0, st>>>(words_in, N, ix->bins.l, ix->bins.alpha, ix->key_scheme,
                                       k0.as<uint64_t>(), v0.as<uint32_t>());
  uint64_t *ka = k0.as<uint64_t>(), *kb = k1.as<uint64_t>();
  uint32_t *va = v0.as<uint32_t>(), *vb = v1.as<uint32_t>();
  for (int shift = 0; shift < 64; shift += 8) {
    uint32_t* ds = dsum.as<uint32_t>() + 256 * (shift / 8);
    k_rs_hist<<<(unsigned)ntiles, 256, 0, st>>>(ka, N, shift, hist.as<uint32_t>(), ntiles, ds);
    k_rs_scan<<<256, 1024, 0, st>>>(hist.as<uint32_t>(), ntiles, ds);
    k_rs_scatter<<<(unsigned)ntiles, 256, 0, st>>>(ka, va, kb, vb, N, shift, hist.as<uint32_t>(), ntiles);
    uint64_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
  }
  // after 8 passes the sorted keys/values are back in k0/v0
  SOFA_TRY(ix->X.alloc(sizeof(float) * N * n_pad));
  SOFA_TRY(ix->words.alloc(kWordBytes * N));
  SOFA_TRY(ix->ids.alloc(4 * N));
  SOFA_TRY(ix->norm2.alloc(8 * N));
  SOFA_TRY(ix->env.alloc(32 * ix->n_leaves));
  k_permute<<<grid_blocks(N, 4 * kPermRows), 256, 0, st>>>(X, n, va, N, n_pad, ix->X.as<float>(), words_in,
                                        ix->words.as<uint8_t>(), norm2_in, ix->norm2.as<double>(),
                                        ix->ids.as<int32_t>());
  k_envelope<<<nblk(ix->n_leaves, 4), 256, 0, st>>>(ix->words.as<uint8_t>(), N, ix->L, ix->n_leaves,
                                                   ix->env.as<uint8_t>());
  SOFA_HIP(hipMemsetAsync(mx.p, 0, 8, st));
  k_max_norm<<<1024, 256, 0, st>>>(ix->norm2.as<double>(), N, mx.as<unsigned long long>());
  SOFA_HIP(hipGetLastError());
  unsigned long long bits = 0;
  SOFA_HIP(hipMemcpyAsync(&bits, mx.p, 8, hipMemcpyDeviceToHost, st));
  SOFA_HIP(hipStreamSynchronize(st));
  double mn2;
  memcpy(&mn2, &bits, 8);
  ix->max_norm = sqrt(mn2);
  // keep the sorted keys for inspection
  ix->keys.take(k0);
  return SOFA_OK;
}

}  // namespace sofa
