// k_bf16.hip -- batched-distance prune on the matrix cores (BF16 inputs,
// FP32 accumulation), used only to discard rows under a rigorous bound; the
// survivors are refined with exact FP32 distances and ranked in FP64.
//
// For a query q and a row x (both FP32) with BF16 copies qh, xh,
//   q.x = qh.xh + q.(x - xh) + (q - qh).xh
// so with P the FP32 MFMA sum of the exact BF16 products,
//   q.x <= P + g*|qh||xh| + |q| r_x + r_q |xh|,   r_x = |x - xh|, r_q = |q - qh|,
// where g = (K + 16) 2^-23 bounds the FP32 accumulation of K products.  Then
//   d^2 = |q|^2 + |x|^2 - 2 q.x >= |q|^2 + |x|^2 - 2 P - 2 (g|qh||xh| + |q| r_x + r_q |xh|),
// and a row is kept only when this lower bound does not exceed the query's
// bound U on the k-th distance.  |x|^2 and |q|^2 are rounded down, r_x, r_q,
// |xh|, |qh| up, and a relative 2^-20 of |q|^2 + |x|^2 covers the FP32
// evaluation of the bound.  Per leaf, |xh| and r_x enter through their
// maxima over the leaf, so the per-pair epilogue is one FMA and a compare.
//
// Layout: the BF16 copy is stored in v_mfma_f32_32x32x16_bf16 A-operand
// order, so that one wave's fragment load for a 32-row x 16-column block is
// one contiguous 1 KB read.  A workgroup takes 256 rows (4 waves x 64 rows,
// operand held in registers) and loops over the 64-query groups that have a
// surviving (query, leaf) pair; each group's BF16 query fragments are staged
// in LDS.  Queries are ordered by their number of surviving leaves, so that
// queries the SFA bound cannot prune share groups.
#include "bf16.h"

namespace sofa {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));  // plain 16-byte vector (no struct copies)

static inline unsigned nblk(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return u >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t h) { return __uint_as_float(h << 16); }

// FP32 -> OCP e4m3 (no infinities, largest finite 448), round to nearest
// even; |v| <= 448 (the power-of-two scales guarantee it), so the NaN code
// 0x7F never appears
__device__ __forceinline__ uint32_t e4m3_code(float v) {
  const uint32_t sgn = (__float_as_uint(v) >> 31) << 7;
  const float a = fabsf(v);
  uint32_t code;
  if (a < 0x1p-6f) {
    code = (uint32_t)rintf(a * 0x1p9f);  // subnormal step 2^-9; 8 is the smallest normal
  } else {
    int ex;
    (void)frexpf(a, &ex);  // a = f 2^ex, f in [0.5, 1)
    int e = ex - 1;        // a in [2^e, 2^(e+1))
    uint32_t m = (uint32_t)rintf(ldexpf(a, 3 - e));  // 8..16
    if (m == 16) {
      m = 8;
      e++;
    }
    code = ((uint32_t)(e + 7) << 3) | (m - 8);
  }
  return sgn | code;
}
__device__ __forceinline__ float e4m3_val(uint32_t c) {
  const int ef = (int)((c >> 3) & 15u);
  const float m = (float)(c & 7u);
  const float mag = ef == 0 ? ldexpf(m, -9) : ldexpf(8.0f + m, ef - 10);
  return (c & 0x80u) ? -mag : mag;
}
// smallest power of two s with 448 s >= maxabs (1 for an all-zero block)
__device__ __forceinline__ float fp8_scale_for(float maxabs) {
  if (!(maxabs > 0.0f)) return 1.0f;
  int e = ilogbf(maxabs) - 8;
  while (ldexp(448.0, e) < (double)maxabs) e++;
  while (ldexp(448.0, e - 1) >= (double)maxabs) e--;
  return ldexpf(1.0f, e);
}
// 16 consecutive FP32 values scaled by inv (a power of two) -> 16 e4m3 codes
__device__ __forceinline__ uint4 fp8_pack16(const float* __restrict__ p, float inv) {
  uint32_t w[4];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const float4 v = *reinterpret_cast<const float4*>(p + 4 * j);
    w[j] = e4m3_code(v.x * inv) | (e4m3_code(v.y * inv) << 8) | (e4m3_code(v.z * inv) << 16) |
           (e4m3_code(v.w * inv) << 24);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// ----------------------------------------------------------------------------
// per row: |x|^2 rounded down, r_x = |x - xh| up, |xh| up (one wave per row)
__device__ __forceinline__ void norms_of(const float* __restrict__ row, int n_pad, int lane,
                                         float4& out) {
  double s2 = 0.0, r2 = 0.0, h2 = 0.0;
  for (int c = lane * 4; c < n_pad; c += 256) {
    float4 v = *reinterpret_cast<const float4*>(row + c);
    float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      double x = xs[e], h = bf16_val(bf16_bits(xs[e]));
      s2 += x * x;
      r2 += (x - h) * (x - h);
      h2 += h * h;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s2 += __shfl_xor(s2, o);
    r2 += __shfl_xor(r2, o);
    h2 += __shfl_xor(h2, o);
  }
  out = make_float4(__double2float_rd(s2 * (1.0 - 1e-12)), __double2float_ru(sqrt(r2) * (1.0 + 1e-12)),
                    __double2float_ru(sqrt(h2) * (1.0 + 1e-12)), 0.0f);
}

// the same for the FP8 copy: xh = sc * e4m3(x / sc)
__device__ __forceinline__ void norms_of_fp8(const float* __restrict__ row, int n_pad, int lane,
                                             float sc, float4& out) {
  const float inv = 1.0f / sc;  // exact: sc is a power of two
  double s2 = 0.0, r2 = 0.0, h2 = 0.0;
  for (int c = lane * 4; c < n_pad; c += 256) {
    float4 v = *reinterpret_cast<const float4*>(row + c);
    float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      double x = xs[e], h = (double)sc * (double)e4m3_val(e4m3_code(xs[e] * inv));
      s2 += x * x;
      r2 += (x - h) * (x - h);
      h2 += h * h;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s2 += __shfl_xor(s2, o);
    r2 += __shfl_xor(r2, o);
    h2 += __shfl_xor(h2, o);
  }
  out = make_float4(__double2float_rd(s2 * (1.0 - 1e-12)), __double2float_ru(sqrt(r2) * (1.0 + 1e-12)),
                    __double2float_ru(sqrt(h2) * (1.0 + 1e-12)), 0.0f);
}

// build: the swizzled BF16 copy and its per-row terms in one read of X.
// Fragment slot ((rb*KS + ks)*64 + lane) holds the 8 values of row
// rb*32 + lane%32, columns ks*16 + 8*(lane/32) + e.  One wave per 32-row
// block writes the block's fragments and sums each row's terms over its
// half of the columns in FP64; the two halves meet by one exchange.
__global__ __launch_bounds__(256) void k_bf16_copy_meta(const float* __restrict__ X, int64_t N, int n_pad,
                                                        int64_t nrb, uint4* __restrict__ xb,
                                                        float4* __restrict__ meta) {
  const int KS = n_pad / 16;
  const int lane = threadIdx.x & 63;
  for (int64_t rb = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); rb < nrb; rb += (int64_t)gridDim.x * 4) {
    const int64_t row = rb * 32 + lane % 32;
    const bool live = row < N;
    double s2 = 0.0, r2 = 0.0, h2 = 0.0;
    for (int ks = 0; ks < KS; ks++) {
      const int k0 = ks * 16 + 8 * (lane / 32);
      uint32_t w[4] = {0, 0, 0, 0};
      if (live) {
        const float4 a = *reinterpret_cast<const float4*>(X + row * n_pad + k0);
        const float4 b = *reinterpret_cast<const float4*>(X + row * n_pad + k0 + 4);
        const float xs[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int e = 0; e < 8; e++) {
          const uint32_t h = bf16_bits(xs[e]);
          w[e / 2] |= h << (16 * (e & 1));
          const double x = xs[e], hv = bf16_val(h);
          s2 += x * x;
          r2 += (x - hv) * (x - hv);
          h2 += hv * hv;
        }
      }
      xb[(rb * KS + ks) * 64 + lane] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    s2 += __shfl_xor(s2, 32);
    r2 += __shfl_xor(r2, 32);
    h2 += __shfl_xor(h2, 32);
    if (lane < 32 && live)
      meta[row] = make_float4(__double2float_rd(s2 * (1.0 - 1e-12)), __double2float_ru(sqrt(r2) * (1.0 + 1e-12)),
                              __double2float_ru(sqrt(h2) * (1.0 + 1e-12)), 0.0f);
  }
}

// per leaf: (max |xh|, max r_x, max |x|^2)
__global__ __launch_bounds__(256) void k_bf16_leafmeta(const float4* __restrict__ meta, int64_t N,
                                                       int L, int64_t n_leaves,
                                                       float4* __restrict__ lm) {
  const int lane = threadIdx.x & 63;
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (leaf >= n_leaves) return;
  float xh = 0.0f, rx = 0.0f, xn = 0.0f;
  for (int64_t p = leaf * L + lane; p < (leaf + 1) * L && p < N; p += 64) {
    float4 m = meta[p];
    xh = fmaxf(xh, m.z);
    rx = fmaxf(rx, m.y);
    xn = fmaxf(xn, m.x);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    xh = fmaxf(xh, __shfl_xor(xh, o));
    rx = fmaxf(rx, __shfl_xor(rx, o));
    xn = fmaxf(xn, __shfl_xor(xn, o));
  }
  // |x|^2 was rounded down: the margin below uses a value rounded up
  if (lane == 0) lm[leaf] = make_float4(xh, rx, xn * (1.0f + 0x1p-20f), 0.0f);
}

// ----------------------------------------------------------------------------
// build: FP8 copy.  A power-of-two scale per 256-row chunk, then the e4m3
// copy and each row's terms, one workgroup per chunk: the chunk's maximum
// |x| first (its 256 rows then sit in the caches), then wave w writes row
// blocks 2w and 2w + 1 of the chunk.  Fragment half h of slot
// ((rb*KS + ks)*2 + h)*64 + lane holds row rb*32 + lane%32, columns
// 64 ks + 32 (lane/32) + 16 h + (0..15); the lane sums its row's terms over
// its half of the columns in FP64, and the two halves meet by one exchange.
__global__ __launch_bounds__(256) void k_fp8_chunk_build(const float* __restrict__ X, int64_t N, int n_pad,
                                                         float* __restrict__ cscale, uint4* __restrict__ xf,
                                                         float4* __restrict__ meta) {
  __shared__ float red[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int KS = n_pad / 64;
  const int64_t n_chunks = (N + 255) / 256;
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int64_t c0 = chunk * 256;
    float m = 0.0f;
    for (int r = wave; r < 256 && c0 + r < N; r += 4)
      for (int c = lane * 4; c < n_pad; c += 256) {
        const float4 v = *reinterpret_cast<const float4*>(X + (c0 + r) * n_pad + c);
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) red[wave] = m;
    __syncthreads();
    const float sc = fp8_scale_for(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
    __syncthreads();  // red is rewritten by the next chunk
    if (threadIdx.x == 0) cscale[chunk] = sc;
    const float inv = 1.0f / sc;  // exact: sc is a power of two
    for (int b2 = 0; b2 < 2; b2++) {
      const int64_t rb = chunk * 8 + 2 * wave + b2;
      const int64_t row = rb * 32 + lane % 32;
      const bool live = row < N;
      double s2 = 0.0, r2 = 0.0, h2 = 0.0;
      for (int ks = 0; ks < KS; ks++)
        for (int hh = 0; hh < 2; hh++) {
          const int k0 = ks * 64 + 32 * (lane / 32) + 16 * hh;
          uint32_t w[4] = {0, 0, 0, 0};
          if (live) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
              const float4 v = *reinterpret_cast<const float4*>(X + row * n_pad + k0 + 4 * j);
              const float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
              for (int e = 0; e < 4; e++) {
                const uint32_t code = e4m3_code(xs[e] * inv);
                w[j] |= code << (8 * e);
                const double x = xs[e], hv = (double)sc * (double)e4m3_val(code);
                s2 += x * x;
                r2 += (x - hv) * (x - hv);
                h2 += hv * hv;
              }
            }
          }
          xf[((rb * KS + ks) * 2 + hh) * 64 + lane] = make_uint4(w[0], w[1], w[2], w[3]);
        }
      s2 += __shfl_xor(s2, 32);
      r2 += __shfl_xor(r2, 32);
      h2 += __shfl_xor(h2, 32);
      if (lane < 32 && live)
        meta[row] = make_float4(__double2float_rd(s2 * (1.0 - 1e-12)), __double2float_ru(sqrt(r2) * (1.0 + 1e-12)),
                                __double2float_ru(sqrt(h2) * (1.0 + 1e-12)), 0.0f);
    }
  }
}

// ----------------------------------------------------------------------------
// query side
// surviving leaves per query
// surviving leaves per query; grid (query blocks, slices of the leaf blocks),
// cnt cleared beforehand
__global__ void k_qcount(const uint64_t* __restrict__ masks, int64_t n_blocks, int B,
                         uint32_t* __restrict__ cnt) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B) return;
  uint32_t c = 0;
  for (int64_t b = blockIdx.y; b < n_blocks; b += gridDim.y) c += __popcll(masks[b * B + q]);
  if (c) atomicAdd(cnt + q, c);
}

// Query order for the groups: density class first (0 when at least half of
// the leaves survive, c when the surviving fraction is in [2^-(c+1), 2^-c),
// at most 7), then the query's best leaf, so that a group gathers queries
// whose surviving leaves overlap; ties by query index.
__device__ __forceinline__ uint64_t qorder_key(uint32_t cnt, uint64_t best, int64_t n_leaves) {
  int cls = 7;
  if (cnt > 0) {
    cls = 0;
    while (cls < 7 && ((uint64_t)cnt << (cls + 1)) < (uint64_t)n_leaves) cls++;
  }
  const uint64_t leaf = best == kEmpty ? 0xFFFFFFFFFFFFull : (uint64_t)(uint32_t)best;
  return ((uint64_t)cls << 48) | leaf;
}

// rank sort, one wave per query (best may be null: order by density only)
__global__ __launch_bounds__(256) void k_qsort(const uint32_t* __restrict__ cnt,
                                               const uint64_t* __restrict__ best, int B,
                                               int64_t n_leaves, int32_t* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= B) return;
  const uint64_t kq = qorder_key(cnt[q], best ? best[q] : kEmpty, n_leaves);
  int rank = 0;
  for (int o = lane; o < B; o += 64) {
    const uint64_t ko = qorder_key(cnt[o], best ? best[o] : kEmpty, n_leaves);
    rank += (ko < kq || (ko == kq && o < q)) ? 1 : 0;
  }
  for (int off = 32; off > 0; off >>= 1) rank += __shfl_xor(rank, off);
  if (lane == 0) perm[rank] = q;
}

// smask[blk][s]: the survivor mask of the query in sorted slot s (0 past B)
__global__ void k_smask(const uint64_t* __restrict__ masks, int64_t n_blocks, int B, int Spad,
                        const int32_t* __restrict__ perm, uint64_t* __restrict__ smask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_blocks * Spad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / Spad;
    const int s = (int)(i % Spad);
    smask[i] = s < B ? masks[b * B + perm[s]] : 0ull;
  }
}

// per leaf, the sorted slots of the queries whose (query, leaf) pair
// survives.  Workgroup g takes the 16 leaves of sub-block g (a quarter of
// mask block g / 4), whose mask row it stages through LDS 1024 slots at a
// time; wave w handles leaves 4w .. 4w + 3 of the sub-block.  PASS 0 counts
// (lcnt) and sums the sub-block (bsum); PASS 1 takes the sub-block's offset
// from boff (the exclusive scan of bsum), writes each leaf's offset (loff)
// and fills lslot.
constexpr int kSubLeaves = 16;
constexpr int kSubPerBlock = kLeavesPerItem / kSubLeaves;

template <int PASS>
__global__ __launch_bounds__(256) void k_leaf_lists(const uint64_t* __restrict__ smask, int64_t n_leaves,
                                                    int Spad, uint32_t* __restrict__ lcnt,
                                                    uint32_t* __restrict__ bsum,
                                                    const int64_t* __restrict__ boff,
                                                    int64_t* __restrict__ loff,
                                                    uint16_t* __restrict__ lslot) {
  constexpr int kRow = 1024;
  __shared__ uint64_t row[kRow];
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t sub = blockIdx.x;
  const int64_t blk = sub / kSubPerBlock;
  const int shift = (int)(sub % kSubPerBlock) * kSubLeaves + 4 * wave;  // bit of leaf j: shift + j
  const uint64_t* sm = smask + blk * Spad;
  const int64_t leaf0 = sub * kSubLeaves + 4 * wave;
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t c[4];
  int64_t base[4];
  if (PASS) {
    // offsets of the sub-block's leaves: an exclusive scan of their counts
    const int64_t leaf = sub * kSubLeaves + lane;
    const uint32_t cl = lane < kSubLeaves && leaf < n_leaves ? lcnt[leaf] : 0u;
    uint32_t incl = cl;
#pragma unroll
    for (int o = 1; o < kSubLeaves; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    const int64_t off = boff[sub] + (int64_t)(incl - cl);
    if (wave == 0 && lane < kSubLeaves && leaf < n_leaves) loff[leaf] = off;
#pragma unroll
    for (int j = 0; j < 4; j++) base[j] = __shfl(off, 4 * wave + j);
  }
#pragma unroll
  for (int j = 0; j < 4; j++) c[j] = 0;
  for (int s0 = 0; s0 < Spad; s0 += kRow) {
    const int m = Spad - s0 < kRow ? Spad - s0 : kRow;  // a multiple of 64
    __syncthreads();  // the previous piece has been read
    for (int i = threadIdx.x; i < m; i += 256) row[i] = sm[s0 + i];
    __syncthreads();
    for (int t0 = 0; t0 < m; t0 += 64) {
      const uint64_t wv = row[t0 + lane] >> shift;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const bool on = leaf0 + j < n_leaves && ((wv >> j) & 1ull);
        const uint64_t bal = __ballot(on);
        if (PASS && on) lslot[base[j] + c[j] + __popcll(bal & lt)] = (uint16_t)(s0 + t0 + lane);
        c[j] += (uint32_t)__popcll(bal);
      }
    }
  }
  if (PASS == 0) {
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (lane == 0 && leaf0 + j < n_leaves) lcnt[leaf0 + j] = c[j];
      tot += c[j];
    }
    if (lane == 0) wsum[wave] = tot;
    __syncthreads();
    if (threadIdx.x == 0) bsum[sub] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  }
}

// exclusive prefix sum of counts (the leaf blocks' list lengths): one
// workgroup walks tiles of 4096 counts (4 per thread, a block-wide scan
// each) while the next tile loads
__global__ __launch_bounds__(1024) void k_scan_counts(const uint32_t* __restrict__ cnt, int64_t n,
                                                      int64_t* __restrict__ off) {
  constexpr int kTile = 4096;
  __shared__ int64_t wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t cur[4], nxt[4];
#pragma unroll
  for (int e = 0; e < 4; e++) {
    const int64_t i = 4 * t + e;
    cur[e] = i < n ? cnt[i] : 0u;
  }
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += kTile) {
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int64_t i = base + kTile + 4 * t + e;
      nxt[e] = i < n ? cnt[i] : 0u;
    }
    const int64_t sv = (int64_t)cur[0] + cur[1] + cur[2] + cur[3];
    int64_t incl = sv;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int64_t wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const int64_t v = wsum[i];
      wpre += i < w ? v : 0;
      tot += v;
    }
    int64_t ex = carry + wpre + incl - sv;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int64_t i = base + 4 * t + e;
      if (i < n) off[i] = ex;
      ex += cur[e];
    }
    carry += tot;
    __syncthreads();  // wsum is rewritten by the next tile
#pragma unroll
    for (int e = 0; e < 4; e++) cur[e] = nxt[e];
  }
}

// per slot, for the current pass: with t = |x|^2 - 2P, a row survives when
//   t <= a + b * max|xh| + c * max r_x + 2^-20 * max|x|^2   (leaf maxima)
// where a = U lb_f - |q|^2 (1 - 2^-20), b = 2 (g |qh| + r_q), c = 2 |q|; .w = query id
// With ccnt (B entries) and the work counter given, the same launch clears
// them for the pass.
__global__ void k_slotc(const float4* __restrict__ qmeta, const int32_t* __restrict__ perm, int B,
                        int Spad, const uint32_t* __restrict__ U, float lb_f, float gam,
                        float4* __restrict__ slotc, uint32_t* __restrict__ ccnt,
                        uint32_t* __restrict__ counter) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (counter && s == 0) *counter = 0u;
  if (ccnt && s < B) ccnt[s] = 0u;
  if (s >= Spad) return;
  float4 c = make_float4(-INFINITY, 0.0f, 0.0f, __int_as_float(-1));
  if (s < B) {
    const int q = perm[s];
    const float4 qm = qmeta[s];
    const float u = __uint_as_float(U[q]);
    c = make_float4(u * lb_f - qm.x * (1.0f - 0x1p-20f), 2.0f * (gam * qm.z + qm.y), 2.0f * qm.w,
                    __int_as_float(q));
  }
  slotc[s] = c;
}

// BF16 query rows per sorted slot (n_pad values, zero past B); a lane's
// fragment of the 32x32x16 B operand is 16 contiguous bytes of one row
__global__ void k_qrows_bf16(const float* __restrict__ Qp, int B, int n_pad, int Spad,
                             const int32_t* __restrict__ perm, uint4* __restrict__ qb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = n_pad / 8;
  if (i >= (int64_t)Spad * per) return;
  const int s = (int)(i / per), k0 = (int)(i % per) * 8;
  uint32_t w[4] = {0, 0, 0, 0};
  if (s < B) {
    const float* qr = Qp + (int64_t)perm[s] * n_pad;
    float4 a = *reinterpret_cast<const float4*>(qr + k0);
    float4 b = *reinterpret_cast<const float4*>(qr + k0 + 4);
    w[0] = bf16_bits(a.x) | (bf16_bits(a.y) << 16);
    w[1] = bf16_bits(a.z) | (bf16_bits(a.w) << 16);
    w[2] = bf16_bits(b.x) | (bf16_bits(b.y) << 16);
    w[3] = bf16_bits(b.z) | (bf16_bits(b.w) << 16);
  }
  qb[i] = make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ __launch_bounds__(256) void k_qmeta_bf16(const float* __restrict__ Qp, int B, int n_pad,
                                                    const int32_t* __restrict__ perm, int Spad,
                                                    float4* __restrict__ qmeta) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= Spad) return;
  float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
  if (s < B) norms_of(Qp + (int64_t)perm[s] * n_pad, n_pad, lane, m);
  // m = (|q|^2 down, r_q up, |qh| up); the bound also needs |q| (up)
  if (lane == 0) {
    m.w = __double2float_ru(sqrt((double)m.x) * (1.0 + 1e-7) + 1e-30);
    qmeta[s] = m;
  }
}

// FP8 query side: a power-of-two scale per slot, e4m3 rows, the same bound
// terms
__global__ __launch_bounds__(256) void k_qscale_fp8(const float* __restrict__ Qp, int B, int n_pad,
                                                    const int32_t* __restrict__ perm, int Spad,
                                                    float* __restrict__ qscale) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= Spad) return;
  float m = 0.0f;
  if (s < B) {
    const float* qr = Qp + (int64_t)perm[s] * n_pad;
    for (int c = lane * 4; c < n_pad; c += 256) {
      const float4 v = *reinterpret_cast<const float4*>(qr + c);
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) qscale[s] = fp8_scale_for(m);
}

__global__ void k_qrows_fp8(const float* __restrict__ Qp, int B, int n_pad, int Spad,
                            const int32_t* __restrict__ perm, const float* __restrict__ qscale,
                            uint4* __restrict__ qb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = n_pad / 16;
  if (i >= (int64_t)Spad * per) return;
  const int s = (int)(i / per), k0 = (int)(i % per) * 16;
  uint4 w = make_uint4(0u, 0u, 0u, 0u);
  if (s < B) w = fp8_pack16(Qp + (int64_t)perm[s] * n_pad + k0, 1.0f / qscale[s]);
  qb[i] = w;
}

__global__ __launch_bounds__(256) void k_qmeta_fp8(const float* __restrict__ Qp, int B, int n_pad,
                                                   const int32_t* __restrict__ perm, int Spad,
                                                   const float* __restrict__ qscale,
                                                   float4* __restrict__ qmeta) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= Spad) return;
  float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
  if (s < B) norms_of_fp8(Qp + (int64_t)perm[s] * n_pad, n_pad, lane, qscale[s], m);
  if (lane == 0) {
    m.w = __double2float_ru(sqrt((double)m.x) * (1.0 + 1e-7) + 1e-30);
    qmeta[s] = m;
  }
}

// ----------------------------------------------------------------------------
// tiles: one 256-row chunk per work item
//
// Per group, the two 32-query column blocks are taken one after the other
// (32 accumulators live instead of 64; each query fragment is read from LDS
// once).  With f = 2 (BF16) or f = 2 s_q s_c (FP8; exact, both scales are
// powers of two), t = |x|^2 - f P.  The usual fragment has no hit, so the
// epilogue first tests a superset: for the 16 rows e of a lane's fragment,
//   min_e fl(|x_e|^2 - f P_e) >= fl(min_e |x_e|^2 - f max_e P_e)
// (rounding is monotone), and only when that value passes the per-query
// threshold for some lane of the wave are the 16 pairs tested one by one.
//
// The groups of a chunk alternate between two LDS buffers: while the matrix
// cores read one, the next group's fragments stream into the other by LDS
// DMA (global_load_lds_dwordx4, no registers), and the next group's
// per-column terms are loaded into registers.  The two buffers are separate
// arrays so that reads of one never wait on the DMA into the other.
//
// PREC 1: BF16, v_mfma_f32_32x32x16_bf16, fragment = 8 values (16 bytes) per
// lane, K step 16.  PREC 2: FP8 e4m3, v_mfma_f32_32x32x64_f8f6f4, fragment =
// 32 values per lane stored as two 16-byte halves, K step 64.  KS = n_pad /
// (K step).  Rows and queries use the same fragment order, so the products
// pair up whatever order the instruction takes within a fragment.

typedef int v8i __attribute__((ext_vector_type(8)));

template <int PREC> struct TileTraits;
template <> struct TileTraits<1> {
  typedef bf8v frag;
  static constexpr int kHalves = 1, kStep = 16;
};
template <> struct TileTraits<2> {
  typedef v8i frag;
  static constexpr int kHalves = 2, kStep = 64;
};

template <int PREC>
__device__ __forceinline__ typename TileTraits<PREC>::frag load_frag(const u4v* p) {
  if constexpr (PREC == 1) {
    return __builtin_bit_cast(bf8v, p[0]);
  } else {
    const u4v lo = p[0], hi = p[64];
    return __builtin_bit_cast(v8i, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
  }
}

template <int PREC>
__device__ __forceinline__ f16v mma(typename TileTraits<PREC>::frag a, typename TileTraits<PREC>::frag b,
                                    f16v c) {
  if constexpr (PREC == 1)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  else  // A and B formats 0 = FP8 e4m3; no block scales
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// A group: 64 consecutive entries of the leaf's list of surviving queries
// (sorted slots).  Each lane serves columns lane%32 and 32 + lane%32.
struct GroupSlots {
  int s0, s1;     // sorted slots of the lane's two columns
  bool v0, v1;    // whether those columns exist (the last group may be short)
};

__device__ __forceinline__ GroupSlots group_slots(const Bf16Args& b, int64_t off, uint32_t cnt, int g,
                                                  int lane) {
  const uint32_t c0 = (uint32_t)g * kGroup + (lane & 31), c1 = c0 + 32;
  GroupSlots r;
  r.v0 = c0 < cnt;
  r.v1 = c1 < cnt;
  r.s0 = b.lslot[off + (r.v0 ? c0 : 0)];  // a short group repeats its first slot (unused)
  r.s1 = b.lslot[off + (r.v1 ? c1 : 0)];
  return r;
}

// per-column terms of a group's two 32-query blocks
struct ColTerms {
  float4 c0, c1;    // bound terms (a, b, c) and query id
  float s0, s1;     // FP8 query scales
  bool v0, v1;
};

template <int PREC>
__device__ __forceinline__ void load_cols(const Bf16Args& b, const GroupSlots& gs, ColTerms& t) {
  t.c0 = b.slotc[gs.s0];
  t.c1 = b.slotc[gs.s1];
  t.v0 = gs.v0;
  t.v1 = gs.v1;
  if constexpr (PREC == 2) {
    t.s0 = b.qscale[gs.s0];
    t.s1 = b.qscale[gs.s1];
  } else {
    t.s0 = t.s1 = 1.0f;
  }
}

// u4v (16-byte) units of one group's fragments
template <int PREC, int KS>
constexpr int group_units() { return 2 * KS * 64 * TileTraits<PREC>::kHalves; }

// LDS DMA of a group's B fragments into dst, gathered from the query rows:
// piece p (64 lanes x 16 B, a quarter of the pieces per wave) is column
// block cb, K step ks (and half hh for FP8); lane l reads the 16 contiguous
// bytes of its column's row that the instruction's operand layout puts there.
// The gathers are buffer loads (qr: the query rows of every slot) rather
// than global ones: while a global load to LDS is in flight the compiler
// makes every LDS read wait for all earlier ones (it may be an LDS access of
// either kind), which would serialise the B reads of the MFMA loop.
template <int PREC, int KS>
__device__ __forceinline__ void stage_group(const GroupSlots& gs, int wave, int lane,
                                            __amdgpu_buffer_rsrc_t qr, u4v* dst) {
  constexpr int H = TileTraits<PREC>::kHalves;
  constexpr int kPieces = 2 * KS * H;
  constexpr int kRowUnits = PREC == 1 ? 2 * KS : 4 * KS;  // u4v per query row
  static_assert(kPieces % 4 == 0, "whole pieces per wave");
#pragma unroll
  for (int i = 0; i < kPieces / 4; i++) {
    const int piece = wave + 4 * i;
    const int cb = piece / (KS * H), rem = piece % (KS * H);
    const int ks = rem / H, hh = rem % H;
    const int slot = cb ? gs.s1 : gs.s0;
    const int u = PREC == 1 ? 2 * ks + (lane >> 5) : 4 * ks + 2 * (lane >> 5) + hh;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(qr, (__attribute__((address_space(3))) void*)(dst + piece * 64), 16,
                                             (slot * kRowUnits + u) * 16, 0, 0, 0);
  }
}

// chunk-level state shared by the group steps
struct ChunkState {
  int64_t c0, blk;
  int bit, wave, lane;
  float4 lmx;
  float lead, gam, sc;
  float xmin[2];
};

// max of the 16 accumulators of a lane's fragment, as a depth-3 tree
__device__ __forceinline__ float max16(const f16v& v) {
  auto mx3 = [](float x, float y, float z) { return fmaxf(fmaxf(x, y), z); };
  const float m0 = mx3(v[0], v[1], v[2]), m1 = mx3(v[3], v[4], v[5]), m2 = mx3(v[6], v[7], v[8]);
  const float m3 = mx3(v[9], v[10], v[11]), m4 = mx3(v[12], v[13], v[14]);
  return fmaxf(mx3(m0, m1, m2), mx3(m3, m4, v[15]));
}

// epilogue of one 32-query column block: D[i][j] with j = lane%32 (query),
// i = 8(e/4) + 4(lane/32) + e%4 (row of the row block r)
template <int PREC, bool DUMP>
__device__ __forceinline__ void col_epilogue(const SearchArgs& a, const Bf16Args& b, const ChunkState& cs,
                                             const float* xn2s, int slot, int q, float cq, bool mbit,
                                             float f, const f16v& acc0, const f16v& acc1) {
  const int wave = cs.wave, lane = cs.lane;
  if (DUMP) {
    // inspection: the lower bound t - o of every pair
    const float4 qm = b.qmeta[slot];
    const float o = -qm.x + 2.0f * (cs.gam * qm.z + qm.y) * cs.lmx.x + 2.0f * qm.w * cs.lmx.y +
                    (qm.x + cs.lmx.z) * 0x1p-20f;
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const int ri = 64 * wave + 32 * r + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
        const float t = fmaf(-f, r ? acc1[e] : acc0[e], xn2s[ri]);
        if (cs.c0 + ri < a.N && q >= 0) b.dump[(int64_t)q * a.N + cs.c0 + ri] = t - o;
      }
    return;
  }
  const bool any = fmaf(-f, max16(acc0), cs.xmin[0]) <= cq || fmaf(-f, max16(acc1), cs.xmin[1]) <= cq;
  if (!__ballot(mbit && any)) return;
  // rare: exact per-pair test and one append atomic per lane
  uint32_t hits[2];
#pragma unroll
  for (int r = 0; r < 2; r++) {
    uint32_t h = 0;
#pragma unroll
    for (int e = 0; e < 16; e++) {
      const int ri = 64 * wave + 32 * r + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
      h |= fmaf(-f, r ? acc1[e] : acc0[e], xn2s[ri]) <= cq ? (1u << e) : 0u;
    }
    hits[r] = h;
  }
  const uint32_t nh = mbit ? (uint32_t)(__popc(hits[0]) + __popc(hits[1])) : 0u;
  if (nh) {
    uint32_t slot = atomicAdd(b.ccnt + q, nh);
    bool dropped = false;
#pragma unroll
    for (int r = 0; r < 2; r++) {
      uint32_t h = hits[r];
      while (h) {
        const int e = __builtin_ctz(h);
        h &= h - 1;
        const int ri = 64 * wave + 32 * r + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
        if (slot < (uint32_t)b.cap)
          b.cand[(int64_t)q * b.cap + slot] = (uint32_t)(cs.c0 + ri);
        else
          dropped = true;
        slot++;
      }
    }
    // a dropped candidate: the query is finished exhaustively
    if (dropped && b.cevmin[q] != 0u) atomicMin(b.cevmin + q, 0u);
  }
}

// chunk of work item it (slices consecutive items share a chunk); skip > 0
// enumerates the chunks that are not multiples of skip
__device__ __forceinline__ int64_t item_chunk(const Bf16Args& b, uint32_t it) {
  const int64_t c = (int64_t)(it / (uint32_t)b.slices);
  return b.chunk_mult * (b.skip > 0 ? (c / (b.skip - 1)) * b.skip + c % (b.skip - 1) + 1
                                    : c * b.chunk_stride + b.chunk_first);
}

// A operand of one wave: row blocks rb and rb + 1 (32 rows each), all K
// steps.  The rows stream through once per pass: non-temporal loads keep
// them from evicting the query rows the B gathers reuse.
template <int PREC>
__device__ __forceinline__ typename TileTraits<PREC>::frag load_frag_nt(const u4v* p) {
  if constexpr (PREC == 1) {
    return __builtin_bit_cast(bf8v, __builtin_nontemporal_load(p));
  } else {
    const u4v lo = __builtin_nontemporal_load(p), hi = __builtin_nontemporal_load(p + 64);
    return __builtin_bit_cast(v8i, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
  }
}

template <int PREC, int KS>
__device__ __forceinline__ void load_a(const u4v* xv, int64_t rb, int lane,
                                       typename TileTraits<PREC>::frag (&av)[2][KS]) {
  constexpr int H = TileTraits<PREC>::kHalves;
#pragma unroll
  for (int r = 0; r < 2; r++)
#pragma unroll
    for (int ks = 0; ks < KS; ks++) av[r][ks] = load_frag_nt<PREC>(xv + ((rb + r) * KS + ks) * 64 * H + lane);
}

// raw buffer descriptor (fourth word for gfx9 raw, untyped access) over
// bytes [base, base + bytes); reads past the end return zero
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
}

// fragment at byte offset voff + soff of a buffer (the halves of an FP8
// fragment 1 KB apart, as in load_frag)
template <int PREC>
__device__ __forceinline__ typename TileTraits<PREC>::frag load_frag_buf(__amdgpu_buffer_rsrc_t r, int voff,
                                                                         int soff) {
  // cache policy 2: non-temporal (streamed once)
  if constexpr (PREC == 1) {
    return __builtin_bit_cast(bf8v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 2));
  } else {
    const u4v lo = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 2);
    const u4v hi = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + 1024, 2);
    return __builtin_bit_cast(v8i, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
  }
}

// the MFMAs of one 32-query column block over the wave's two row blocks.  B
// fragments are read from LDS two K steps ahead of their MFMAs (one for the
// widest FP8 rows, which leave too few registers); the scheduling barriers
// keep the compiler from sinking the reads back to their use.  RELOAD: each
// A fragment is replaced from buffer ra (the next chunk's two row blocks) as
// soon as its two MFMAs have issued, so the next chunk's HBM reads overlap
// this block's matrix work in the registers they will occupy.
template <int PREC, int KS, bool RELOAD>
__device__ __forceinline__ void col_mfma(typename TileTraits<PREC>::frag (&av)[2][KS], const u4v* bcol,
                                         __amdgpu_buffer_rsrc_t ra, int lane, f16v& acc0, f16v& acc1) {
  constexpr int H = TileTraits<PREC>::kHalves;
  constexpr int kAhead = (PREC == 2 && KS >= 8) ? 1 : 2;
  constexpr int kBlockBytes = KS * 64 * H * 16;
#pragma unroll
  for (int e = 0; e < 16; e++) acc0[e] = acc1[e] = 0.0f;
  typename TileTraits<PREC>::frag bq[KS];
#pragma unroll
  for (int ks = 0; ks < kAhead && ks < KS; ks++) bq[ks] = load_frag<PREC>(bcol + ks * 64 * H + lane);
#pragma unroll
  for (int ks = 0; ks < KS; ks++) {
    if (ks + kAhead < KS) bq[ks + kAhead] = load_frag<PREC>(bcol + (ks + kAhead) * 64 * H + lane);
    __builtin_amdgcn_sched_barrier(0);
    acc0 = mma<PREC>(av[0][ks], bq[ks], acc0);
    acc1 = mma<PREC>(av[1][ks], bq[ks], acc1);
    if (RELOAD) {
      av[0][ks] = load_frag_buf<PREC>(ra, lane * 16, ks * 64 * H * 16);
      av[1][ks] = load_frag_buf<PREC>(ra, lane * 16, kBlockBytes + ks * 64 * H * 16);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// one group: thresholds from the terms loaded one group ahead, the DMA and
// terms of the next group (when there is one), the slots of the group after
// it, the two column blocks one after the other, and the barrier that
// publishes the next buffer.  LAST (the chunk's last group): column block 1
// runs first, then block 0, which always runs (its lane 0 is a listed entry)
// and reloads the A registers from ra, the next chunk's rows (an empty
// buffer when there is none: the loads return zero).
template <int PREC, int KS, bool DUMP, bool LAST>
__device__ __forceinline__ void group_step(const SearchArgs& a, const Bf16Args& b,
                                           const ChunkState& cs,
                                           typename TileTraits<PREC>::frag (&av)[2][KS],
                                           const float* xn2s, const GroupSlots& gcur, const GroupSlots& gnext,
                                           bool has_next2, GroupSlots& gnext2, int64_t off, uint32_t cnt,
                                           int g2, ColTerms& cols, const u4v* cur, u4v* nxt,
                                           __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t qr,
                                           unsigned long long& st_pairs) {
  constexpr int H = TileTraits<PREC>::kHalves;
  const int wave = cs.wave, lane = cs.lane;
  const int q0 = cols.v0 ? __float_as_int(cols.c0.w) : -1;
  const int q1 = cols.v1 ? __float_as_int(cols.c1.w) : -1;
  const float cq0 = cols.c0.x + cols.c0.y * cs.lmx.x + cols.c0.z * cs.lmx.y + cs.lead;
  const float cq1 = cols.c1.x + cols.c1.y * cs.lmx.x + cols.c1.z * cs.lmx.y + cs.lead;
  // every listed query needs the leaf
  const bool mb0 = q0 >= 0, mb1 = q1 >= 0;
  const float f0 = PREC == 1 ? 2.0f : 2.0f * cs.sc * cols.s0;
  const float f1 = PREC == 1 ? 2.0f : 2.0f * cs.sc * cols.s1;
  if (!LAST) {
    stage_group<PREC, KS>(gnext, wave, lane, qr, nxt);
    load_cols<PREC>(b, gnext, cols);
    if (has_next2) gnext2 = group_slots(b, off, cnt, g2, lane);
  }
  const bool act0 = LAST || DUMP || __ballot(mb0), act1 = DUMP || __ballot(mb1);
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const int cb = LAST ? 1 - i : i;
    if (!(cb ? act1 : act0)) continue;
    st_pairs += 64 * 32;
    f16v acc[2];
    const u4v* bcol = cur + cb * KS * 64 * H;
    if (LAST && cb == 0)
      col_mfma<PREC, KS, true>(av, bcol, ra, lane, acc[0], acc[1]);
    else
      col_mfma<PREC, KS, false>(av, bcol, ra, lane, acc[0], acc[1]);
    col_epilogue<PREC, DUMP>(a, b, cs, xn2s, cb ? gcur.s1 : gcur.s0, cb ? q1 : q0, cb ? cq1 : cq0,
                             cb ? mb1 : mb0, cb ? f1 : f0, acc[0], acc[1]);
  }
  // the next group's fragments and terms have landed (LAST: the reload of A
  // may still be in flight); every wave is done with cur
  if (!LAST) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __syncthreads();
}

template <int PREC, int KS, bool DUMP, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, WAVES)))
void k_bf16_tiles(SearchArgs a, Bf16Args b) {
  typedef typename TileTraits<PREC>::frag frag;
  __shared__ __attribute__((aligned(16))) u4v Bs0[group_units<PREC, KS>()];
  __shared__ __attribute__((aligned(16))) u4v Bs1[group_units<PREC, KS>()];
  __shared__ float xn2s[256];
  __shared__ uint32_t item_sh;
  ChunkState cs;
  // uniform within the wave: the branches on the reload row block stay scalar
  cs.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  cs.lane = threadIdx.x & 63;
  cs.gam = (float)(KS * TileTraits<PREC>::kStep + TileTraits<PREC>::kStep) * 0x1p-23f;
  const int wave = cs.wave, lane = cs.lane;
  const u4v* xv = reinterpret_cast<const u4v*>(b.xb);
  // the query rows of every slot (G groups of 64), as a buffer for the gathers
  constexpr int kQRowBytes = (PREC == 1 ? 2 * KS : 4 * KS) * 16;
  const __amdgpu_buffer_rsrc_t qr = raw_rsrc(b.qb, b.G * kGroup * kQRowBytes);
  unsigned long long st_pairs = 0, st_needed = 0, st_rows = 0;
  // work items are fetched one ahead, so that a chunk's last group can load
  // the next chunk's A operand; thread 0 writes item_sh between the barriers
  // that separate it from every thread's reads
  uint32_t it_next = 0;
  if (threadIdx.x == 0) item_sh = atomicAdd(b.counter, 1u);
  __syncthreads();
  it_next = __builtin_amdgcn_readfirstlane(item_sh);
  int64_t a_chunk = -1;  // the chunk whose A operand av holds (or is loading)
  frag av[2][KS];
  for (;;) {
    const uint32_t it = it_next;
    if ((int64_t)it >= b.n_items) break;
    __syncthreads();
    if (threadIdx.x == 0) item_sh = atomicAdd(b.counter, 1u);
    __syncthreads();
    it_next = __builtin_amdgcn_readfirstlane(item_sh);
    const int64_t chunk = item_chunk(b, it);
    cs.c0 = chunk * 256;
    const int64_t leaf = cs.c0 / a.L;
    cs.blk = leaf / kLeavesPerItem;
    cs.bit = (int)(leaf % kLeavesPerItem);
    // the queries whose (query, leaf) pair survives, in groups of 64
    const uint32_t cnt = b.lcnt[leaf];
    const int64_t off = b.loff[leaf];
    const int ng_all = (int)((cnt + kGroup - 1) / kGroup);
    // this item's share [g0, g1) of the chunk's groups
    const int slice = (int)(it % (uint32_t)b.slices);
    const int g0 = (int)((int64_t)slice * ng_all / b.slices);
    const int g1 = (int)((int64_t)(slice + 1) * ng_all / b.slices);
    if (g1 == g0) continue;  // uniform across the workgroup
    {
      const uint32_t e0 = (uint32_t)g0 * kGroup, e1 = (uint32_t)g1 * kGroup < cnt ? (uint32_t)g1 * kGroup : cnt;
      const unsigned long long rows = (unsigned long long)(a.N - cs.c0 < 256 ? a.N - cs.c0 : 256);
      st_needed += (unsigned long long)(e1 - e0) * rows;
      if (g0 == 0) st_rows += rows;  // the chunk's rows are streamed once per pass
    }
    GroupSlots gcur = group_slots(b, off, cnt, g0, lane);
    ColTerms cols;
    stage_group<PREC, KS>(gcur, wave, lane, qr, Bs0);
    load_cols<PREC>(b, gcur, cols);
    GroupSlots gnext = gcur;
    if (g1 - g0 > 1) gnext = group_slots(b, off, cnt, g0 + 1, lane);
    // A operand: this wave's 64 rows, all K steps, in registers (already
    // loading when the previous chunk's last group reloaded them)
    if (a_chunk != chunk) load_a<PREC, KS>(xv, (cs.c0 + 64 * wave) / 32, lane, av);
    {
      // rows past N (zero in the copy) get a NaN |x|^2: no compare passes
      const int64_t row = cs.c0 + threadIdx.x;
      xn2s[threadIdx.x] = row < a.N ? b.meta[row].x : __builtin_nanf("");
    }
    cs.lmx = b.leafmeta[leaf];
    cs.lead = cs.lmx.z * 0x1p-20f;
    cs.sc = PREC == 2 ? b.cscale[chunk] : 1.0f;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the first group's fragments
    __syncthreads();
    // the next chunk's rows for the last group's reload of A
    const bool has_following = (int64_t)it_next < b.n_items;
    const int64_t next_chunk = has_following ? item_chunk(b, it_next) : (int64_t)0;
    constexpr int kABytes = 2 * KS * 64 * TileTraits<PREC>::kHalves * 16;
    const __amdgpu_buffer_rsrc_t ra =
        raw_rsrc(xv + (next_chunk * 256 + 64 * wave) / 32 * (kABytes / 32), has_following ? kABytes : 0);
    // smallest |x|^2 over the 16 rows of this lane's fragment, per row block
#pragma unroll
    for (int r = 0; r < 2; r++) {
      float m = INFINITY;  // NaN rows are skipped; all-NaN leaves +inf (a superset)
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const float v = xn2s[64 * wave + 32 * r + 8 * (e / 4) + 4 * (lane / 32) + (e % 4)];
        m = v < m ? v : m;
      }
      cs.xmin[r] = m;
    }
    // groups alternate between the two buffers (the item's first in Bs0)
    for (int g = g0; g + 1 < g1; g++) {
      GroupSlots gnext2 = gnext;
      const bool odd = (g - g0) & 1;
      group_step<PREC, KS, DUMP, false>(a, b, cs, av, xn2s, gcur, gnext, g + 2 < g1, gnext2, off, cnt, g + 2,
                                        cols, odd ? Bs1 : Bs0, odd ? Bs0 : Bs1, ra, qr, st_pairs);
      gcur = gnext;
      gnext = gnext2;
    }
    {
      const bool odd = (g1 - 1 - g0) & 1;
      GroupSlots unused = gnext;
      group_step<PREC, KS, DUMP, true>(a, b, cs, av, xn2s, gcur, gnext, false, unused, off, cnt, 0, cols,
                                       odd ? Bs1 : Bs0, odd ? Bs0 : Bs1, ra, qr, st_pairs);
    }
    a_chunk = has_following ? next_chunk : (int64_t)-1;
  }
  if (lane == 0 && st_pairs && a.stats) atomicAdd(a.stats + 3, st_pairs);
  if (threadIdx.x == 0 && st_needed && a.stats) atomicAdd(a.stats + 5, st_needed);
  if (threadIdx.x == 0 && st_rows && a.stats) atomicAdd(a.stats + 6, st_rows);
}

// waves per SIMD of the tile kernel: the two waves of a SIMD hide each
// other's epilogues and LDS waits (one wave running both column blocks of a
// group together, with 512 registers, measured slower on 10M x 256)
constexpr int kTileWaves = 2;

// launch over the supported (precision, K steps) pairs.  FP8 rows of 1024
// values: the A operand alone takes 256 VGPRs and the two B buffers 128 KB
// of LDS, so one workgroup per CU, one wave per SIMD (512 registers).
template <bool DUMP>
static sofa_status launch_tiles(const SearchArgs& a, const Bf16Args& b, unsigned grid, hipStream_t st) {
#define SOFA_TILE(P, K) k_bf16_tiles<P, K, DUMP, kTileWaves><<<grid, 256, 0, st>>>(a, b)
  if (b.prec == 1) {
    switch (a.n_pad / 16) {
      case 4: SOFA_TILE(1, 4); break;
      case 8: SOFA_TILE(1, 8); break;
      case 16: SOFA_TILE(1, 16); break;
      default: return set_error(SOFA_EINVAL, "the BF16 prune supports n <= 256 (padded %d)", a.n_pad);
    }
  } else if (b.prec == 2) {
    switch (a.n_pad / 64) {
      case 1: SOFA_TILE(2, 1); break;
      case 2: SOFA_TILE(2, 2); break;
      case 4: SOFA_TILE(2, 4); break;
      case 8: SOFA_TILE(2, 8); break;
      case 16: k_bf16_tiles<2, 16, DUMP, 1><<<grid < 256u ? grid : 256u, 256, 0, st>>>(a, b); break;
      default: return set_error(SOFA_EINVAL, "the FP8 prune supports n <= 1024 (padded %d)", a.n_pad);
    }
  } else {
    return set_error(SOFA_EINVAL, "unknown prune precision %d", b.prec);
  }
#undef SOFA_TILE
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// ----------------------------------------------------------------------------
// exact FP32 refinement of the candidate lists: workgroup (q, z) of a
// (B x kCandSplit) grid; wave w takes 64-candidate chunks z*4+w, +4*kCandSplit, ...
constexpr int kCandSplit = 8;
template <int NIT, int R>
__global__ __launch_bounds__(256) void k_refine_cand(SearchArgs a, Bf16Args b) {
  constexpr int kStep = 4 * kRefRows;  // candidates per step of a wave
  const int q = blockIdx.x, z = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const uint32_t cnt_all = b.ccnt[q];
  const uint32_t cnt = cnt_all < (uint32_t)b.cap ? cnt_all : (uint32_t)b.cap;
  if (z == 0 && threadIdx.x == 0 && a.stats) atomicMax(a.stats + 4, (unsigned long long)cnt_all);
  if ((uint32_t)(z * 4 + wave) * 64 >= cnt) return;
  float4 qr[NIT];
  load_q<NIT>(a.Qp + (int64_t)q * a.n_pad, li, qr);
  float Umin = __uint_as_float(__atomic_load_n(a.U + q, __ATOMIC_RELAXED));
  float Upub = Umin;
  WaveList<R> wl;
  wl.reset();
  unsigned long long st_refined = 0;
  for (uint32_t ch = z * 4 + wave; ch * 64 < cnt; ch += 4 * kCandSplit) {
    const uint32_t idx = ch * 64 + lane;
    uint32_t pos = idx < cnt ? b.cand[(int64_t)q * b.cap + idx] : 0u;
    const bool valid = idx < cnt && (int64_t)pos < a.N;
    pos = valid ? pos : 0u;
    uint64_t bal = __ballot(valid);
    st_refined += (unsigned long long)__popcll(bal);
    const float ug = __uint_as_float(__atomic_load_n(a.U + q, __ATOMIC_RELAXED));
    Umin = ug < Umin ? ug : Umin;
    while (bal) {
      // the next kStep candidates in lane order: the t-th goes to group t % 4,
      // row t / 4 (-1: none)
      int c[kStep];
#pragma unroll
      for (int t = 0; t < kStep; t++) {
        c[t] = bal ? __builtin_ctzll(bal) : -1;
        bal = bal ? (bal & (bal - 1)) : 0ull;
      }
      int cm[kRefRows];
      uint32_t pm[kRefRows];
      bool am[kRefRows];
#pragma unroll
      for (int r = 0; r < kRefRows; r++) {
        const int t0 = c[4 * r], t1 = c[4 * r + 1], t2 = c[4 * r + 2], t3 = c[4 * r + 3];
        cm[r] = g == 0 ? t0 : (g == 1 ? t1 : (g == 2 ? t2 : t3));
        am[r] = cm[r] >= 0;
        pm[r] = __shfl(pos, am[r] ? cm[r] : 0);
      }
      float d[kRefRows];
      dist_rows<NIT>(a.X, a.n_pad, pm, am, qr, li, Umin * a.abandon_f, d);
      float band = Umin * a.band_f;
      bool mine = false;
#pragma unroll
      for (int r = 0; r < kRefRows; r++) mine = mine || (am[r] && d[r] <= band);
      uint64_t ins = __ballot(li == 0 && mine);
      while (ins) {
        const int gl = __builtin_ctzll(ins);
        ins &= ins - 1;
#pragma unroll
        for (int r = 0; r < kRefRows; r++) {
          const float dr = __shfl(d[r], gl);
          const bool ar = __shfl((int)am[r], gl) != 0;
          const uint32_t pr = __shfl(pm[r], gl);
          if (ar && dr <= band) wl.insert(((uint64_t)__float_as_uint(dr) << 32) | pr, lane);
        }
        const uint64_t kth = wl.at(a.k - 1);
        if (kth != kEmpty) {
          const float uw = key_d(kth) * a.upd_f;
          if (uw < Umin) {
            Umin = uw;
            band = Umin * a.band_f;
          }
        }
      }
    }
    if (Umin < Upub) {
      if (lane == 0) atomicMin(a.U + q, __float_as_uint(Umin));
      Upub = Umin;
    }
  }
  flush_wave_list<R>(a, q, wl, Umin, lane);
  if (lane == 0 && st_refined && a.stats) atomicAdd(a.stats + 2, st_refined);
}

// ----------------------------------------------------------------------------
sofa_status launch_bf16_build(const float* X, int64_t N, int n_pad, int L, int64_t n_leaves,
                              uint4* xb, float4* meta, float4* leafmeta, hipStream_t st) {
  const int64_t nrb = ((N + 255) / 256) * 8;  // 32-row blocks, padded to whole 256-row chunks
  k_bf16_copy_meta<<<grid_blocks(nrb, 4), 256, 0, st>>>(X, N, n_pad, nrb, xb, meta);
  k_bf16_leafmeta<<<nblk(n_leaves, 4), 256, 0, st>>>(meta, N, L, n_leaves, leafmeta);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_fp8_build(const float* X, int64_t N, int n_pad, int L, int64_t n_leaves,
                             uint4* xf, float* cscale, float4* meta, float4* leafmeta, hipStream_t st) {
  const int64_t n_chunks = (N + 255) / 256;
  k_fp8_chunk_build<<<grid_blocks(n_chunks, 1), 256, 0, st>>>(X, N, n_pad, cscale, xf, meta);
  k_bf16_leafmeta<<<nblk(n_leaves, 4), 256, 0, st>>>(meta, N, L, n_leaves, leafmeta);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// slot-order masks, then per leaf the slots of the queries that need it:
// count, offsets, fill
// slot_masks: the slot-order masks are already in b.smask
static void launch_lists(const SearchArgs& a, const Bf16Args& b, hipStream_t st, bool slot_masks = false) {
  const int Spad = b.G * kGroup;
  const int64_t n_sub = a.n_blocks * kSubPerBlock;
  if (!slot_masks)
    k_smask<<<grid_blocks(a.n_blocks * Spad, 256), 256, 0, st>>>(a.masks, a.n_blocks, a.B, Spad, b.perm, b.smask);
  k_leaf_lists<0><<<(unsigned)n_sub, 256, 0, st>>>(b.smask, a.n_leaves, Spad, b.lcnt, b.bsum, nullptr, nullptr,
                                                   nullptr);
  k_scan_counts<<<1, 1024, 0, st>>>(b.bsum, n_sub, b.boff);
  k_leaf_lists<1><<<(unsigned)n_sub, 256, 0, st>>>(b.smask, a.n_leaves, Spad, b.lcnt, nullptr, b.boff, b.loff,
                                                   b.lslot);
}

sofa_status launch_bf16_relist(const SearchArgs& a, const Bf16Args& b, hipStream_t st) {
  // the masks from the tightened U, straight into slot order (the first
  // masks counted the visited leaves; the query-order masks are not read again)
  SOFA_TRY(launch_slot_masks(a, b.G * kGroup, b.perm, b.smask, st));
  launch_lists(a, b, st, true);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_bf16_queries(const SearchArgs& a, Bf16Args& b, hipStream_t st) {
  const int B = a.B;
  SOFA_TRY(launch_fill_u32(b.qcount, 0u, B, st));
  {
    const int64_t sl = a.n_blocks < 64 ? a.n_blocks : 64;
    dim3 grid(nblk(B, 256), (unsigned)(sl > 0 ? sl : 1));
    k_qcount<<<grid, 256, 0, st>>>(a.masks, a.n_blocks, B, b.qcount);
  }
  k_qsort<<<nblk(B, 4), 256, 0, st>>>(b.qcount, a.best, B, a.n_leaves, b.perm);
  const int Spad = b.G * kGroup;
  launch_lists(a, b, st);
  if (b.prec == 2) {
    k_qscale_fp8<<<nblk(Spad, 4), 256, 0, st>>>(a.Qp, B, a.n_pad, b.perm, Spad, b.qscale);
    k_qrows_fp8<<<nblk((int64_t)Spad * (a.n_pad / 16), 256), 256, 0, st>>>(a.Qp, B, a.n_pad, Spad, b.perm,
                                                                          b.qscale, b.qb);
    k_qmeta_fp8<<<nblk(Spad, 4), 256, 0, st>>>(a.Qp, B, a.n_pad, b.perm, Spad, b.qscale, b.qmeta);
  } else {
    k_qrows_bf16<<<nblk((int64_t)Spad * (a.n_pad / 8), 256), 256, 0, st>>>(a.Qp, B, a.n_pad, Spad, b.perm,
                                                                          b.qb);
    k_qmeta_bf16<<<nblk(Spad, 4), 256, 0, st>>>(a.Qp, B, a.n_pad, b.perm, Spad, b.qmeta);
  }
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// accumulation bound g = (K + K step) 2^-23 of the FP32 MFMA sums
static float prune_gamma(const SearchArgs& a, const Bf16Args& b) {
  const int step = b.prec == 2 ? 64 : 16;
  return (float)(a.n_pad + step) * 0x1p-23f;
}

// the bound terms of every slot from the current U; the candidate counts
// (when `clear_ccnt`) and the work counter cleared in the same launch
static sofa_status launch_slotc(const SearchArgs& a, const Bf16Args& b, bool clear_ccnt, hipStream_t st) {
  const int Spad = b.G * kGroup;  // >= B
  k_slotc<<<nblk(Spad, 256), 256, 0, st>>>(b.qmeta, b.perm, a.B, Spad, a.U, a.lb_f, prune_gamma(a, b),
                                           b.slotc, clear_ccnt ? b.ccnt : nullptr, b.counter);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_bf16_dump(const SearchArgs& a, Bf16Args b, float* d_lb, hipStream_t st) {
  b.dump = d_lb;
  b.skip = 0;
  b.chunk_mult = 1;
  b.chunk_first = 0;
  b.chunk_stride = 1;
  b.slices = 1;
  b.n_items = (a.N + 255) / 256;
  SOFA_TRY(launch_slotc(a, b, false, st));
  unsigned grid = 256 * kTileWaves;
  if ((int64_t)grid > b.n_items) grid = (unsigned)b.n_items;
  return launch_tiles<true>(a, b, grid, st);
}

sofa_status launch_bf16_pass(const SearchArgs& a, Bf16Args b, int64_t mult, int64_t first,
                             int64_t stride, int64_t n_items, int skip, hipStream_t st,
                             hipEvent_t* ev) {
  b.chunk_mult = mult;
  b.chunk_first = first;
  b.chunk_stride = stride;
  b.skip = skip;
  // a pass of few chunks (the coarse sampled passes) splits each chunk's
  // query groups over several work items, so that it fills the grid
  unsigned grid = 256 * kTileWaves;
  b.slices = 1;
  while (b.slices < 16 && n_items * b.slices < 2 * (int64_t)grid) b.slices *= 2;
  b.n_items = n_items * b.slices;
  if (n_items <= 0) {
    // keep the pass's timers valid (zero length)
    if (ev)
      for (int i = 0; i < 3; i++) (void)hipEventRecord(ev[i], st);
    return SOFA_OK;
  }
  // the bounds U of this pass (earlier passes tighten them), cleared counts
  SOFA_TRY(launch_slotc(a, b, true, st));
  if ((int64_t)grid > b.n_items) grid = (unsigned)b.n_items;
  if (ev) (void)hipEventRecord(ev[0], st);
  SOFA_TRY(launch_tiles<false>(a, b, grid, st));
  if (ev) (void)hipEventRecord(ev[1], st);
  dim3 gr((unsigned)a.B, kCandSplit);
  const int R = (a.k + 16 <= 64) ? 1 : 2;
#define SOFA_RC(NI)                                                     \
  case NI:                                                              \
    if (R == 1) k_refine_cand<NI, 1><<<gr, 256, 0, st>>>(a, b);         \
    else k_refine_cand<NI, 2><<<gr, 256, 0, st>>>(a, b);                \
    break;
  switch (a.n_pad / 64) {
    SOFA_RC(1)
    SOFA_RC(2)
    SOFA_RC(4)
    SOFA_RC(8)
    SOFA_RC(16)
    default: return set_error(SOFA_EINVAL, "the batched-distance prune supports n <= 1024");
  }
#undef SOFA_RC
  if (ev) (void)hipEventRecord(ev[2], st);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

}  // namespace sofa
