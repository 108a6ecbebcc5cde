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
// one contiguous 1 KB read.  The tile kernel (k_tiles.hip) gives a
// workgroup 256 rows (4 waves x 64 rows, operand held in registers) and loops
// over the 64-query groups that have a surviving (query, leaf) pair; each
// group's BF16 query fragments are staged in LDS.  Queries are ordered by
// their number of surviving leaves, so that queries the SFA bound cannot
// prune share groups.  This file builds the copies and their bound terms,
// the query side, the per-leaf lists, and refines the kept rows.
#include "bf16.h"

namespace sofa {

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

// Per leaf, the sorted slots of the queries whose (query, leaf) pair
// survives, in one launch: workgroup g takes the 16 leaves of a sub-block (a
// quarter of a 64-leaf block).  It stages each slot's 16 survivor bits in
// LDS (kListPiece slots at a time) and fills each leaf's list in slot order
// (wave w takes leaves 4w .. 4w + 3).  Leaf l's list starts at l * B in
// lslot, which holds B entries per leaf (every query may need every leaf),
// so no count or offset pass precedes the fill.  FROM_CODES: the bits come
// from the stored FP16 bound codes under the current U (as block_mask);
// else from the query-order masks, through perm.
constexpr int kSubLeaves = 16;
constexpr int kSubPerBlock = kLeavesPerItem / kSubLeaves;
static_assert(kSubPerBlock == 4, "k_lists numbers the workgroups of 8 blocks in groups of 32");
constexpr int kListPiece = 4096;

// kStageU slots per thread and round: their loads (the slot's query, then
// its bound and codes) are issued together rather than one chain per slot
constexpr int kStageU = 4;

// per slot, for the current pass: with t = |x|^2 - 2P, a row survives when
//   t <= a + b * max|xh| + c * max r_x + 2^-20 * max|x|^2   (leaf maxima)
// where a = U lb_f - |q|^2 (1 - 2^-20), b = 2 (g |qh| + r_q), c = 2 |q|; .w = query id.
// With ccnt (B entries) and the work counter given, they are cleared for the
// pass as well.
struct SlotTerms {
  const float4* qmeta;
  const int32_t* perm;
  int B, Spad;
  const uint32_t* U;
  float lb_f, gam;
  float4* slotc;     // null: nothing to do
  uint32_t* ccnt;    // nullable
  uint32_t* counter; // nullable
};

__device__ __forceinline__ void slot_terms(const SlotTerms& t, int s) {
  if (t.counter && s == 0) *t.counter = 0u;
  if (t.ccnt && s < t.B) t.ccnt[s] = 0u;
  if (s >= t.Spad) return;
  float4 c = make_float4(-INFINITY, 0.0f, 0.0f, __int_as_float(-1));
  if (s < t.B) {
    const int q = t.perm[s];
    const float4 qm = t.qmeta[s];
    const float u = __uint_as_float(t.U[q]);
    c = make_float4(u * t.lb_f - qm.x * (1.0f - 0x1p-20f), 2.0f * (t.gam * qm.z + qm.y), 2.0f * qm.w,
                    __int_as_float(q));
  }
  t.slotc[s] = c;
}

__global__ void k_slotc(SlotTerms t) { slot_terms(t, blockIdx.x * blockDim.x + threadIdx.x); }

template <bool FROM_CODES>
__device__ __forceinline__ void stage_sub_bits(const SearchArgs& a, const int32_t* __restrict__ perm,
                                               int64_t blk, int sub_in, uint32_t valid, int s0, int m,
                                               uint16_t* sm) {
  for (int i0 = 0; i0 < m; i0 += 256 * kStageU) {
    int q[kStageU];
#pragma unroll
    for (int u = 0; u < kStageU; u++) {
      const int s = s0 + i0 + 256 * u + (int)threadIdx.x;
      q[u] = (i0 + 256 * u + (int)threadIdx.x < m && s < a.B) ? perm[s] : -1;
    }
    uint32_t bits[kStageU];
    if (FROM_CODES) {
      uint32_t t[kStageU];
      uint4 v0[kStageU], v1[kStageU];
#pragma unroll
      for (int u = 0; u < kStageU; u++) {
        const int qq = q[u] >= 0 ? q[u] : 0;
        t[u] = u_code(a, qq);
        const uint4* src = reinterpret_cast<const uint4*>(a.lbh + (blk * a.B + qq) * kLeavesPerItem +
                                                          sub_in * kSubLeaves);
        v0[u] = src[0];
        v1[u] = src[1];
      }
#pragma unroll
      for (int u = 0; u < kStageU; u++) {
        const uint32_t w[8] = {v0[u].x, v0[u].y, v0[u].z, v0[u].w, v1[u].x, v1[u].y, v1[u].z, v1[u].w};
        uint32_t b = 0;
#pragma unroll
        for (int e = 0; e < 8; e++) {
          b |= (uint32_t)((w[e] & 0xFFFFu) <= t[u]) << (2 * e);
          b |= (uint32_t)((w[e] >> 16) <= t[u]) << (2 * e + 1);
        }
        bits[u] = q[u] >= 0 ? b : 0u;
      }
    } else {
#pragma unroll
      for (int u = 0; u < kStageU; u++) {
        const int qq = q[u] >= 0 ? q[u] : 0;
        const uint32_t b = (uint32_t)(a.masks[blk * a.B + qq] >> (sub_in * kSubLeaves)) & 0xFFFFu;
        bits[u] = q[u] >= 0 ? b : 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < kStageU; u++) {
      const int i = i0 + 256 * u + (int)threadIdx.x;
      if (i < m) sm[i] = (uint16_t)(bits[u] & valid);
    }
  }
}

// sp > 0: only the leaves of the chunks that a pass over the multiples of sp
// (not of prev, when prev > 0) takes get their lists; the others get none
// With terms.slotc given, the launch also writes the slot terms (and clears
// the counts) of the pass that follows: U does not change in between.
template <bool FROM_CODES>
__global__ __launch_bounds__(256) void k_lists(SearchArgs a, int Spad, const int32_t* __restrict__ perm,
                                               uint32_t* __restrict__ lcnt, int64_t* __restrict__ loff,
                                               uint16_t* __restrict__ lslot, int64_t sp, int64_t prev,
                                               SlotTerms terms) {
  __shared__ uint16_t sm[kListPiece];
  if (terms.slotc) {
    const int ns = terms.Spad > terms.B ? terms.Spad : terms.B;
    for (int s = blockIdx.x * 256 + (int)threadIdx.x; s < ns; s += gridDim.x * 256) slot_terms(terms, s);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // Workgroups go to the 8 XCDs round robin, and the four sub-blocks of a
  // block read the four quarters of the same 128-byte rows of codes: the
  // workgroups of 8 blocks are numbered so that a block's four land on one
  // XCD and share its L2 (a last group of m < 8 blocks numbers them m apart).
  const int64_t g = blockIdx.x, g8 = g / 32;
  const int m8 = (int)(a.n_blocks - g8 * 8 < 8 ? a.n_blocks - g8 * 8 : 8);
  const int r = (int)(g % 32);
  const int64_t blk = g8 * 8 + r % m8;
  const int sub_in = r / m8;
  const int64_t leaf0 = (blk * kSubPerBlock + sub_in) * kSubLeaves + 4 * wave;  // this wave's first leaf
  // leaves of the sub-block that exist
  const int64_t nl = a.n_leaves - (blk * kSubPerBlock + sub_in) * kSubLeaves;
  uint32_t valid = nl >= kSubLeaves ? 0xFFFFu : ((1u << (nl > 0 ? nl : 0)) - 1u);
  if (sp > 0) {
    // lane j < 16 tests leaf j of the sub-block: its L / 256 chunks
    const int64_t per = a.L / 256, c0 = ((blk * kSubPerBlock + sub_in) * kSubLeaves + lane) * per;
    bool need = false;
    if (lane < kSubLeaves)
      for (int64_t c = c0; c < c0 + per; c++) need = need || (c % sp == 0 && (prev <= 0 || c % prev != 0));
    valid &= (uint32_t)__ballot(need) & 0xFFFFu;
  }
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t c[4] = {0u, 0u, 0u, 0u};
  for (int s0 = 0; s0 < Spad; s0 += kListPiece) {
    const int m = Spad - s0 < kListPiece ? Spad - s0 : kListPiece;  // a multiple of 64
    if (s0) __syncthreads();  // the previous piece has been read
    stage_sub_bits<FROM_CODES>(a, perm, blk, sub_in, valid, s0, m, sm);
    __syncthreads();
    for (int t0 = 0; t0 < m; t0 += 64) {
      const uint32_t v = (uint32_t)sm[t0 + lane] >> (4 * wave);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const bool on = (v >> j) & 1u;
        const uint64_t bal = __ballot(on);
        if (on) lslot[(leaf0 + j) * a.B + c[j] + __popcll(bal & lt)] = (uint16_t)(s0 + t0 + lane);
        c[j] += (uint32_t)__popcll(bal);
      }
    }
  }
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (leaf0 + j < a.n_leaves) {
        lcnt[leaf0 + j] = c[j];
        loff[leaf0 + j] = (leaf0 + j) * a.B;
      }
}

// BF16 query side, a wave per sorted slot: the slot's BF16 row (n_pad values,
// zero past B; a lane's fragment of the 32x32x16 B operand is 16 contiguous
// bytes of it), its bound terms and, U being final once the seed has run,
// its slot terms for the first pass
__global__ __launch_bounds__(256) void k_qmeta_bf16(const float* __restrict__ Qp, int B, int n_pad,
                                                    const int32_t* __restrict__ perm, int Spad,
                                                    float4* __restrict__ qmeta, uint4* __restrict__ qb,
                                                    SlotTerms terms) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= Spad) return;
  const float* qr = s < B ? Qp + (int64_t)perm[s] * n_pad : nullptr;
  const int per = n_pad / 8;
  for (int c = lane; c < per; c += 64) {
    uint32_t w[4] = {0, 0, 0, 0};
    if (qr) {
      const float4 a = *reinterpret_cast<const float4*>(qr + 8 * c);
      const float4 b = *reinterpret_cast<const float4*>(qr + 8 * c + 4);
      w[0] = bf16_bits(a.x) | (bf16_bits(a.y) << 16);
      w[1] = bf16_bits(a.z) | (bf16_bits(a.w) << 16);
      w[2] = bf16_bits(b.x) | (bf16_bits(b.y) << 16);
      w[3] = bf16_bits(b.z) | (bf16_bits(b.w) << 16);
    }
    qb[(int64_t)s * per + c] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
  if (qr) norms_of(qr, n_pad, lane, m);
  // m = (|q|^2 down, r_q up, |qh| up); the bound also needs |q| (up)
  if (lane == 0) {
    m.w = __double2float_ru(sqrt((double)m.x) * (1.0 + 1e-7) + 1e-30);
    qmeta[s] = m;
    slot_terms(terms, s);  // reads the qmeta just written (same thread)
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
                                                   float4* __restrict__ qmeta, SlotTerms terms) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= Spad) return;
  float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
  if (s < B) norms_of_fp8(Qp + (int64_t)perm[s] * n_pad, n_pad, lane, qscale[s], m);
  if (lane == 0) {
    m.w = __double2float_ru(sqrt((double)m.x) * (1.0 + 1e-7) + 1e-30);
    qmeta[s] = m;
    slot_terms(terms, s);  // the first pass's slot terms (see k_qmeta_bf16)
  }
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
  if (z == 0 && threadIdx.x == 0) stat_max(a, 4, (unsigned long long)cnt_all);
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
  if (lane == 0) stat_add(a, 2, st_refined);
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

// per leaf, the slots of the queries that need it
// accumulation bound g = (K + K step) 2^-23 of the FP32 MFMA sums
static float prune_gamma(const SearchArgs& a, const Bf16Args& b) {
  const int step = b.prec == 2 ? 64 : 16;
  return (float)(a.n_pad + step) * 0x1p-23f;
}

// the slot terms of the current U; the candidate counts (when `clear_ccnt`)
// and the work counter cleared with them
static SlotTerms slot_terms_of(const SearchArgs& a, const Bf16Args& b, bool clear_ccnt) {
  SlotTerms t;
  t.qmeta = b.qmeta;
  t.perm = b.perm;
  t.B = a.B;
  t.Spad = b.G * kGroup;  // >= B
  t.U = a.U;
  t.lb_f = a.lb_f;
  t.gam = prune_gamma(a, b);
  t.slotc = b.slotc;
  t.ccnt = clear_ccnt ? b.ccnt : nullptr;
  t.counter = b.counter;
  return t;
}

template <bool FROM_CODES>
static void launch_lists(const SearchArgs& a, const Bf16Args& b, hipStream_t st, int64_t sp, int64_t prev,
                         const SlotTerms& terms) {
  const int64_t n_sub = a.n_blocks * kSubPerBlock;
  k_lists<FROM_CODES><<<(unsigned)n_sub, 256, 0, st>>>(a, b.G * kGroup, b.perm, b.lcnt, b.loff, b.lslot, sp,
                                                       prev, terms);
}

sofa_status launch_bf16_relist(const SearchArgs& a, const Bf16Args& b, int64_t sp, int64_t prev,
                               hipStream_t st) {
  // straight from the stored bound codes under the tightened U, in slot
  // order, with the next pass's slot terms
  launch_lists<true>(a, b, st, sp, prev, slot_terms_of(a, b, true));
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_bf16_queries(const SearchArgs& a, Bf16Args& b, hipStream_t st, bool clear_qcount) {
  const int B = a.B;
  if (clear_qcount) SOFA_TRY(launch_fill_u32(b.qcount, 0u, B, st));
  {
    const int64_t sl = a.n_blocks < 64 ? a.n_blocks : 64;
    dim3 grid(nblk(B, 256), (unsigned)(sl > 0 ? sl : 1));
    k_qcount<<<grid, 256, 0, st>>>(a.masks, a.n_blocks, B, b.qcount);
  }
  k_qsort<<<nblk(B, 4), 256, 0, st>>>(b.qcount, a.best, B, a.n_leaves, b.perm);
  const int Spad = b.G * kGroup;
  SlotTerms none{};
  launch_lists<false>(a, b, st, 0, 0, none);
  if (b.prec == 2) {
    k_qscale_fp8<<<nblk(Spad, 4), 256, 0, st>>>(a.Qp, B, a.n_pad, b.perm, Spad, b.qscale);
    k_qrows_fp8<<<nblk((int64_t)Spad * (a.n_pad / 16), 256), 256, 0, st>>>(a.Qp, B, a.n_pad, Spad, b.perm,
                                                                          b.qscale, b.qb);
    k_qmeta_fp8<<<nblk(Spad, 4), 256, 0, st>>>(a.Qp, B, a.n_pad, b.perm, Spad, b.qscale, b.qmeta,
                                               slot_terms_of(a, b, true));
  } else {
    k_qmeta_bf16<<<nblk(Spad, 4), 256, 0, st>>>(a.Qp, B, a.n_pad, b.perm, Spad, b.qmeta, b.qb,
                                                slot_terms_of(a, b, true));
  }
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// the bound terms of every slot from the current U; the candidate counts
// (when `clear_ccnt`) and the work counter cleared in the same launch
static sofa_status launch_slotc(const SearchArgs& a, const Bf16Args& b, bool clear_ccnt, hipStream_t st) {
  k_slotc<<<nblk(b.G * kGroup, 256), 256, 0, st>>>(slot_terms_of(a, b, clear_ccnt));
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
  return launch_bf16_tiles(a, b, grid, true, st);
}

sofa_status launch_bf16_pass(const SearchArgs& a, Bf16Args b, int64_t mult, int64_t first,
                             int64_t stride, int64_t n_items, int skip, bool terms_ready, hipStream_t st,
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
  // (already written when the lists were rebuilt just before)
  if (!terms_ready) SOFA_TRY(launch_slotc(a, b, true, st));
  if ((int64_t)grid > b.n_items) grid = (unsigned)b.n_items;
  if (ev) (void)hipEventRecord(ev[0], st);
  SOFA_TRY(launch_bf16_tiles(a, b, grid, false, st));
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
