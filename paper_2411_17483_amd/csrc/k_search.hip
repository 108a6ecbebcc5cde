// k_search.hip -- exact k-NN under the GEMINI filter-and-refine scheme with
// the SFA lower bound (Section II-A; Eq. 2 and Eq. 3; Section IV-C search).
//
// Per batch of B queries:
//  1. k_tables   per query: lower-bound table T[j][s] = w_j * mind_j(s, v_j)^2
//                (Eq. 3, widened by the projection error bounds, rounded down;
//                w = 2 for SFA, 1 for the iSAX summary of Section IV-D),
//                the query's own symbols, in HBM (16 KB per query).
//  2. k_leaf_lb  every (query, leaf): envelope bound sum_j T[j][clamp(s_q,lo,hi)]
//                (valid because each table row is unimodal with its zero at the
//                query's own symbol), computed once: it finds the best leaf
//                per query and keeps every bound as an FP16 code rounded
//                down; after the seed, k_leaf_mask turns the codes into a
//                64-leaf survivor mask per (leaf block, query).
//  3. k_seed     exact distances to the best leaf's rows (the approximate search
//                of Section IV-C) give the first best-so-far bound.
//  4. k_refine   persistent kernel over (leaf block, query) items, leaf-block
//                major so that concurrent queries share the same rows in L2:
//                table in LDS, word lower bounds (16-byte coalesced loads),
//                ballot compaction of the survivors, gathered FP32 distances
//                (16 lanes x float4 per row, chunked early abandoning), a
//                sorted per-wave candidate list in registers, atomicMin of the
//                bound, and a flush of the in-band candidates per item.
//  5. k_finalize per query: candidates inside the FP32 error band of the final
//                bound are recomputed in FP64 in time order (no contraction)
//                and ranked by (distance, row id).
//
// Rigour.  Every prune compares a quantity that can only be smaller than the
// exact squared distance against a bound U that can only be larger than the
// exact k-th squared distance D*:
//   U is +inf, a radius the caller vouches for (checked afterwards), or
//   K32 * (1 + 2 eps) where K32 is the k-th smallest FP32 distance seen by
//   one wave and eps bounds |d32 - d| / d.  Lower bounds are kept when
//   LB32 <= U * (1 + 2^-16) (the FP32 table sum overestimates by at most
//   ~20 ulp).  Distances are kept when d32 <= U * (1 + 3 eps), which contains
//   every series whose exact distance is <= U.  The final ranking uses FP64.
#include "search_dev.h"

namespace sofa {

static inline unsigned nblk(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

// ----------------------------------------------------------------------------
// 1. lower-bound tables
__global__ __launch_bounds__(256) void k_tables(const float* __restrict__ pool, int ld_pool,
                                                const double* __restrict__ qnorm2,
                                                const int* __restrict__ sel, int l,
                                                const float* __restrict__ beta32,
                                                double eta_x, double eta_per_norm, double weight,
                                                float* __restrict__ tables,
                                                uint4* __restrict__ sq) {
  __shared__ float v[16];
  __shared__ uint8_t sym[16];
  // the breakpoints, staged with every thread's loads in flight at once (the
  // binary search and the table read them from LDS)
  __shared__ float4 bs4[kTable / 4];
  const float* bs = reinterpret_cast<const float*>(bs4);
  const int q = blockIdx.x, t = threadIdx.x;
  const double eta_q = eta_per_norm * sqrt(qnorm2[q]) + 1e-30;
  {
    const float4* b4 = reinterpret_cast<const float4*>(beta32);
    const int nb4 = l * kAlphaMax / 4;
    float4 w[kTable / 4 / 256];
#pragma unroll
    for (int u = 0; u < kTable / 4 / 256; u++) w[u] = b4[u * 256 + t < nb4 ? u * 256 + t : 0];
    // entries past the l rows hold a repeat of the first (never read)
#pragma unroll
    for (int u = 0; u < kTable / 4 / 256; u++) bs4[u * 256 + t] = w[u];
  }
  const float vq = (t < l) ? pool[(int64_t)q * ld_pool + sel[t]] : 0.0f;
  __syncthreads();
  if (t < 16) {
    v[t] = vq;
    int s = 0;
    if (t < l) {
      const float* bj = bs + t * kAlphaMax;
      for (int step = 128; step > 0; step >>= 1)
        if (bj[s + step - 1] <= vq) s += step;
    }
    sym[t] = (uint8_t)s;
  }
  __syncthreads();
  if (t == 0) {
    uint32_t w[4] = {0, 0, 0, 0};
    for (int j = 0; j < 16; j++) w[j >> 2] |= (uint32_t)sym[j] << (8 * (j & 3));
    sq[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  const double eta = eta_x + eta_q;
  for (int i = t; i < kTable; i += 256) {
    int j = i / kAlphaMax, s = i % kAlphaMax;
    float out = 0.0f;
    if (j < l) {
      double vj = (double)v[j];
      double lo = (s == 0) ? -INFINITY : (double)bs[j * kAlphaMax + s - 1] - eta;
      double hi = (double)bs[j * kAlphaMax + s] + eta;  // +inf beyond alpha-1
      double gap = 0.0;
      if (lo - vj > gap) gap = lo - vj;
      if (vj - hi > gap) gap = vj - hi;
      double T = weight * gap * gap * (1.0 - 0x1p-40);
      out = __double2float_rd(T);
    }
    tables[(int64_t)q * kTable + i] = out;
  }
}

// 2. envelope bounds of every (query, leaf), computed once: the smallest
// (bound bits << 32 | leaf) per query goes to `best` (atomicMin) and every
// bound is kept as an FP16 code rounded down, from which k_leaf_mask makes
// the survivor masks once the seed has set U.
constexpr int kSegLeaves = 16384;  // leaves per workgroup: one 16 KB table load serves them all

__global__ __launch_bounds__(256) void k_leaf_lb(SearchArgs a) {
  __shared__ float T[kTable];
  const int q = blockIdx.y;
  const int64_t seg0 = (int64_t)blockIdx.x * kSegLeaves;
  const float4* src = reinterpret_cast<const float4*>(a.tables + (int64_t)q * kTable);
  for (int i = threadIdx.x; i < kTable / 4; i += 256) reinterpret_cast<float4*>(T)[i] = src[i];
  __syncthreads();
  const uint4 sq = a.sq[q];
  const int lane = threadIdx.x & 63;
  const int64_t last = a.n_leaves - 1;
  uint64_t best = kEmpty;
  // kU leaves per thread and iteration: their envelope loads are issued
  // together (a leaf past the end reads the last one; its bound is dropped)
  constexpr int kU = 4;
  for (int it = 0; it < kSegLeaves / 256; it += kU) {
    if (seg0 + (int64_t)it * 256 >= a.n_leaves) break;  // uniform over the workgroup
    uint4 lo[kU], hi[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int64_t leaf = seg0 + (it + u) * 256 + threadIdx.x;
      const uint4* e = reinterpret_cast<const uint4*>(a.env + (leaf < last ? leaf : last) * 32);
      lo[u] = e[0];
      hi[u] = e[1];
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int64_t leaf = seg0 + (it + u) * 256 + threadIdx.x;
      const bool valid = leaf < a.n_leaves;
      const float lb = lb_leaf(T, sq, lo[u], hi[u]);
      // computed for every leaf (a select, not a branch), so that the loads
      // stay ahead of the arithmetic
      const uint64_t key = valid ? ((uint64_t)__float_as_uint(lb) << 32) | (uint64_t)(uint32_t)leaf : kEmpty;
      best = key < best ? key : best;
      if (valid)
        a.lbh[((leaf / kLeavesPerItem) * a.B + q) * kLeavesPerItem + leaf % kLeavesPerItem] = f16_down(lb);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(best, off);
    best = o < best ? o : best;
  }
  if (lane == 0 && best != kEmpty) atomicMin(reinterpret_cast<unsigned long long*>(a.best) + q, best);
}

// the survivor mask of query q in 64-leaf block blk under the current U
__device__ __forceinline__ uint64_t block_mask(const SearchArgs& a, int64_t blk, int q) {
  const uint32_t t = u_code(a, q);
  const int64_t nl = a.n_leaves - blk * kLeavesPerItem;  // leaves of this block
  const uint64_t valid = nl >= kLeavesPerItem ? ~0ull : ((1ull << nl) - 1ull);
  const uint4* src = reinterpret_cast<const uint4*>(a.lbh + (blk * a.B + q) * kLeavesPerItem);
  uint4 v[8];
#pragma unroll
  for (int i = 0; i < 8; i++) v[i] = src[i];
  uint64_t m = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const uint32_t w[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int bit = 8 * i + 2 * e;
      m |= (uint64_t)((w[e] & 0xFFFFu) <= t) << bit;
      m |= (uint64_t)((w[e] >> 16) <= t) << (bit + 1);
    }
  }
  return m & valid;
}

// survivor masks per 64-leaf block from the stored bounds: a leaf survives
// when its bound is within U (with the slack of the FP32 bound sum).  The
// codes of non-negative values order like the values, so the test is an
// integer compare against the code of U rounded down.  Workgroup (blk, y):
// thread t takes query 256y + t, reads its 64 codes of the block (128
// contiguous bytes) and writes the block's mask (consecutive queries,
// consecutive words); one statistics atomic per workgroup.
__global__ __launch_bounds__(256) void k_leaf_mask(SearchArgs a) {
  __shared__ unsigned long long vis[4];
  const int64_t blk = blockIdx.x;
  const int q = blockIdx.y * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long visited = 0;
  if (q < a.B) {
    const uint64_t m = block_mask(a, blk, q);
    a.masks[blk * a.B + q] = m;
    visited = (unsigned long long)__popcll(m);
  }
  if (a.stats) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) visited += __shfl_xor(visited, o);
    if (lane == 0) vis[wave] = visited;
    __syncthreads();
    if (threadIdx.x == 0) {
      stat_add(a, 0, vis[0] + vis[1] + vis[2] + vis[3]);
    }
  }
}

// 3. seed: one workgroup per query scans the best leaf's rows, wave w taking
// the 16-row steps w, w + 4, ... with its own candidate list; the four lists'
// k smallest keys then give the k-th smallest key of the leaf (every key
// below it is among some wave's k smallest), so U is the same as one wave
// scanning the whole leaf would set.
static_assert(kMaxK + 16 <= 64 * 2, "a wave list of two registers per lane holds every k's keys");

template <int NIT, int R>
__global__ __launch_bounds__(256) void k_seed(SearchArgs a) {
  __shared__ uint64_t keys[4 * 64 * R];  // wave w's rank r at w * k + r
  __shared__ uint64_t kth_sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int q = blockIdx.x;
  const float U0 = a.U0[q];
  const uint64_t bestk = a.best[q];
  if (bestk == kEmpty || a.seed_leaf == 0) {
    if (threadIdx.x == 0) {
      a.U[q] = __float_as_uint(U0);
      a.hbase[q] = U0;
    }
    return;
  }
  const int64_t leaf = (int64_t)(uint32_t)bestk;
  const int64_t start = leaf * a.L, end = start + a.L < a.N ? start + a.L : a.N;
  float4 qr[NIT];
  load_q<NIT>(a.Qp + (int64_t)q * a.n_pad, li, qr);
  WaveList<R> wl;
  wl.reset();
  float Umin = U0;
  // 16 rows per step: row p0 + 4r + g in 16-lane group g, slot r
  for (int64_t p0 = start + 4 * kRefRows * wave; p0 < end; p0 += 16 * kRefRows) {
    uint32_t pm[kRefRows];
    bool am[kRefRows];
#pragma unroll
    for (int r = 0; r < kRefRows; r++) {
      const int64_t p = p0 + 4 * r + g;
      am[r] = p < end;
      pm[r] = (uint32_t)(am[r] ? p : start);
    }
    float d[kRefRows];
    dist_rows<NIT>(a.X, a.n_pad, pm, am, qr, li, Umin * a.abandon_f, d);
#pragma unroll
    for (int r = 0; r < kRefRows; r++)
#pragma unroll
      for (int gi = 0; gi < 4; gi++) {
        const int64_t p = p0 + 4 * r + gi;
        const float dd = __shfl(d[r], 16 * gi);
        if (p < end && dd <= Umin * a.band_f) {
          const uint64_t key = ((uint64_t)__float_as_uint(dd) << 32) | (uint64_t)p;
          wl.insert(key, lane);
        }
      }
    uint64_t kth = wl.at(a.k - 1);
    if (kth != kEmpty) {
      float uw = key_d(kth) * a.upd_f;
      Umin = uw < Umin ? uw : Umin;
    }
  }
  // the waves' k smallest keys (kEmpty past a short list)
#pragma unroll
  for (int r = 0; r < R; r++)
    if (64 * r + lane < a.k) keys[wave * a.k + 64 * r + lane] = wl.e[r];
  if (threadIdx.x == 0) kth_sh = kEmpty;
  __syncthreads();
  // the key with exactly k - 1 smaller keys among the 4k (keys are distinct:
  // they hold the row position)
  const int nk = 4 * a.k;
  for (int i = threadIdx.x; i < nk; i += 256) {
    const uint64_t ki = keys[i];
    if (ki == kEmpty) continue;
    int below = 0;
    for (int j = 0; j < nk; j++) below += keys[j] < ki ? 1 : 0;
    if (below == a.k - 1) kth_sh = ki;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float U = U0;
    if (kth_sh != kEmpty) {
      const float uw = key_d(kth_sh) * a.upd_f;
      U = uw < U ? uw : U;
    }
    a.U[q] = __float_as_uint(U);
    a.hbase[q] = U;
  }
}

// 4. refinement over (leaf sub-block, query) work items.  Workgroup w feeds
// from queue w % 8, and queue x holds the sub-blocks of the 64-leaf blocks
// b = x mod 8, query-minor: workgroups are dispatched to the 8 XCDs round
// robin, so the rows that concurrent queries share stay in one XCD's L2.
constexpr int kSub = 8;                        // leaves per work item
constexpr int kSubPerBlock = kLeavesPerItem / kSub;
constexpr int kQueues = 8;

// early-abandon check period of the plain path's distances, in 64-element
// steps.  Checking every 64 or 128 elements puts each row's later loads
// behind a 16-lane reduction and a compare, and measured slower on 10M x 256
// (3.5k and 4.0k against 4.2k queries/s) although most refined rows are far.
constexpr int kPlainCheck = 4;

template <int NIT, int R>
__global__ __launch_bounds__(256) void k_refine(SearchArgs a) {
  __shared__ float T[kTable];
  __shared__ uint32_t item_sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  unsigned long long st_words = 0, st_refined = 0;
  const int xq = blockIdx.x % kQueues;
  // blocks of this queue: b = xq, xq + 8, ...
  const int64_t nb_q = a.n_blocks > xq ? (a.n_blocks - xq + kQueues - 1) / kQueues : 0;
  const uint64_t total = (uint64_t)nb_q * kSubPerBlock * (uint64_t)a.B;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(a.counter + xq, 1u);
    __syncthreads();
    const uint64_t item = item_sh;
    __syncthreads();
    if (item >= total) break;
    const int q = (int)(item % (uint64_t)a.B);
    const uint64_t bs = item / (uint64_t)a.B;
    const int64_t blk = (int64_t)(bs / kSubPerBlock) * kQueues + xq;
    const int sub = (int)(bs % kSubPerBlock);
    const uint32_t mask = (uint32_t)(a.masks[blk * a.B + q] >> (kSub * sub)) & ((1u << kSub) - 1u);
    if (mask == 0u) continue;
    const float4* src = reinterpret_cast<const float4*>(a.tables + (int64_t)q * kTable);
    for (int i = threadIdx.x; i < kTable / 4; i += 256) reinterpret_cast<float4*>(T)[i] = src[i];
    const uint4 sq = a.sq[q];
    float4 qr[NIT];
    load_q<NIT>(a.Qp + (int64_t)q * a.n_pad, li, qr);
    __syncthreads();
    float Umin = __uint_as_float(__atomic_load_n(a.U + q, __ATOMIC_RELAXED));
    float Upub = Umin;
    WaveList<R> wl;
    wl.reset();
    int zc = 0;
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
      const int64_t leaf = blk * kLeavesPerItem + kSub * sub + __builtin_ctz(mm);
      const int64_t start = leaf * a.L, end = start + a.L < a.N ? start + a.L : a.N;
      const int nsl = (int)((end - start + 63) / 64);
      for (int s = 0; s < nsl; s++, zc++) {
        if ((zc & 3) != wave) continue;
        // current bound: the shared one and this wave's own
        const float ug = __uint_as_float(__atomic_load_n(a.U + q, __ATOMIC_RELAXED));
        Umin = ug < Umin ? ug : Umin;
        {
          const uint4* e = reinterpret_cast<const uint4*>(a.env + leaf * 32);
          if (lb_leaf(T, sq, e[0], e[1]) > Umin * a.lb_f) continue;
        }
        const int64_t base = start + 64 * s;
        const int64_t p = base + lane;
        const bool valid = p < end;
        uint4 w = valid ? *reinterpret_cast<const uint4*>(a.words + p * kWordBytes)
                        : make_uint4(0, 0, 0, 0);
        const float lb = lb_word(T, w);
        uint64_t bal = __ballot(valid && lb <= Umin * a.lb_f);
        st_words += (unsigned long long)__popcll(__ballot(valid));
        st_refined += (unsigned long long)__popcll(bal);
        while (bal) {
          // two groups of four candidates per pass: lane group g takes c0 and c1
          int c0[4], c1[4];
#pragma unroll
          for (int gi = 0; gi < 4; gi++) {
            c0[gi] = bal ? __builtin_ctzll(bal) : -1;
            bal = bal ? (bal & (bal - 1)) : 0ull;
          }
#pragma unroll
          for (int gi = 0; gi < 4; gi++) {
            c1[gi] = bal ? __builtin_ctzll(bal) : -1;
            bal = bal ? (bal & (bal - 1)) : 0ull;
          }
          const int ca = c0[g], cb = c1[g];
          const float abandon = Umin * a.abandon_f;
          float da = dist4<NIT, kPlainCheck>(a.X + (base + (ca >= 0 ? ca : 0)) * a.n_pad, ca >= 0, qr, li, abandon);
          float db = INFINITY;
          if (c1[0] >= 0)
            db = dist4<NIT, kPlainCheck>(a.X + (base + (cb >= 0 ? cb : 0)) * a.n_pad, cb >= 0, qr, li, abandon);
          float band = Umin * a.band_f;
          uint64_t ins = __ballot(li == 0 && ((ca >= 0 && da <= band) || (cb >= 0 && db <= band)));
          while (ins) {
            const int gl = __builtin_ctzll(ins);
            ins &= ins - 1;
            const int gg = gl >> 4;
            const float dA = __shfl(da, gl), dB = __shfl(db, gl);
            if (c0[gg] >= 0 && dA <= band)
              wl.insert(((uint64_t)__float_as_uint(dA) << 32) | (uint64_t)(base + c0[gg]), lane);
            if (c1[gg] >= 0 && dB <= band)
              wl.insert(((uint64_t)__float_as_uint(dB) << 32) | (uint64_t)(base + c1[gg]), lane);
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
    }
    flush_wave_list<R>(a, q, wl, Umin, lane);
    __syncthreads();
  }
  if (lane == 0) {
    stat_add(a, 1, st_words);
    stat_add(a, 2, st_refined);
  }
}

// 5. finalize: FP64 recomputation of the in-band candidates and ranking.
// The rows are staged in LDS a batch at a time, every thread's loads in
// flight together; then one thread per row sums its distance in dimension
// order.  (A thread reading its row from memory itself waits for one round
// trip per eight float4 loads.)
constexpr int kSMax = 1024;
constexpr int kFinStageFloats = 4096;  // staged row values per batch (16 KB)
static_assert(kFinStageFloats >= kMaxN, "at least one row per batch");

// exact_d2 over rows staged in LDS: the same operations in the same order,
// one float4 at a time (few registers: four workgroups fit on a SIMD set)
__device__ __forceinline__ double lds_d2(const float4* q, const float4* x, int n) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int i = 0; i < n / 4; i++) {
    const float4 a = q[i], b = x[i];
    const double d0 = (double)a.x - (double)b.x;
    const double s0 = d0 * d0;
    s = s + s0;
    const double d1 = (double)a.y - (double)b.y;
    const double s1 = d1 * d1;
    s = s + s1;
    const double d2 = (double)a.z - (double)b.z;
    const double s2 = d2 * d2;
    s = s + s2;
    const double d3 = (double)a.w - (double)b.w;
    const double s3 = d3 * d3;
    s = s + s3;
  }
  return s;
}

__global__ __launch_bounds__(256) void k_finalize(SearchArgs a, int64_t* __restrict__ out_ids,
                                                  float* __restrict__ out_d,
                                                  int32_t* __restrict__ status) {
  __shared__ uint32_t spos[kSMax];
  __shared__ double sd[kSMax];
  __shared__ int32_t sid[kSMax];
  __shared__ float4 sq4[kMaxN / 4];
  __shared__ float4 sx4[kFinStageFloats / 4 + kFinStageFloats / 64];  // rows padded by one float4
  __shared__ uint32_t scount;
  __shared__ int sstat;
  const int q = blockIdx.x, t = threadIdx.x;
  if (t == 0) {
    scount = 0;
    sstat = 0;
  }
  __syncthreads();
  const uint32_t cnt = a.rescnt[q];
  const float band = __uint_as_float(a.U[q]) * a.band_f;
  // exact unless a key inside the final band was ever evicted or dropped
  const uint64_t ev = a.evmin[q];
  // overflow reasons: 2 an evicted or dropped candidate lies in the final
  // band, 4 a BF16 candidate was dropped, 5 the band holds more than kSMax rows
  int ovf = (ev != kEmpty && key_d(ev) <= band) ? 2 : 0;
  if (a.cevmin && a.cevmin[q] != 0xFFFFFFFFu &&
      __uint_as_float(a.cevmin[q]) <= __uint_as_float(a.U[q]) * a.lb_f)
    ovf = 4;
  const uint32_t lim = cnt < (uint32_t)a.cap ? cnt : (uint32_t)a.cap;
  for (uint32_t i = t; i < lim; i += 256) {
    uint64_t key = a.res[(int64_t)q * a.cap + i];
    if (key_d(key) <= band) {
      uint32_t slot = atomicAdd(&scount, 1u);
      if (slot < kSMax) spos[slot] = (uint32_t)key;
    }
  }
  __syncthreads();
  const uint32_t s = scount;
  if (ovf || s > kSMax) {
    if (t == 0) status[q] = ovf ? ovf : 5;
    return;
  }
  // n_pad is a power of two >= 64, so a row is 2^lg float4
  const int nq4 = a.n_pad / 4, lg = __builtin_ctz((unsigned)nq4);
  const float4* q4 = reinterpret_cast<const float4*>(a.Qp + (int64_t)q * a.n_pad);
  const float4* x4 = reinterpret_cast<const float4*>(a.X);
  for (int i = t; i < nq4; i += 256) sq4[i] = q4[i];
  const uint32_t per = (uint32_t)(kFinStageFloats / a.n_pad);  // rows per batch
  for (uint32_t r0 = 0; r0 < s; r0 += per) {
    const int tot = (int)((s - r0 < per ? s - r0 : per) << lg);  // <= kFinStageFloats / 4
    float4 v[kFinStageFloats / 4 / 256];
#pragma unroll
    for (int u = 0; u < kFinStageFloats / 4 / 256; u++) {
      const int i = u * 256 + t < tot ? u * 256 + t : 0;  // past the batch: a repeat of its first value
      v[u] = x4[((int64_t)spos[r0 + (i >> lg)] << lg) + (i & (nq4 - 1))];
    }
    // row r at r (nq4 + 1), so that rows start in different banks; values
    // past the batch land past its rows (never read)
#pragma unroll
    for (int u = 0; u < kFinStageFloats / 4 / 256; u++) {
      const int i = u * 256 + t;
      sx4[i + (i >> lg)] = v[u];
    }
    __syncthreads();
    if ((int)t < tot >> lg) {
      sd[r0 + t] = lds_d2(sq4, sx4 + t * (nq4 + 1), a.n);
      sid[r0 + t] = a.ids[spos[r0 + t]];
    }
    __syncthreads();  // the batch's rows are read before the next overwrites them
  }
  const int k = a.k;
  for (uint32_t i = t; i < s; i += 256) {
    double di = sd[i];
    int64_t ii = sid[i];  // the index's ids are 32-bit
    uint32_t rank = 0;
    for (uint32_t j = 0; j < s; j++) rank += (sd[j] < di || (sd[j] == di && sid[j] < ii)) ? 1u : 0u;
    if (rank < (uint32_t)k) {
      out_ids[(int64_t)q * k + rank] = ii;
      out_d[(int64_t)q * k + rank] = (float)sqrt(di);
    }
    if (rank == (uint32_t)(k - 1)) {
      float r0 = a.U0[q];
      if (isfinite(r0) && !(di <= (double)r0 * (1.0 - 1e-9))) sstat = 1;
    }
  }
  __syncthreads();
  if (t == 0) {
    int st = sstat;
    if (s < (uint32_t)k) st = isfinite(a.U0[q]) ? 1 : 3;
    status[q] = st;
  }
  for (uint32_t r = s + t; r < (uint32_t)k; r += 256) {
    out_ids[(int64_t)q * k + r] = -1;
    out_d[(int64_t)q * k + r] = INFINITY;
  }
}

// Exhaustive pass for one query whose candidate lists overflowed (e.g. many
// exact duplicates): every row's FP32 distance, all rows inside the band of
// the bound U[q] appended to a large buffer.
template <int NIT>
__global__ __launch_bounds__(256) void k_exhaustive(SearchArgs a, int q, uint32_t* __restrict__ pos_out,
                                                    uint32_t* __restrict__ cnt, uint32_t cap) {
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  float4 qr[NIT];
  load_q<NIT>(a.Qp + (int64_t)q * a.n_pad, li, qr);
  const float band = __uint_as_float(a.U[q]) * a.band_f;
  const int64_t wave_id = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t p0 = wave_id * 4; p0 < a.N; p0 += nwaves * 4) {
    int64_t p = p0 + g;
    bool act = p < a.N;
    float d = dist4<NIT>(a.X + (act ? p : 0) * a.n_pad, act, qr, li, band * 2.0f);
    if (li == 0 && act && d <= band) {
      uint32_t slot = atomicAdd(cnt, 1u);
      if (slot < cap) pos_out[slot] = (uint32_t)p;
    }
  }
}

// rows of query q's list of refined rows inside the final FP32 band.  When
// no row of the band was evicted or dropped, the list holds all of them:
// the band only shrinks, so each was inside it when it was refined.
__global__ void k_band_collect(SearchArgs a, int q, uint32_t* __restrict__ pos_out,
                               uint32_t* __restrict__ cnt, uint32_t cap) {
  const float band = __uint_as_float(a.U[q]) * a.band_f;
  const uint32_t c = a.rescnt[q];
  const uint32_t lim = c < (uint32_t)a.cap ? c : (uint32_t)a.cap;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < lim; i += gridDim.x * blockDim.x) {
    const uint64_t key = a.res[(int64_t)q * a.cap + i];
    if (key_d(key) <= band) {
      const uint32_t slot = atomicAdd(cnt, 1u);
      if (slot < cap) pos_out[slot] = (uint32_t)key;
    }
  }
}

// FP64 distances of the exhaustive survivors
__global__ void k_exh_exact(SearchArgs a, int q, const uint32_t* __restrict__ pos, uint32_t s,
                            double* __restrict__ d, int64_t* __restrict__ id) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  d[i] = exact_d2(a.Qp + (int64_t)q * a.n_pad, a.X + (int64_t)pos[i] * a.n_pad, a.n);
  id[i] = a.ids[pos[i]];
}

__global__ void k_exh_rank(int k, int q, uint32_t s, const double* __restrict__ d,
                           const int64_t* __restrict__ id, int64_t* __restrict__ out_ids,
                           float* __restrict__ out_d) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  double di = d[i];
  int64_t ii = id[i];
  uint32_t rank = 0;
  for (uint32_t j = 0; j < s; j++) rank += (d[j] < di || (d[j] == di && id[j] < ii)) ? 1u : 0u;
  if (rank < (uint32_t)k) {
    out_ids[(int64_t)q * k + rank] = ii;
    out_d[(int64_t)q * k + rank] = (float)sqrt(di);
  }
}

// small fills (kept as kernels so that the sequence can be captured)
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_pad_queries(const float* __restrict__ Q, int64_t B, int n, int n_pad,
                              float* __restrict__ Qp, const float* __restrict__ radius,
                              float* __restrict__ U0, unsigned* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B * n_pad) {
    int64_t b = i / n_pad;
    int c = (int)(i % n_pad);
    float v = c < n ? Q[b * n + c] : 0.0f;
    if (!isfinite(v)) atomicOr(bad, 1u);
    Qp[i] = v;
  }
  if (i < B) {
    float u = INFINITY;
    if (radius) {
      float r = radius[i];
      if (isfinite(r) && r >= 0.0f) {
        // squared radius rounded up
        double r2 = (double)r * (double)r;
        u = __double2float_ru(r2 * (1.0 + 1e-12));
      }
    }
    U0[i] = u;
  }
}

// word lower bound of every (query, leaf-order row) pair, for inspection
template <int QB>
__global__ __launch_bounds__(256) void k_all_lb(const float* __restrict__ tables,
                                                const uint8_t* __restrict__ words, int64_t N, int B,
                                                float* __restrict__ out) {
  // QB queries per workgroup share every word load; their tables sit in LDS
  __shared__ float T[QB][kTable];
  const int q0 = blockIdx.y * QB;
  for (int qq = 0; qq < QB; qq++) {
    const int q = q0 + qq < B ? q0 + qq : B - 1;
    const float4* src = reinterpret_cast<const float4*>(tables + (int64_t)q * kTable);
    for (int i = threadIdx.x; i < kTable / 4; i += 256) reinterpret_cast<float4*>(T[qq])[i] = src[i];
  }
  __syncthreads();
  // independent 16-byte word loads per thread in flight (coalesced:
  // consecutive lanes read consecutive words), then the table lookups
  constexpr int U = QB == 1 ? 4 : 8;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p0 = (int64_t)blockIdx.x * 256 + threadIdx.x; p0 < N; p0 += U * stride) {
    uint4 w[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t p = p0 + u * stride;
      w[u] = p < N ? *reinterpret_cast<const uint4*>(words + p * kWordBytes) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int qq = 0; qq < QB; qq++) {
      if (q0 + qq >= B) break;
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int64_t p = p0 + u * stride;
        if (p < N) out[(int64_t)(q0 + qq) * N + p] = lb_word(T[qq], w[u]);
      }
    }
  }
}

// ----------------------------------------------------------------------------
// host launchers
sofa_status launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill_u32<<<nblk(n, 256), 256, 0, st>>>(p, v, n);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

__global__ void k_fill_ranges(FillRanges f) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
#pragma unroll
  for (int r = 0; r < 4; r++)
    for (int64_t i = i0; i < f.n[r]; i += stride) f.p[r][i] = f.v[r];
}

sofa_status launch_fill_ranges(const FillRanges& f, hipStream_t st) {
  int64_t m = 0;
  for (int r = 0; r < 4; r++) m = f.n[r] > m ? f.n[r] : m;
  if (m > 0) k_fill_ranges<<<nblk(m, 256) < 1024 ? nblk(m, 256) : 1024u, 256, 0, st>>>(f);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_all_lb(const SearchArgs& a, float* d_lb, hipStream_t st) {
  unsigned gx = nblk(a.N, a.B == 1 ? 1024 : 2048);
  if (gx > 2048) gx = 2048;
  if (a.B == 1) {
    k_all_lb<1><<<dim3(gx, 1), 256, 0, st>>>(a.tables, a.words, a.N, a.B, d_lb);
  } else if (a.B == 2) {
    k_all_lb<2><<<dim3(gx, 1), 256, 0, st>>>(a.tables, a.words, a.N, a.B, d_lb);
  } else {
    k_all_lb<4><<<dim3(gx, (unsigned)((a.B + 3) / 4)), 256, 0, st>>>(a.tables, a.words, a.N, a.B, d_lb);
  }
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

inline void mark(hipEvent_t* ev, int i, hipStream_t st) {
  if (ev) (void)hipEventRecord(ev[i], st);
}

template <int NIT, int R>
static void launch_front_t(const SearchArgs& a, hipStream_t st, hipEvent_t* ev) {
  dim3 gl((unsigned)((a.n_leaves + kSegLeaves - 1) / kSegLeaves), (unsigned)a.B);
  mark(ev, 1, st);
  k_leaf_lb<<<gl, 256, 0, st>>>(a);
  mark(ev, 2, st);
  k_seed<NIT, R><<<(unsigned)a.B, 256, 0, st>>>(a);
  mark(ev, 3, st);
  (void)launch_leaf_mask(a, st);
  mark(ev, 4, st);
}

sofa_status launch_leaf_mask(const SearchArgs& a, hipStream_t st) {
  const dim3 gm((unsigned)a.n_blocks, nblk(a.B, 256));
  k_leaf_mask<<<gm, 256, 0, st>>>(a);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

template <int NIT>
static void launch_exh_t(const SearchArgs& a, int q, uint32_t* pos, uint32_t* cnt, uint32_t cap,
                         hipStream_t st) {
  k_exhaustive<NIT><<<1024, 256, 0, st>>>(a, q, pos, cnt, cap);
}

sofa_status launch_prepare(const SearchArgs& a, const float* Q, const float* radius,
                           const sofa_bins& bins, float* pool, double* qnorm2, unsigned* bad,
                           hipStream_t st) {
  const int64_t B = a.B;
  k_pad_queries<<<nblk(B * a.n_pad, 256), 256, 0, st>>>(Q, B, a.n, a.n_pad,
                                                         const_cast<float*>(a.Qp), radius,
                                                         const_cast<float*>(a.U0), bad);
  SOFA_TRY(launch_project(a.Qp, B, a.n_pad, a.n_pad, bins.d_bt_pool.as<float>(), bins.ncol_pool / 16,
                          a.n_pad, pool, bins.ncol_pool, nullptr, 0, nullptr, qnorm2, nullptr, st));
  // Eq. 2 weighs each kept DFT value by 2 (a conjugate pair); PAA rows weigh 1
  const double weight = bins.summary == 1 ? 1.0 : 2.0;
  k_tables<<<(unsigned)B, 256, 0, st>>>(pool, bins.ncol_pool, qnorm2, bins.d_sel.as<int>(), bins.l,
                                        bins.d_beta32.as<float>(), a.eta_x, bins.eta_per_norm, weight,
                                        const_cast<float*>(a.tables), const_cast<uint4*>(a.sq));
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// the per-call state cleared in one launch: best leaves, result counts,
// smallest evicted keys, histograms, work-queue counters
__global__ void k_front_clear(SearchArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.B) {
    a.best[i] = kEmpty;
    a.rescnt[i] = 0u;
    a.evmin[i] = kEmpty;
  }
  if (i < (int64_t)a.B * kHistBins) a.hist[i] = 0u;
  if (i < kQueues) a.counter[i] = 0u;
}

static sofa_status front_fills(const SearchArgs& a, hipStream_t st) {
  const int64_t n = std::max<int64_t>((int64_t)a.B * kHistBins, kQueues);
  k_front_clear<<<nblk(n, 256), 256, 0, st>>>(a);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_front(const SearchArgs& a, hipStream_t st, hipEvent_t* ev) {
  SOFA_TRY(front_fills(a, st));
  const int R = (a.k + 16 <= 64) ? 1 : 2;
  switch (a.n_pad / 64) {
#define SOFA_CASE(NI)                                              \
  case NI:                                                         \
    if (R == 1) launch_front_t<NI, 1>(a, st, ev);                  \
    else launch_front_t<NI, 2>(a, st, ev);                         \
    break;
    SOFA_CASE(1)
    SOFA_CASE(2)
    SOFA_CASE(4)
    SOFA_CASE(8)
    SOFA_CASE(16)
#undef SOFA_CASE
    default: return set_error(SOFA_EINTERNAL, "unsupported padded length %d", a.n_pad);
  }
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_finalize(const SearchArgs& a, int64_t* out_ids, float* out_d, int32_t* status,
                            hipStream_t st, hipEvent_t* ev) {
  mark(ev, 5, st);
  k_finalize<<<(unsigned)a.B, 256, 0, st>>>(a, out_ids, out_d, status);
  mark(ev, 6, st);
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

// ----------------------------------------------------------------------------
// Approximate search (no exactness guarantee): the first answer of Section
// IV-C (descend to the leaf of smallest lower bound and scan it) widened to
// the M leaves of smallest envelope bound per query.

// the M leaves of smallest envelope bound of query blockIdx.x (ties: lower
// leaf), from the stored FP16 codes: wave w scans mask blocks w, w + 4, ...
// and keeps a sorted list of its M smallest (code, leaf) keys; wave 0 merges
__global__ __launch_bounds__(256) void k_approx_leaves(SearchArgs a, int M, int32_t* __restrict__ out) {
  __shared__ uint64_t part[4][64];
  const int q = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  WaveList<1> wl;
  wl.reset();
  auto offer = [&](uint64_t key) {
    uint64_t ins = __ballot(key < wl.at(M - 1));
    while (ins) {
      const int l = __builtin_ctzll(ins);
      ins &= ins - 1;
      const uint64_t kk = __shfl(key, l);
      if (kk < wl.at(M - 1)) wl.insert(kk, lane);
    }
  };
  for (int64_t blk = wave; blk < a.n_blocks; blk += 4) {
    const int64_t leaf = blk * kLeavesPerItem + lane;
    const uint64_t key = leaf < a.n_leaves
                             ? ((uint64_t)a.lbh[(blk * a.B + q) * kLeavesPerItem + lane] << 32) | (uint64_t)leaf
                             : kEmpty;
    offer(key);
  }
  part[wave][lane] = wl.e[0];
  __syncthreads();
  if (wave == 0) {
    for (int w = 1; w < 4; w++) offer(part[w][lane]);
    if (lane < M) out[(int64_t)q * kApproxMax + lane] = wl.e[0] == kEmpty ? -1 : (int32_t)(uint32_t)wl.e[0];
  }
}

// exact FP32 distances to the rows of the selected leaves (waves take leaves
// round-robin, 16 rows in flight per step), in-band candidates flushed for
// the final FP64 ranking
template <int NIT, int R>
__global__ __launch_bounds__(256) void k_approx_scan(SearchArgs a, int M, const int32_t* __restrict__ leaves) {
  const int q = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  float4 qr[NIT];
  load_q<NIT>(a.Qp + (int64_t)q * a.n_pad, li, qr);
  float Umin = __uint_as_float(__atomic_load_n(a.U + q, __ATOMIC_RELAXED));
  const float U_in = Umin;
  WaveList<R> wl;
  wl.reset();
  unsigned long long scanned = 0;
  for (int i = wave; i < M; i += 4) {
    const int leaf = leaves[(int64_t)q * kApproxMax + i];
    if (leaf < 0) continue;  // fewer leaves than M
    const int64_t start = (int64_t)leaf * a.L, end = start + a.L < a.N ? start + a.L : a.N;
    scanned += (unsigned long long)(end - start);
    for (int64_t p0 = start; p0 < end; p0 += 4 * kRefRows) {
      uint32_t pm[kRefRows];
      bool am[kRefRows];
#pragma unroll
      for (int r = 0; r < kRefRows; r++) {
        const int64_t p = p0 + 4 * r + g;
        am[r] = p < end;
        pm[r] = (uint32_t)(am[r] ? p : start);
      }
      float d[kRefRows];
      dist_rows<NIT>(a.X, a.n_pad, pm, am, qr, li, Umin * a.abandon_f, d);
#pragma unroll
      for (int r = 0; r < kRefRows; r++)
#pragma unroll
        for (int gi = 0; gi < 4; gi++) {
          const int64_t p = p0 + 4 * r + gi;
          const float dd = __shfl(d[r], 16 * gi);
          if (p < end && dd <= Umin * a.band_f) wl.insert(((uint64_t)__float_as_uint(dd) << 32) | (uint64_t)p, lane);
        }
      const uint64_t kth = wl.at(a.k - 1);
      if (kth != kEmpty) {
        const float uw = key_d(kth) * a.upd_f;
        Umin = uw < Umin ? uw : Umin;
      }
    }
  }
  if (lane == 0 && Umin < U_in) atomicMin(a.U + q, __float_as_uint(Umin));
  flush_wave_list<R>(a, q, wl, Umin, lane);
  if (lane == 0) stat_add(a, 2, scanned);
}

template <int NIT, int R>
static void launch_approx_t(const SearchArgs& a, int M, int32_t* leaves, hipStream_t st) {
  k_approx_leaves<<<(unsigned)a.B, 256, 0, st>>>(a, M, leaves);
  k_approx_scan<NIT, R><<<(unsigned)a.B, 256, 0, st>>>(a, M, leaves);
}

sofa_status launch_approx(const SearchArgs& a, int M, int32_t* leaves, hipStream_t st, hipEvent_t* ev) {
  if (M < 1 || M > kApproxMax) return set_error(SOFA_EINVAL, "approx_leaves=%d outside [1,%d]", M, kApproxMax);
  SOFA_TRY(launch_front(a, st, ev));
  const int R = (a.k + 16 <= 64) ? 1 : 2;
  switch (a.n_pad / 64) {
#define SOFA_CASE(NI)                                              \
  case NI:                                                         \
    if (R == 1) launch_approx_t<NI, 1>(a, M, leaves, st);          \
    else launch_approx_t<NI, 2>(a, M, leaves, st);                 \
    break;
    SOFA_CASE(1)
    SOFA_CASE(2)
    SOFA_CASE(4)
    SOFA_CASE(8)
    SOFA_CASE(16)
#undef SOFA_CASE
    default: return set_error(SOFA_EINTERNAL, "unsupported padded length %d", a.n_pad);
  }
  SOFA_HIP(hipGetLastError());
  return SOFA_OK;
}

sofa_status launch_search(const SearchArgs& a, int64_t* out_ids, float* out_d, int32_t* status,
                          hipStream_t st, hipEvent_t* ev) {
  SOFA_TRY(launch_front(a, st, ev));
  // persistent grid: a multiple of the queue count so every queue has workers
  unsigned grid = 256 * 6;
  uint64_t total = (uint64_t)a.n_blocks * kSubPerBlock * (uint64_t)a.B;
  if (total < grid) grid = (unsigned)(((total + kQueues - 1) / kQueues) * kQueues);
  if (grid == 0) grid = kQueues;
  const int R = (a.k + 16 <= 64) ? 1 : 2;
  switch (a.n_pad / 64) {
#define SOFA_CASE(NI)                                              \
  case NI:                                                         \
    if (R == 1) k_refine<NI, 1><<<grid, 256, 0, st>>>(a);          \
    else k_refine<NI, 2><<<grid, 256, 0, st>>>(a);                 \
    break;
    SOFA_CASE(1)
    SOFA_CASE(2)
    SOFA_CASE(4)
    SOFA_CASE(8)
    SOFA_CASE(16)
#undef SOFA_CASE
    default: return set_error(SOFA_EINTERNAL, "unsupported padded length %d", a.n_pad);
  }
  SOFA_HIP(hipGetLastError());
  return launch_finalize(a, out_ids, out_d, status, st, ev);
}

// FP64 ranking of the s rows collected in pos: the query's k nearest
static sofa_status rank_collected(const SearchArgs& a, int q, uint32_t* pos, uint32_t* cnt, uint32_t cap,
                                  double* d, int64_t* id, int64_t* out_ids, float* out_d, hipStream_t st,
                                  uint32_t* s_out, const char* what) {
  uint32_t s = 0;
  SOFA_HIP(hipMemcpyAsync(&s, cnt, 4, hipMemcpyDeviceToHost, st));
  SOFA_HIP(hipStreamSynchronize(st));
  if (s > cap)
    return set_error(SOFA_EINTERNAL, "query %d: %u series tie within the FP32 error band "
                                     "(limit %u)", q, s, cap);
  if (s < (uint32_t)a.k) return set_error(SOFA_EINTERNAL, "query %d: %s found %u < k rows", q, what, s);
  k_exh_exact<<<nblk(s, 256), 256, 0, st>>>(a, q, pos, s, d, id);
  k_exh_rank<<<nblk(s, 256), 256, 0, st>>>(a.k, q, s, d, id, out_ids, out_d);
  SOFA_HIP(hipGetLastError());
  *s_out = s;
  return SOFA_OK;
}

sofa_status launch_exhaustive(const SearchArgs& a, int q, uint32_t* pos, uint32_t* cnt,
                              uint32_t cap, double* d, int64_t* id, int64_t* out_ids, float* out_d,
                              hipStream_t st, uint32_t* s_out) {
  k_fill_u32<<<1, 64, 0, st>>>(cnt, 0u, 1);
  switch (a.n_pad / 64) {
    case 1: launch_exh_t<1>(a, q, pos, cnt, cap, st); break;
    case 2: launch_exh_t<2>(a, q, pos, cnt, cap, st); break;
    case 4: launch_exh_t<4>(a, q, pos, cnt, cap, st); break;
    case 8: launch_exh_t<8>(a, q, pos, cnt, cap, st); break;
    case 16: launch_exh_t<16>(a, q, pos, cnt, cap, st); break;
    default: return set_error(SOFA_EINTERNAL, "unsupported padded length %d", a.n_pad);
  }
  return rank_collected(a, q, pos, cnt, cap, d, id, out_ids, out_d, st, s_out, "exhaustive pass");
}

sofa_status launch_band_rank(const SearchArgs& a, int q, uint32_t* pos, uint32_t* cnt, uint32_t cap,
                             double* d, int64_t* id, int64_t* out_ids, float* out_d, hipStream_t st,
                             uint32_t* s_out) {
  k_fill_u32<<<1, 64, 0, st>>>(cnt, 0u, 1);
  k_band_collect<<<64, 256, 0, st>>>(a, q, pos, cnt, cap);
  return rank_collected(a, q, pos, cnt, cap, d, id, out_ids, out_d, st, s_out, "band ranking");
}

}  // namespace sofa
