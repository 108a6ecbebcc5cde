// k_tiles.hip -- the tile kernel of the batched-distance prune: for every
// (query, row) pair on the per-leaf lists, the BF16 (or FP8 e4m3) inner
// product on the matrix cores with FP32 accumulation, and the rigorous
// per-pair test that keeps a row only when its lower bound on the squared
// distance does not exceed the query's bound U.  The copies, the per-row and
// per-leaf bound terms, the lists and the refinement of the kept rows are
// built in k_bf16.hip.
#include "bf16.h"

namespace sofa {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));  // plain 16-byte vector (no struct copies)

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
  if (lane == 0) stat_add(a, 3, st_pairs);
  if (threadIdx.x == 0) {
    stat_add(a, 5, st_needed);
    stat_add(a, 6, st_rows);
  }
}

// launch over the supported (precision, K steps) pairs.  FP8 rows of 1024
// values: the A operand alone takes 256 VGPRs and the two B buffers 128 KB
// of LDS, so one workgroup per CU, one wave per SIMD (512 registers).
template <bool DUMP>
static sofa_status launch_tiles_t(const SearchArgs& a, const Bf16Args& b, unsigned grid, hipStream_t st) {
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

sofa_status launch_bf16_tiles(const SearchArgs& a, const Bf16Args& b, unsigned grid, bool dump, hipStream_t st) {
  return dump ? launch_tiles_t<true>(a, b, grid, st) : launch_tiles_t<false>(a, b, grid, st);
}

}  // namespace sofa
