// bf16.h -- arguments of the BF16 / FP8 batched-distance prune (internal).
#pragma once

#include "search_dev.h"

namespace sofa {

constexpr int kGroup = 64;  // queries per MFMA query group
// waves per SIMD of the tile kernel: the two waves of a SIMD hide each
// other's epilogues and LDS waits (one wave running both column blocks of a
// group together, with 512 registers, measured slower on 10M x 256)
constexpr int kTileWaves = 2;

struct Bf16Args {
  int prec;                 // 1: BF16 copy, 2: FP8 (e4m3) copy
  const uint4* xb;          // BF16 or FP8 rows in MFMA A-operand order
  const float4* meta;       // per row: |x|^2 (down), r_x (up), |xh| (up)
  const float4* leafmeta;   // per leaf: max |xh|, max r_x, max |x|^2
  const float* cscale;      // FP8: power-of-two scale per 256-row chunk
  uint4* qb;                // BF16 or FP8 query rows (n_pad values) per sorted slot
  float* qscale;            // FP8: power-of-two scale per sorted slot
  float4* qmeta;            // per slot: |q|^2 (down), r_q (up), |qh| (up), |q| (up)
  int32_t* perm;            // sorted slot -> query
  uint32_t* qcount;         // surviving leaves per query
  uint32_t* lcnt;           // n_leaves: queries whose (query, leaf) pair survives
  int64_t* loff;            // n_leaves: start of each leaf's list in lslot
  uint16_t* lslot;          // per leaf (B entries from leaf * B), the sorted slots of those queries
  float4* slotc;            // per slot and pass: bound terms (a, b, c) and the query id
  int G;                    // query groups
  uint32_t* cand;           // B x cap candidate rows
  uint32_t* ccnt;           // B
  uint32_t* cevmin;         // B smallest lower bound of a dropped candidate (FP32 bits)
  int cap;
  uint32_t* counter;
  int64_t chunk_first, chunk_stride, n_items;  // 256-row chunks of this pass
  int skip;                 // > 0: the pass enumerates the chunks that are not multiples of skip
  int64_t chunk_mult;       // chunk = chunk_mult * (enumerated index)
  int slices;               // work items per chunk, each taking a share of its query groups
  float* dump;              // inspection only: B x N lower bounds of every pair (no pruning)
};

sofa_status launch_bf16_build(const float* X, int64_t N, int n_pad, int L, int64_t n_leaves,
                              uint4* xb, float4* meta, float4* leafmeta, hipStream_t st);
// FP8 copy: xf in 32x32x64 operand order (two 16-byte halves per lane
// fragment), cscale per 256-row chunk, per-row meta and per-leaf maxima
sofa_status launch_fp8_build(const float* X, int64_t N, int n_pad, int L, int64_t n_leaves,
                             uint4* xf, float* cscale, float4* meta, float4* leafmeta, hipStream_t st);
// the query side of the prune: density sort, first lists, query rows and
// terms, and the slot terms of the first pass from the current U (with the
// candidate counts and work counter cleared).  clear_qcount false: b.qcount
// (B entries) is already zero.
sofa_status launch_bf16_queries(const SearchArgs& a, Bf16Args& b, hipStream_t st, bool clear_qcount = true);
// rebuild the (query, leaf) lists from the current bounds U, keeping the slot
// order: later passes see only the pairs that still survive.  Only the leaves
// of the next pass (the multiples of sp that are not multiples of prev, when
// prev > 0) get lists; the others are left empty.  The same launch writes
// that pass's slot terms and clears its counts (launch_bf16_pass with
// terms_ready).
sofa_status launch_bf16_relist(const SearchArgs& a, const Bf16Args& b, int64_t sp, int64_t prev,
                               hipStream_t st);
sofa_status launch_bf16_dump(const SearchArgs& a, Bf16Args b, float* d_lb, hipStream_t st);
// the tile kernel over b's work items on a persistent grid (dump: write
// every pair's lower bound to b.dump instead of pruning)
sofa_status launch_bf16_tiles(const SearchArgs& a, const Bf16Args& b, unsigned grid, bool dump, hipStream_t st);
// ev (nullable): events recorded before the tile kernel, between it and the
// candidate refinement, and after
// terms_ready: the query side (first pass) or a relist launched just before
// wrote this pass's slot terms
sofa_status launch_bf16_pass(const SearchArgs& a, Bf16Args b, int64_t mult, int64_t first,
                             int64_t stride, int64_t n_items, int skip, bool terms_ready, hipStream_t st,
                             hipEvent_t* ev);

}  // namespace sofa
