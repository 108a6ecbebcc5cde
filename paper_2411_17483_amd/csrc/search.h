// search.h -- arguments of the search kernels (internal).
#pragma once

#include "kernels.h"

namespace sofa {

// Search statistics are kept in kStatShards copies of kStatSlots counters,
// each copy on its own 128-byte line; a workgroup adds to the copy its
// block index selects, and the host sums the copies (slot 4: the maximum).
// Thousands of workgroups adding to one counter would queue on one address.
constexpr int kStatSlots = 16, kStatShards = 64;

struct SearchArgs {
  // index (leaf order)
  const float* X;        // N x n_pad
  const uint8_t* words;  // N x 16
  const int32_t* ids;    // N
  const uint8_t* env;    // n_leaves x 32
  int64_t N;
  int n, n_pad, L;
  int64_t n_leaves, n_blocks;
  // batch
  int B, k, cap, seed_leaf;
  float* Qp;             // B x n_pad, zero padded
  float* tables;         // B x 16 x 256
  uint4* sq;             // B query symbols
  uint32_t* U;           // B bounds on the k-th squared distance (FP32 bits)
  float* U0;             // B radius bounds (+inf when none)
  uint64_t* best;        // B best leaf (bound bits << 32 | leaf)
  uint64_t* masks;       // n_blocks x B survivor masks
  uint16_t* lbh;         // n_blocks x B x 64 envelope bounds, FP16 codes rounded down
  uint32_t* counter;     // work-queue counters (one per XCD queue)
  uint64_t* res;         // B x cap candidates (d32 bits << 32 | position)
  uint32_t* rescnt;      // B
  uint64_t* evmin;       // B smallest candidate key evicted from a list or dropped
  uint32_t* hist;        // B x 256 counts of flushed candidate distances
  float* hbase;          // B histogram range [0, hbase) (the bound after the seed)
  const uint32_t* cevmin;  // nullable: B smallest lower bound of a dropped BF16 candidate
  unsigned long long* stats;  // kStatShards x kStatSlots (nullable): [0] leaves visited
                              // [1] words checked [2] rows refined [3] tile pairs computed
                              // [4] most candidates of a query [5] tile pairs needed
                              // [6] prune-copy rows streamed
  // factors derived from the FP32 error bounds
  float lb_f, band_f, upd_f, abandon_f;
  double eta_x;
};

sofa_status launch_prepare(const SearchArgs& a, const float* Q, const float* radius,
                           const sofa_bins& bins, float* pool, double* qnorm2, unsigned* bad,
                           hipStream_t st);
// ev (nullable): 6 events recorded around the stages (see sofa_knn_stats).
// launch_search = launch_front + the SFA refinement + launch_finalize.
sofa_status launch_search(const SearchArgs& a, int64_t* out_ids, float* out_d, int32_t* status,
                          hipStream_t st, hipEvent_t* ev);
sofa_status launch_front(const SearchArgs& a, hipStream_t st, hipEvent_t* ev);
// survivor masks from the stored envelope bounds and the current U
sofa_status launch_leaf_mask(const SearchArgs& a, hipStream_t st);
// approximate search: the front, then the M (<= kApproxMax) leaves of
// smallest envelope bound per query (B x kApproxMax leaf ids in `leaves`)
// scanned exactly; launch_finalize ranks what they hold
constexpr int kApproxMax = 64;
sofa_status launch_approx(const SearchArgs& a, int M, int32_t* leaves, hipStream_t st, hipEvent_t* ev);
sofa_status launch_finalize(const SearchArgs& a, int64_t* out_ids, float* out_d, int32_t* status,
                            hipStream_t st, hipEvent_t* ev);
sofa_status launch_all_lb(const SearchArgs& a, float* d_lb, hipStream_t st);
sofa_status launch_exhaustive(const SearchArgs& a, int q, uint32_t* pos, uint32_t* cnt,
                              uint32_t cap, double* d, int64_t* id, int64_t* out_ids, float* out_d,
                              hipStream_t st, uint32_t* s_out);
// the final band of query q ranked in FP64 from its list of refined rows
// (valid when no row of the band was evicted or dropped)
sofa_status launch_band_rank(const SearchArgs& a, int q, uint32_t* pos, uint32_t* cnt, uint32_t cap,
                             double* d, int64_t* id, int64_t* out_ids, float* out_d, hipStream_t st,
                             uint32_t* s_out);

}  // namespace sofa
