// sofa_internal.h -- internal declarations of the SOFA GPU library (not ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/sofa.h"

namespace sofa {

// ----------------------------------------------------------------------------
// error reporting
sofa_status set_error(sofa_status st, const char* fmt, ...);
#define SOFA_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t _e = (call);                                                             \
    if (_e != hipSuccess)                                                               \
      return ::sofa::set_error(SOFA_EDEVICE, "%s failed: %s (%s:%d)", #call,            \
                               hipGetErrorString(_e), __FILE__, __LINE__);              \
  } while (0)
#define SOFA_TRY(expr)                  \
  do {                                  \
    sofa_status _s = (expr);            \
    if (_s != SOFA_OK) return _s;       \
  } while (0)

// ----------------------------------------------------------------------------
// fixed sizes of the packed layouts
constexpr int kWordBytes = 16;    // one SFA word: up to 16 symbols of 8 bits
constexpr int kMaxL = 16;         // word positions
constexpr int kAlphaMax = 256;    // symbols per position
constexpr int kTable = kMaxL * kAlphaMax;  // lower-bound table entries per query
constexpr int kLeavesPerItem = 64;         // leaves per refinement work item (one u64 mask)
constexpr int kMaxK = 100;
constexpr int kMaxN = 1024;

// A dispatch counts the work-items of each grid dimension in 32 bits, so a
// grid of 2^32 threads or more wraps and silently skips its tail.  Kernels
// whose size grows with the collection take at most kMaxGridBlocks
// workgroups and stride over the rest.
constexpr int64_t kMaxGridBlocks = 1 << 16;
static inline unsigned grid_blocks(int64_t items, int64_t per_block) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (unsigned)(b < 1 ? 1 : (b > kMaxGridBlocks ? kMaxGridBlocks : b));
}

// n_pad: row length of the permuted copy, a power-of-two multiple of 64 so that
// 16 lanes x float4 cover a row in n_pad/64 steps
int pad_len(int n);

// Device memory comes from hipMalloc, or from the caller's allocator once
// sofa_set_allocator installed one.  A buffer remembers where its memory came
// from and returns it there.
struct Allocator {
  sofa_alloc_fn alloc = nullptr;  // null: hipMalloc / hipFree
  sofa_free_fn free = nullptr;
  void* ctx = nullptr;
};
Allocator current_allocator();

// device buffer owned by a host object
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Allocator from;                 // where p came from
  hipStream_t stream = nullptr;   // the stream it was allocated for (may be null)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;  // one owner per allocation
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { take(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    take(o);
    return *this;
  }
  ~DevBuf() { release(); }
  void release();
  // takes o's memory (and where it came from); o is left empty
  void take(DevBuf& o);
  // exact size, drops old contents; `st` is passed to the caller's allocator
  sofa_status alloc(size_t b, hipStream_t st = nullptr);
  sofa_status reserve(size_t b, hipStream_t st = nullptr);  // grows only
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Device bytes a sofa_knn batch takes in its workspace: the batch's regions
// and its reserved fall-back buffers (params as given to sofa_knn).
int64_t knn_workspace_bytes(const sofa_index* ix, int64_t B, int k, const sofa_knn_params* p);
// bytes a workspace holds now (it keeps the capacity of its largest batch)
int64_t workspace_held_bytes(sofa_workspace* ws);
// frees what the workspace holds; false (nothing freed) while a call uses it
bool workspace_trim(sofa_workspace* ws);

}  // namespace sofa

// ----------------------------------------------------------------------------
// handle types (opaque in the ABI)
struct sofa_bins {
  int32_t n = 0, n_pad = 0, l = 16, alpha = 256, pool = 16, binning = 0;
  int32_t summary = 0;        // 0 SFA, 1 iSAX (PAA means, N(0,1) breakpoints)
  int32_t selection = 0;      // SFA: 0 largest variance, 1 first l pool values
  int32_t sel[16] = {0};
  std::vector<double> beta;  // l x (alpha-1)
  std::vector<double> var;   // 2*pool
  int ncol_pool = 0;         // 2*pool rounded up to 16
  double eta_per_norm = 0;   // projection error bound per unit row norm
  // device copies
  sofa::DevBuf d_bt_sel;     // 16 x n_pad FP32: basis rows of the kept values (transposed)
  sofa::DevBuf d_bt_pool;    // ncol_pool x n_pad FP32: basis rows of every pool value
  sofa::DevBuf d_beta32;     // 16 x 256 FP32 breakpoints, +inf beyond alpha-1 and for j >= l
  sofa::DevBuf d_sel;        // 16 int32
};

struct sofa_workspace;

struct sofa_index {
  const sofa_bins* bins_ref = nullptr;  // not owned; copied below
  sofa_bins bins;                       // private copy (device tables included)
  int64_t N = 0;
  int32_t n = 0, n_pad = 0, L = 256, key_scheme = 0;
  int64_t n_leaves = 0, n_blocks = 0;
  double eta_x = 0;            // |c32 - c| bound for every data row
  double max_norm = 0;
  sofa::DevBuf X;              // N x n_pad FP32, leaf order, zero padded
  sofa::DevBuf words;          // N x 16 u8, leaf order
  sofa::DevBuf ids;            // N int32: row id per leaf-order position
  sofa::DevBuf keys;           // N u64 sort keys, leaf order
  sofa::DevBuf env;            // n_leaves x 32 u8: lo[16], hi[16]
  sofa::DevBuf norm2;          // N FP64 squared norms, leaf order
  // BF16 tier
  int has_bf16 = 0;
  sofa::DevBuf xb;             // BF16 copy, MFMA-tile order
  sofa::DevBuf xb_meta;        // per row: ||x||^2 (rd), r_x (ru), ||xhat|| (ru) as float4
  sofa::DevBuf xb_leafmeta;    // per leaf: max ||xhat||, max r_x, max ||x||^2
  // FP8 (e4m3) tier
  int has_fp8 = 0;
  sofa::DevBuf xf;             // FP8 copy, MFMA-tile order (two 16-byte halves per fragment)
  sofa::DevBuf xf_cscale;      // per 256-row chunk: power-of-two scale
  sofa::DevBuf xf_meta;        // per row, as xb_meta for the FP8 copy
  sofa::DevBuf xf_leafmeta;    // per leaf, as xb_leafmeta for the FP8 copy
  sofa_workspace* own_ws = nullptr;
  int64_t device_bytes() const;
};
