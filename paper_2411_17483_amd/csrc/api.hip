// api.hip -- C ABI entry points of the SOFA GPU library: argument checks,
// device memory, and the order of the kernel launches.  All arithmetic of the
// search runs in the kernels of k_learn.hip, k_build.hip and k_search.hip.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "bf16.h"
#include "mlp.h"

namespace sofa {

static thread_local std::string g_err;

sofa_status set_error(sofa_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

int pad_len(int n) {
  int p = 64;
  while (p < n) p <<= 1;
  return p;
}

static std::mutex g_alloc_mu;
static Allocator g_alloc;

Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

sofa_status DevBuf::alloc(size_t b, hipStream_t st) {
  release();
  if (b == 0) return SOFA_OK;
  from = current_allocator();
  stream = st;
  if (from.alloc) {
    p = from.alloc(b, (void*)st, from.ctx);
    if (!p) return set_error(SOFA_ENOMEM, "the caller's allocator returned no memory for %zu bytes", b);
  } else {
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return set_error(SOFA_ENOMEM, "device allocation of %zu bytes failed: %s", b, hipGetErrorString(e));
    }
  }
  bytes = b;
  return SOFA_OK;
}

void DevBuf::release() {
  if (p) {
    if (from.free) {
      // the caller's allocator may hand the memory out again at once: no
      // queued kernel may still use it (hipFree waits the same way)
      if (stream) (void)hipStreamSynchronize(stream);
      else (void)hipDeviceSynchronize();
      from.free(p, (void*)stream, from.ctx);
    } else {
      (void)hipFree(p);
    }
  }
  p = nullptr;
  bytes = 0;
  from = Allocator{};
  stream = nullptr;
}

void DevBuf::take(DevBuf& o) {
  if (&o == this) return;
  release();
  p = o.p;
  bytes = o.bytes;
  from = o.from;
  stream = o.stream;
  o.p = nullptr;
  o.bytes = 0;
  o.from = Allocator{};
  o.stream = nullptr;
}

sofa_status DevBuf::reserve(size_t b, hipStream_t st) {
  if (b <= bytes) return SOFA_OK;
  return alloc(b, st);
}

static inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// error bound of the FP32 projection per unit row norm: any accumulation
// order of n_pad products (each exact or rounded once) plus the rounding of
// the basis to FP32 stays within (n_pad + 4) u * sum|x_t b_t|, and
// sum|x_t b_t| <= ||x|| ||b|| with ||b|| = 1/sqrt(2) for every DFT pool
// value and 1 for a PAA row.
static double eta_per_norm_for(int n_pad, int summary) {
  return (double)(n_pad + 4) * 0x1p-24 * 1.01 * (summary == 1 ? 1.0 : 0.70711);
}

}  // namespace sofa

using namespace sofa;

// ============================================================================
extern "C" const char* sofa_last_error(void) { return g_err.c_str(); }

extern "C" sofa_status sofa_set_allocator(sofa_alloc_fn alloc, sofa_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return set_error(SOFA_EINVAL, "give both an allocation and a release function, or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.free = free_fn;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return SOFA_OK;
}

static sofa_status check_bin_params(int n, const sofa_bin_params* p) {
  if (!p) return set_error(SOFA_EINVAL, "null bin parameters");
  if (p->l < 1 || p->l > kMaxL) return set_error(SOFA_EINVAL, "l=%d outside [1,16]", p->l);
  if (p->alpha < 1 || p->alpha > kAlphaMax)
    return set_error(SOFA_EINVAL, "alpha=%d outside [1,256]", p->alpha);
  if (p->summary != 0 && p->summary != 1) return set_error(SOFA_EINVAL, "summary must be 0 (SFA) or 1 (iSAX)");
  if (p->selection != 0 && p->selection != 1) return set_error(SOFA_EINVAL, "selection must be 0 or 1");
  if (p->znormalise != 0 && p->znormalise != 1) return set_error(SOFA_EINVAL, "znormalise must be 0 or 1");
  if (p->summary == 1) {
    if (n < 4 || n > kMaxN || (n & 3)) return set_error(SOFA_EINVAL, "n=%d must be a multiple of 4 in [4,%d]", n, kMaxN);
    if (n % p->l) return set_error(SOFA_EINVAL, "iSAX needs l=%d to divide n=%d", p->l, n);
    return SOFA_OK;
  }
  if (p->pool < 1 || p->pool > 32) return set_error(SOFA_EINVAL, "pool=%d outside [1,32]", p->pool);
  if (p->l > 2 * p->pool) return set_error(SOFA_EINVAL, "l=%d exceeds the pool's %d values", p->l, 2 * p->pool);
  if (p->binning != 0 && p->binning != 1) return set_error(SOFA_EINVAL, "binning must be 0 or 1");
  if (n < 4 || n > kMaxN || (n & 3)) return set_error(SOFA_EINVAL, "n=%d must be a multiple of 4 in [4,%d]", n, kMaxN);
  if (n < 2 * p->pool + 2) return set_error(SOFA_EINVAL, "n=%d too short for pool=%d (need n >= 2*pool+2)", n, p->pool);
  return SOFA_OK;
}

// iSAX: the pool is the l segment values (one zero column when l is odd)
static int pool_for(const sofa_bin_params* p) { return p->summary == 1 ? (p->l + 1) / 2 : p->pool; }

static sofa_status bins_finish(sofa_bins* b, hipStream_t st) {
  b->n_pad = pad_len(b->n);
  b->ncol_pool = ((2 * b->pool + 15) / 16) * 16;
  b->eta_per_norm = eta_per_norm_for(b->n_pad, b->summary);
  return launch_bins_tables(b, st);
}

extern "C" sofa_status sofa_learn_bins(const float* d_series, int64_t N, int32_t n, int64_t m,
                                       const sofa_bin_params* params, void* stream, sofa_bins** out) {
  if (!out) return set_error(SOFA_EINVAL, "null output handle");
  *out = nullptr;
  SOFA_TRY(check_bin_params(n, params));
  if (!d_series || N < 1 || m < 1 || m > N) return set_error(SOFA_EINVAL, "need 1 <= m <= N and a series array");
  if (m > (1ll << 25)) return set_error(SOFA_EINVAL, "the sample holds at most 2^25 rows (asked for %lld)", (long long)m);
  if (N >= (1ll << 31)) return set_error(SOFA_EINVAL, "N must be < 2^31");
  sofa_bins* b = new sofa_bins();
  b->n = n;
  b->l = params->l;
  b->alpha = params->alpha;
  b->summary = params->summary;
  b->selection = params->summary == 1 ? 0 : params->selection;
  b->pool = pool_for(params);
  b->binning = params->summary == 1 ? 0 : params->binning;
  b->var.assign(2 * b->pool, 0.0);
  b->beta.assign((size_t)b->l * (b->alpha > 1 ? b->alpha - 1 : 0), 0.0);
  std::vector<double> beta_tmp((size_t)b->l * (b->alpha > 1 ? b->alpha - 1 : 1));
  // with znormalise, the stride sample is gathered and normalised first; its
  // own stride sample (all of its rows) is then the same rows
  DevBuf zs;
  sofa_status s = SOFA_OK;
  if (params->znormalise) {
    s = zs.alloc((size_t)m * n * 4, S(stream));
    if (s == SOFA_OK) s = launch_znorm(d_series, m, n, zs.as<float>(), S(stream), N);
    if (s == SOFA_OK) {
      d_series = zs.as<float>();
      N = m;
    }
  }
  if (s == SOFA_OK)
    s = launch_learn(d_series, N, n, m, b->pool, b->l, b->alpha, b->binning, b->summary, b->selection,
                     S(stream), b->var.data(), b->sel, beta_tmp.data());
  if (s == SOFA_OK) {
    if (b->alpha > 1) std::copy(beta_tmp.begin(), beta_tmp.begin() + b->beta.size(), b->beta.begin());
    s = bins_finish(b, S(stream));
  }
  if (s != SOFA_OK) {
    delete b;
    return s;
  }
  *out = b;
  return SOFA_OK;
}

extern "C" sofa_status sofa_bins_create(int32_t n, const sofa_bin_params* params, const int32_t* sel,
                                        const double* beta, const double* var, sofa_bins** out) {
  if (!out) return set_error(SOFA_EINVAL, "null output handle");
  *out = nullptr;
  SOFA_TRY(check_bin_params(n, params));
  if (!sel || (params->alpha > 1 && !beta)) return set_error(SOFA_EINVAL, "null sel or beta");
  sofa_bins* b = new sofa_bins();
  b->n = n;
  b->l = params->l;
  b->alpha = params->alpha;
  b->summary = params->summary;
  b->pool = pool_for(params);
  b->binning = params->summary == 1 ? 0 : params->binning;
  for (int j = 0; j < 16; j++) b->sel[j] = j < b->l ? sel[j] : 0;
  for (int j = 0; j < b->l; j++)
    if (sel[j] < 0 || sel[j] >= 2 * b->pool) {
      delete b;
      return set_error(SOFA_EINVAL, "sel[%d]=%d outside the pool", j, sel[j]);
    }
  b->beta.assign((size_t)b->l * (b->alpha > 1 ? b->alpha - 1 : 0), 0.0);
  if (b->alpha > 1) std::copy(beta, beta + b->beta.size(), b->beta.begin());
  for (int j = 0; j < b->l; j++)
    for (int a = 1; a + 1 < b->alpha; a++)
      if (!(b->beta[(size_t)j * (b->alpha - 1) + a - 1] <= b->beta[(size_t)j * (b->alpha - 1) + a])) {
        delete b;
        return set_error(SOFA_EINVAL, "breakpoints of value %d are not sorted", j);
      }
  b->var.assign(2 * b->pool, 0.0);
  if (var) std::copy(var, var + 2 * b->pool, b->var.begin());
  sofa_status s = bins_finish(b, nullptr);
  if (s != SOFA_OK) {
    delete b;
    return s;
  }
  *out = b;
  return SOFA_OK;
}

extern "C" sofa_status sofa_bins_get(const sofa_bins* b, sofa_bin_params* params, int32_t* n,
                                     int32_t* sel, double* beta, double* var) {
  if (!b) return set_error(SOFA_EINVAL, "null bins");
  if (params) {
    params->l = b->l;
    params->alpha = b->alpha;
    params->pool = b->pool;
    params->binning = b->binning;
    params->summary = b->summary;
    params->selection = b->selection;
  }
  if (n) *n = b->n;
  if (sel) memcpy(sel, b->sel, sizeof(int32_t) * b->l);
  if (beta && !b->beta.empty()) memcpy(beta, b->beta.data(), sizeof(double) * b->beta.size());
  if (var) memcpy(var, b->var.data(), sizeof(double) * b->var.size());
  return SOFA_OK;
}

extern "C" void sofa_bins_free(sofa_bins* b) { delete b; }

extern "C" double sofa_bins_eta_per_norm(const sofa_bins* b) { return b ? b->eta_per_norm : 0.0; }

extern "C" sofa_status sofa_transform(const sofa_bins* b, const float* d_x, int64_t m, float* d_pool,
                                      float* d_sel, uint8_t* d_words, void* stream) {
  if (!b || (!d_x && m > 0) || m < 0) return set_error(SOFA_EINVAL, "bad arguments");
  if (d_pool) {
    const int np = 2 * b->pool;
    if (b->ncol_pool == np) {
      SOFA_TRY(launch_project(d_x, m, b->n, b->n, b->d_bt_pool.as<float>(), b->ncol_pool / 16,
                              b->n_pad, d_pool, np, nullptr, 0, nullptr, nullptr, nullptr, S(stream)));
    } else {
      // the projection writes 16-column groups: go through a padded temporary
      DevBuf tmp;
      SOFA_TRY(tmp.alloc((size_t)m * b->ncol_pool * 4, S(stream)));
      SOFA_TRY(launch_project(d_x, m, b->n, b->n, b->d_bt_pool.as<float>(), b->ncol_pool / 16,
                              b->n_pad, tmp.as<float>(), b->ncol_pool, nullptr, 0, nullptr, nullptr,
                              nullptr, S(stream)));
      SOFA_HIP(hipMemcpy2DAsync(d_pool, (size_t)np * 4, tmp.p, (size_t)b->ncol_pool * 4,
                                (size_t)np * 4, (size_t)m, hipMemcpyDeviceToDevice, S(stream)));
      SOFA_HIP(hipStreamSynchronize(S(stream)));
    }
  }
  if (d_sel || d_words) {
    DevBuf tmpw;
    uint8_t* w = d_words;
    if (!w) {
      SOFA_TRY(tmpw.alloc((size_t)m * kWordBytes, S(stream)));
      w = tmpw.as<uint8_t>();
    }
    SOFA_TRY(launch_project(d_x, m, b->n, b->n, b->d_bt_sel.as<float>(), 1, b->n_pad, d_sel, 16,
                            b->d_beta32.as<float>(), b->l, w, nullptr, nullptr, S(stream)));
    if (tmpw.p) SOFA_HIP(hipStreamSynchronize(S(stream)));
  }
  return SOFA_OK;
}

extern "C" sofa_status sofa_znormalise(const float* d_in, int64_t m, int32_t n, float* d_out, void* stream) {
  if (m < 0 || n < 1 || n > (1 << 20)) return set_error(SOFA_EINVAL, "need m >= 0 and 1 <= n <= 2^20");
  if (m == 0) return SOFA_OK;
  if (!d_in || !d_out) return set_error(SOFA_EINVAL, "null array");
  return launch_znorm(d_in, m, n, d_out, S(stream));
}

// ============================================================================
int64_t sofa_index::device_bytes() const {
  return (int64_t)(X.bytes + words.bytes + ids.bytes + keys.bytes + env.bytes + norm2.bytes +
                   xb.bytes + xb_meta.bytes + xb_leafmeta.bytes + xf.bytes + xf_cscale.bytes +
                   xf_meta.bytes + xf_leafmeta.bytes);
}

static sofa_status clone_bins(const sofa_bins* src, sofa_bins* dst) {
  dst->n = src->n;
  dst->l = src->l;
  dst->alpha = src->alpha;
  dst->pool = src->pool;
  dst->binning = src->binning;
  dst->summary = src->summary;
  dst->selection = src->selection;
  memcpy(dst->sel, src->sel, sizeof dst->sel);
  dst->beta = src->beta;
  dst->var = src->var;
  return bins_finish(dst, nullptr);
}

extern "C" sofa_status sofa_build(const sofa_bins* bins, const float* d_series, int64_t N, int32_t n,
                                  const sofa_build_params* params, void* stream, sofa_index** out) {
  if (!out) return set_error(SOFA_EINVAL, "null output handle");
  *out = nullptr;
  if (!bins || !d_series) return set_error(SOFA_EINVAL, "null bins or series");
  if (n != bins->n) return set_error(SOFA_EINVAL, "series length %d differs from the bins' %d", n, bins->n);
  if (N < 1 || N >= (1ll << 31)) return set_error(SOFA_EINVAL, "N=%lld outside [1, 2^31)", (long long)N);
  int L = params ? params->leaf_size : 256;
  if (L == 0) L = 256;
  if (L < 64 || L > 4096 || (L & 63)) return set_error(SOFA_EINVAL, "leaf_size=%d must be a multiple of 64 in [64,4096]", L);
  hipStream_t st = S(stream);
  sofa_index* ix = new sofa_index();
  sofa_status s = clone_bins(bins, &ix->bins);
  ix->bins_ref = bins;
  ix->N = N;
  ix->n = n;
  ix->n_pad = ix->bins.n_pad;
  ix->L = L;
  ix->key_scheme = params ? params->key_scheme : 0;
  if (ix->key_scheme != 0 && ix->key_scheme != 1) {
    delete ix;
    return set_error(SOFA_EINVAL, "key_scheme must be 0 or 1");
  }
  ix->n_leaves = (N + L - 1) / L;
  ix->n_blocks = (ix->n_leaves + kLeavesPerItem - 1) / kLeavesPerItem;
  const int zn = params ? params->znormalise : 0;
  if (zn != 0 && zn != 1) {
    delete ix;
    return set_error(SOFA_EINVAL, "znormalise must be 0 or 1");
  }
  // with znormalise, every later step reads the normalised copy
  DevBuf zcopy;
  if (s == SOFA_OK && zn) {
    s = zcopy.alloc((size_t)N * n * 4, st);
    if (s == SOFA_OK) s = launch_znorm(d_series, N, n, zcopy.as<float>(), st);
    if (s == SOFA_OK) d_series = zcopy.as<float>();
  }
  DevBuf words_in, norm_in, bad;
  if (s == SOFA_OK) s = words_in.alloc((size_t)N * kWordBytes, st);
  if (s == SOFA_OK) s = norm_in.alloc((size_t)N * 8, st);
  if (s == SOFA_OK) s = bad.alloc(4, st);
  if (s == SOFA_OK && hipMemsetAsync(bad.p, 0, 4, st) != hipSuccess) s = set_error(SOFA_EDEVICE, "memset failed");
  if (s == SOFA_OK)
    s = launch_project(d_series, N, n, n, ix->bins.d_bt_sel.as<float>(), 1, ix->n_pad, nullptr, 16,
                       ix->bins.d_beta32.as<float>(), ix->bins.l, words_in.as<uint8_t>(),
                       norm_in.as<double>(), bad.as<unsigned>(), st);
  unsigned hbad = 0;
  if (s == SOFA_OK) {
    if (hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      s = set_error(SOFA_EDEVICE, "reading the validation flag failed: %s", hipGetErrorString(hipGetLastError()));
    else if (hbad)
      s = set_error(SOFA_EINVAL, "the series contain non-finite values");
  }
  if (s == SOFA_OK) s = launch_layout(ix, d_series, words_in.as<uint8_t>(), norm_in.as<double>(), st);
  if (s == SOFA_OK) {
    ix->eta_x = ix->bins.eta_per_norm * ix->max_norm + 1e-30;
    if (params && (params->precision & 1)) {
      if (ix->n_pad > 256)
        s = set_error(SOFA_EINVAL, "the BF16 copy supports n <= 256 (padded length %d)", ix->n_pad);
      else if (ix->L % 256)
        s = set_error(SOFA_EINVAL, "the BF16 copy needs leaf_size to be a multiple of 256");
      else {
        const int64_t nrb = ((N + 255) / 256) * 8;
        const int KS = ix->n_pad / 16;
        if (s == SOFA_OK) s = ix->xb.alloc((size_t)nrb * KS * 64 * 16);
        if (s == SOFA_OK) s = ix->xb_meta.alloc((size_t)N * 16);
        if (s == SOFA_OK) s = ix->xb_leafmeta.alloc((size_t)ix->n_leaves * 16);
        if (s == SOFA_OK)
          s = launch_bf16_build(ix->X.as<float>(), N, ix->n_pad, ix->L, ix->n_leaves, ix->xb.as<uint4>(),
                                ix->xb_meta.as<float4>(), ix->xb_leafmeta.as<float4>(), st);
        if (s == SOFA_OK && hipStreamSynchronize(st) != hipSuccess)
          s = set_error(SOFA_EDEVICE, "BF16 copy failed: %s", hipGetErrorString(hipGetLastError()));
        if (s == SOFA_OK) ix->has_bf16 = 1;
      }
    }
    if (s == SOFA_OK && params && (params->precision & 2)) {
      if (ix->n_pad > 1024)
        s = set_error(SOFA_EINVAL, "the FP8 copy supports n <= 1024 (padded length %d)", ix->n_pad);
      else if (ix->L % 256)
        s = set_error(SOFA_EINVAL, "the FP8 copy needs leaf_size to be a multiple of 256");
      else {
        const int64_t n_chunks = (N + 255) / 256;
        if (s == SOFA_OK) s = ix->xf.alloc((size_t)n_chunks * 256 * ix->n_pad);
        if (s == SOFA_OK) s = ix->xf_cscale.alloc((size_t)n_chunks * 4);
        if (s == SOFA_OK) s = ix->xf_meta.alloc((size_t)N * 16);
        if (s == SOFA_OK) s = ix->xf_leafmeta.alloc((size_t)ix->n_leaves * 16);
        if (s == SOFA_OK)
          s = launch_fp8_build(ix->X.as<float>(), N, ix->n_pad, ix->L, ix->n_leaves, ix->xf.as<uint4>(),
                               ix->xf_cscale.as<float>(), ix->xf_meta.as<float4>(),
                               ix->xf_leafmeta.as<float4>(), st);
        if (s == SOFA_OK && hipStreamSynchronize(st) != hipSuccess)
          s = set_error(SOFA_EDEVICE, "FP8 copy failed: %s", hipGetErrorString(hipGetLastError()));
        if (s == SOFA_OK) ix->has_fp8 = 1;
      }
    }
  }
  if (s != SOFA_OK) {
    delete ix;
    return s;
  }
  *out = ix;
  return SOFA_OK;
}

extern "C" sofa_status sofa_index_get_info(const sofa_index* ix, sofa_index_info* info) {
  if (!ix || !info) return set_error(SOFA_EINVAL, "null argument");
  info->N = ix->N;
  info->n = ix->n;
  info->n_pad = ix->n_pad;
  info->leaf_size = ix->L;
  info->l = ix->bins.l;
  info->alpha = ix->bins.alpha;
  info->n_leaves = ix->n_leaves;
  info->device_bytes = ix->device_bytes();
  info->eta_x = ix->eta_x;
  info->has_bf16 = ix->has_bf16;
  info->has_fp8 = ix->has_fp8;
  return SOFA_OK;
}

extern "C" sofa_status sofa_index_export(const sofa_index* ix, uint8_t* d_words, int32_t* d_ids,
                                         uint8_t* d_env, uint64_t* d_keys, void* stream) {
  if (!ix) return set_error(SOFA_EINVAL, "null index");
  hipStream_t st = S(stream);
  if (d_words) SOFA_HIP(hipMemcpyAsync(d_words, ix->words.p, ix->words.bytes, hipMemcpyDeviceToDevice, st));
  if (d_ids) SOFA_HIP(hipMemcpyAsync(d_ids, ix->ids.p, ix->ids.bytes, hipMemcpyDeviceToDevice, st));
  if (d_env) SOFA_HIP(hipMemcpyAsync(d_env, ix->env.p, ix->env.bytes, hipMemcpyDeviceToDevice, st));
  if (d_keys) SOFA_HIP(hipMemcpyAsync(d_keys, ix->keys.p, ix->keys.bytes, hipMemcpyDeviceToDevice, st));
  return SOFA_OK;
}

// ============================================================================
// sampled BF16 passes: chunk strides, coarsest first, each dividing the one
// before; a pass covers the multiples of its stride that are not multiples
// of the previous stride and selects candidates with the bound U that the
// earlier passes established.  The (query, leaf) lists are fixed before the
// first pass, so finer sampling cuts only the candidate refinement: worth
// two more passes from k = 4 on (10M x 256: k = 10 refines 0.9M instead of
// 1.6M rows), not at k = 1, where each pass costs more than it saves.
constexpr int kPassesFew[] = {1024, 32, 1};
constexpr int kPassesMany[] = {2048, 256, 32, 4, 1};
constexpr int kManyFromK = 4;
constexpr int kMaxPasses = 8;
static_assert(sizeof(kPassesMany) / sizeof(int) <= kMaxPasses, "event slots");

struct sofa_workspace {
  int64_t max_bytes = 0;
  DevBuf buf;  // the regions of one batch (layout_for)
  DevBuf aux;  // its fall-back buffers (aux_layout_for), reserved with it
  std::mutex mu;
  sofa_knn_stats stats{};
  hipEvent_t ev[7 + 3 * kMaxPasses] = {};
  bool ev_ok = false;
  uint8_t* hback = nullptr;  // pinned: what the host reads back after a call
  size_t hback_bytes = 0;
  ~sofa_workspace() {
    if (ev_ok)
      for (auto& e : ev) (void)hipEventDestroy(e);
    if (hback) (void)hipHostFree(hback);
  }
  uint8_t* host_back(size_t bytes) {
    if (bytes > hback_bytes) {
      if (hback) (void)hipHostFree(hback);
      hback = nullptr;
      hback_bytes = 0;
      if (hipHostMalloc((void**)&hback, bytes) != hipSuccess) return nullptr;
      hback_bytes = bytes;
    }
    return hback;
  }
  // stage timers: timing only (the call's read-back synchronises the
  // results), so no system-scope fence: with it, each record cost about
  // 5.6 us of idle GPU between the kernels it separates (20 per call)
  hipEvent_t* events() {
    if (!ev_ok) {
      for (auto& e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      ev_ok = true;
    }
    return ev;
  }
};

extern "C" void sofa_index_free(sofa_index* ix) {
  if (!ix) return;
  delete ix->own_ws;
  delete ix;
}

extern "C" sofa_status sofa_workspace_create(int64_t max_bytes, sofa_workspace** out) {
  if (!out || max_bytes < 0) return set_error(SOFA_EINVAL, "bad arguments");
  sofa_workspace* w = new sofa_workspace();
  w->max_bytes = max_bytes;
  *out = w;
  return SOFA_OK;
}

extern "C" void sofa_workspace_free(sofa_workspace* ws) { delete ws; }

namespace {

constexpr uint32_t kExhCap = 1u << 20;

// Result keys per query (refined rows inside the band when they were
// refined).  A query whose list fills while a dropped row lies in the final
// band is finished by the exhaustive pass, so large k (more rows refined)
// gets a longer list, within a byte budget per batch.
constexpr int64_t kResListBytes = 1ll << 30;
int cap_for(int k, const sofa_knn_params* p, int64_t B) {
  if (p && p->candidate_capacity > 0) return p->candidate_capacity;
  if (k <= 16) return 32768;
  return (int)std::max<int64_t>(65536, std::min<int64_t>(1 << 18, kResListBytes / 8 / std::max<int64_t>(B, 1)));
}

// workspace regions of one batch
enum {
  W_QP, W_POOL, W_QN, W_TAB, W_SQ, W_BEST, W_MASK, W_LBH, W_CTR, W_RES, W_RCNT, W_FLAG, W_HIST, W_HBASE,
  // read back by the host after the call: adjacent, one copy
  W_U, W_U0, W_STAT, W_STATS, W_BAD,
  W_CAND, W_CCNT, W_CEV, W_QCNT, W_PERM, W_LCNT, W_LOFF, W_LSLOT, W_SLOTC, W_QB, W_QMETA, W_QSCALE, W_BCTR,
  W_MLP, W_APPROX, W_QZ, W_END
};

struct Layout {
  size_t off[W_END];  // one offset per region; total = the bytes of all regions
  size_t total;
};

// Candidate slots per query and pass of the batched-distance prune, sized
// so that a pass rarely overflows into the retry pass (a whole pass over the
// prune copy) or the exhaustive pass.  A larger k leaves more rows inside
// the bound, and the FP8 bound is looser (3 fraction bits), so both get
// longer lists, kept within a byte budget per batch and never below the
// BF16 base size.
constexpr int kBf16Cap = 32768, kBf16CapLargeK = 1 << 18;
constexpr int kFp8Cap = 1 << 18, kFp8CapLargeK = 1 << 20;
constexpr int64_t kBf16ListBytes = 1ll << 30, kFp8ListBytes = 1ll << 31;
int bf16_cap(const sofa_knn_params* p, int k, int64_t B) {
  if (p && p->candidate_capacity > 0) return p->candidate_capacity;
  const bool fp8 = p && p->prune == 2;
  const int64_t want = fp8 ? (k > 16 ? kFp8CapLargeK : kFp8Cap) : (k > 16 ? kBf16CapLargeK : kBf16Cap);
  const int64_t fit = (fp8 ? kFp8ListBytes : kBf16ListBytes) / 4 / std::max<int64_t>(B, 1);
  return (int)std::max<int64_t>(kBf16Cap, std::min(want, fit));
}

Layout layout_for(const sofa_index* ix, int64_t B, int k, const sofa_knn_params* p) {
  size_t sz[W_END];
  const bool bf = p && (p->prune == 1 || p->prune == 2);
  const int64_t G = (B + kGroup - 1) / kGroup;
  sz[W_QP] = (size_t)B * ix->n_pad * 4;
  sz[W_POOL] = (size_t)B * ix->bins.ncol_pool * 4;
  sz[W_QN] = (size_t)B * 8;
  sz[W_TAB] = (size_t)B * kTable * 4;
  sz[W_SQ] = (size_t)B * 16;
  sz[W_U] = (size_t)B * 4;
  sz[W_U0] = (size_t)B * 4;
  sz[W_BEST] = (size_t)B * 8;
  sz[W_MASK] = (size_t)ix->n_blocks * B * 8;
  sz[W_LBH] = (size_t)ix->n_blocks * kLeavesPerItem * B * 2;
  sz[W_CTR] = 64;
  sz[W_RES] = (size_t)B * cap_for(k, p, B) * 8;
  sz[W_RCNT] = (size_t)B * 4;
  sz[W_FLAG] = (size_t)B * 8;
  sz[W_STAT] = (size_t)B * 4;
  sz[W_STATS] = (size_t)kStatShards * kStatSlots * 8;
  sz[W_BAD] = 4;
  sz[W_HIST] = (size_t)B * 256 * 4;
  sz[W_HBASE] = (size_t)B * 4;
  sz[W_CAND] = bf ? (size_t)B * bf16_cap(p, k, B) * 4 : 0;
  sz[W_CCNT] = bf ? (size_t)B * 4 : 0;
  sz[W_CEV] = bf ? (size_t)B * 4 : 0;
  sz[W_QCNT] = bf ? (size_t)B * 4 : 0;
  sz[W_PERM] = bf ? (size_t)B * 4 : 0;
  sz[W_LCNT] = bf ? (size_t)ix->n_leaves * 4 : 0;
  sz[W_LOFF] = bf ? (size_t)ix->n_leaves * 8 : 0;
  sz[W_LSLOT] = bf ? (size_t)ix->n_leaves * B * 2 : 0;  // worst case: every query needs every leaf
  sz[W_SLOTC] = bf ? (size_t)G * kGroup * 16 : 0;
  sz[W_QB] = bf ? (size_t)G * kGroup * ix->n_pad * 2 : 0;
  sz[W_QMETA] = bf ? (size_t)G * kGroup * 16 : 0;
  sz[W_QSCALE] = bf ? (size_t)G * kGroup * 4 : 0;
  sz[W_BCTR] = bf ? 64 : 0;
  sz[W_MLP] = (p && p->radius_model && !p->d_radius) ? model_radius_scratch_floats(p->radius_model->dims, B) * 4 : 0;
  sz[W_APPROX] = (p && p->approx_leaves > 0) ? (size_t)B * kApproxMax * 4 : 0;
  sz[W_QZ] = (p && p->znormalise) ? (size_t)B * ix->n * 4 : 0;
  Layout L;
  static_assert(sizeof(L.off) / sizeof(L.off[0]) == W_END, "one offset per workspace region");
  size_t o = 0;
  for (int i = 0; i < W_END; i++) {
    L.off[i] = o;
    o += (sz[i] + 255) & ~(size_t)255;
  }
  L.total = o;
  return L;
}

// Fall-back buffers of a batch of B queries, reserved with the batch so
// that no fall-back allocates: the exhaustive pass's lists, and the copies
// (queries, ids, distances, radii) of the re-searches.  A re-search takes a
// subset of its caller's queries and nests at most twice (a dropped-candidate
// retry with a radius whose query then misses the radius), so two slices
// sized for the top-level batch cover every level.
constexpr int kResearchDepth = 2;
struct AuxLayout {
  size_t exh, research[kResearchDepth], total;
};
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t research_slice_bytes(const sofa_index* ix, int64_t B, int k) {
  return align256((size_t)B * ix->n * 4) + align256((size_t)B * k * 8) + align256((size_t)B * k * 4) +
         align256((size_t)B * 4);
}
AuxLayout aux_layout_for(const sofa_index* ix, int64_t B, int k) {
  AuxLayout A;
  A.exh = 0;
  size_t o = align256((size_t)kExhCap * (4 + 8 + 8) + 256);
  for (int d = 0; d < kResearchDepth; d++) {
    A.research[d] = o;
    o += research_slice_bytes(ix, B, k);
  }
  A.total = o;
  return A;
}

}  // namespace

namespace sofa {
int64_t knn_workspace_bytes(const sofa_index* ix, int64_t B, int k, const sofa_knn_params* p) {
  return (int64_t)(layout_for(ix, B, k, p).total + aux_layout_for(ix, B, k).total);
}
int64_t workspace_held_bytes(sofa_workspace* ws) {
  return ws ? (int64_t)(ws->buf.bytes + ws->aux.bytes) : 0;
}
bool workspace_trim(sofa_workspace* ws) {
  if (!ws) return true;
  std::unique_lock<std::mutex> lk(ws->mu, std::try_to_lock);
  if (!lk.owns_lock()) return false;  // a call is using it
  ws->buf.release();
  ws->aux.release();
  return true;
}
}  // namespace sofa

extern "C" sofa_status sofa_workspace_bytes_for(const sofa_index* ix, int64_t B, int32_t k, int32_t prune,
                                                int64_t* bytes) {
  if (!ix || !bytes || B < 0 || k < 1) return set_error(SOFA_EINVAL, "bad arguments");
  sofa_knn_params p{};
  p.prune = prune;
  *bytes = knn_workspace_bytes(ix, B, k, &p);
  return SOFA_OK;
}

// Where one sofa_knn call keeps its data: the batch's regions (base, at
// least layout_for bytes of the top-level batch), its fall-back buffers (aux,
// aux_layout_for), host memory for the read-back after the search, and the
// stage timers (nullable).
struct KnnMem {
  char* base = nullptr;
  size_t base_bytes = 0;
  char* aux = nullptr;
  uint8_t* hback = nullptr;
  size_t hback_bytes = 0;
  hipEvent_t* ev = nullptr;
};

// bytes the host reads back after a batch of B queries: the bounds, radii,
// statuses and counters, adjacent in the layout
static size_t readback_bytes(const sofa_index* ix, int64_t B, int k, const sofa_knn_params* p) {
  const Layout lay = layout_for(ix, B, k, p);
  return lay.off[W_BAD] + 4 - lay.off[W_U];
}

// B0: the top-level batch, which sizes the fall-back slices of every depth
static sofa_status knn_impl(const sofa_index* ix, const float* d_q, int64_t B, int k,
                            const sofa_knn_params* p, int64_t* d_ids, float* d_d, hipStream_t st,
                            const KnnMem& mem, sofa_knn_stats& stats, int64_t B0, int depth = 0);

// argument checks of sofa_knn
static sofa_status check_knn_args(const sofa_index* ix, const float* d_queries, int64_t B, int32_t k,
                                  const sofa_knn_params* params, int64_t* d_ids, float* d_dists) {
  if (!ix) return set_error(SOFA_EINVAL, "null index");
  if (B < 0 || B > 65535) return set_error(SOFA_EINVAL, "B=%lld outside [0, 65535]", (long long)B);
  if (k < 1 || k > kMaxK || k > ix->N)
    return set_error(SOFA_EINVAL, "k=%d outside [1, min(N, %d)]", k, kMaxK);
  if (B == 0) return SOFA_OK;
  if (!d_queries || !d_ids || !d_dists) return set_error(SOFA_EINVAL, "null array");
  if (params && params->radius_model && !params->d_radius) {
    const sofa_radius* m = params->radius_model;
    if (m->k != k) return set_error(SOFA_EINVAL, "the radius model predicts k=%d, asked k=%d", m->k, k);
    if (m->dims.D != 2 * ix->bins.pool)
      return set_error(SOFA_EINVAL, "the radius model takes %d features, the index has %d pool values",
                       m->dims.D, 2 * ix->bins.pool);
  }
  if (params && params->znormalise != 0 && params->znormalise != 1)
    return set_error(SOFA_EINVAL, "znormalise must be 0 or 1");
  if (params && (params->approx_leaves < 0 || params->approx_leaves > kApproxMax))
    return set_error(SOFA_EINVAL, "approx_leaves=%d outside [0,%d]", params->approx_leaves, kApproxMax);
  if (params && params->prune != 0) {
    if (params->prune != 1 && params->prune != 2)
      return set_error(SOFA_EINVAL, "prune must be 0 (off), 1 (BF16) or 2 (FP8)");
    if (params->sampling < 0 || params->sampling > 2) return set_error(SOFA_EINVAL, "sampling must be 0, 1 or 2");
    if (params->prune == 1 && !ix->has_bf16) return set_error(SOFA_EINVAL, "the index was built without the BF16 copy");
    if (params->prune == 2 && !ix->has_fp8) return set_error(SOFA_EINVAL, "the index was built without the FP8 copy");
  }
  return SOFA_OK;
}

extern "C" sofa_status sofa_knn(const sofa_index* ix, const float* d_queries, int64_t B, int32_t k,
                                const sofa_knn_params* params, int64_t* d_ids, float* d_dists,
                                void* stream) {
  SOFA_TRY(check_knn_args(ix, d_queries, B, k, params, d_ids, d_dists));
  if (B == 0) return SOFA_OK;
  sofa_workspace* ws = params ? params->ws : nullptr;
  if (!ws) {
    sofa_index* mix = const_cast<sofa_index*>(ix);
    if (!mix->own_ws) mix->own_ws = new sofa_workspace();
    ws = mix->own_ws;
  }
  std::unique_lock<std::mutex> lk(ws->mu, std::try_to_lock);
  if (!lk.owns_lock()) return set_error(SOFA_EBUSY, "workspace in use by another call");
  const size_t lay_bytes = layout_for(ix, B, k, params).total;
  const size_t aux_bytes = aux_layout_for(ix, B, k).total;
  if (ws->max_bytes > 0 && (int64_t)(lay_bytes + aux_bytes) > ws->max_bytes)
    return set_error(SOFA_ENOMEM, "batch needs %zu workspace bytes, limit %lld", lay_bytes + aux_bytes,
                     (long long)ws->max_bytes);
  SOFA_TRY(ws->buf.reserve(lay_bytes, S(stream)));
  SOFA_TRY(ws->aux.reserve(aux_bytes, S(stream)));
  KnnMem mem;
  mem.base = ws->buf.as<char>();
  mem.base_bytes = ws->buf.bytes;
  mem.aux = ws->aux.as<char>();
  mem.hback_bytes = readback_bytes(ix, B, k, params);
  mem.hback = ws->host_back(mem.hback_bytes);
  if (!mem.hback) return set_error(SOFA_ENOMEM, "pinned host buffer of %zu bytes", mem.hback_bytes);
  mem.ev = ws->events();
  hipEvent_t e0, e1;
  SOFA_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  SOFA_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  SOFA_HIP(hipEventRecord(e0, S(stream)));
  sofa_knn_stats stats{};
  sofa_status s = knn_impl(ix, d_queries, B, k, params, d_ids, d_dists, S(stream), mem, stats, B);
  (void)hipEventRecord(e1, S(stream));
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  stats.ms_total = ms;
  ws->stats = stats;
  return s;
}

// ----------------------------------------------------------------------------
// sofa_knn_noalloc: the search with every device buffer in one file-scope
// array per GPU.  In host code `scratch` names a host-side stand-in, not
// device memory: kernels and copies get the address hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr size_t kScratchBytes = (size_t)SOFA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
constexpr int64_t kScratchMaxB = SOFA_NOALLOC_MAX_QUERIES;  // bounds the host read-back buffer
static std::mutex g_scratch_mu;         // one no-alloc call at a time
static char* g_scratch_dev[kScratchDevices];
static uint8_t g_scratch_back[kScratchMaxB * 12 + kStatShards * kStatSlots * 8 + 4096];

static sofa_status scratch_of_current_device(char** out) {
  int dev = -1;
  SOFA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return set_error(SOFA_EINVAL, "device %d: the no-alloc search supports devices 0..%d", dev,
                     kScratchDevices - 1);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    SOFA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = (char*)ptr;
  }
  *out = g_scratch_dev[dev];
  return SOFA_OK;
}

extern "C" sofa_status sofa_knn_noalloc(const sofa_index* ix, const float* d_queries, int64_t B, int32_t k,
                                        const sofa_knn_params* params, int64_t* d_ids, float* d_dists,
                                        void* stream) {
  SOFA_TRY(check_knn_args(ix, d_queries, B, k, params, d_ids, d_dists));
  if (B == 0) return SOFA_OK;
  if (params && params->ws) return set_error(SOFA_EINVAL, "the no-alloc search takes no workspace");
  if (B > kScratchMaxB)
    return set_error(SOFA_ENOMEM, "the no-alloc search takes at most %lld queries (asked %lld)",
                     (long long)kScratchMaxB, (long long)B);
  const size_t lay_bytes = align256(layout_for(ix, B, k, params).total);
  const size_t need = lay_bytes + aux_layout_for(ix, B, k).total;
  if (need > kScratchBytes)
    return set_error(SOFA_ENOMEM,
                     "the batch needs %zu bytes, above the %zu-byte scratch of the no-alloc search "
                     "(fewer queries, a smaller k or sofa_knn with a workspace)",
                     need, kScratchBytes);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  char* base = nullptr;
  SOFA_TRY(scratch_of_current_device(&base));
  KnnMem mem;
  mem.base = base;
  mem.base_bytes = lay_bytes;
  mem.aux = base + lay_bytes;
  mem.hback = g_scratch_back;
  mem.hback_bytes = sizeof g_scratch_back;
  mem.ev = nullptr;  // no stage timers
  if (readback_bytes(ix, B, k, params) > mem.hback_bytes)
    return set_error(SOFA_EINTERNAL, "read-back of %zu bytes above %zu", readback_bytes(ix, B, k, params),
                     mem.hback_bytes);
  sofa_knn_stats stats{};
  sofa_status s = knn_impl(ix, d_queries, B, k, params, d_ids, d_dists, S(stream), mem, stats, B);
  // the next call may reuse the scratch on another stream: this call's
  // kernels must have finished
  const hipError_t e = hipStreamSynchronize(S(stream));
  if (s == SOFA_OK && e != hipSuccess)
    s = set_error(SOFA_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  return s;
}

static sofa_status knn_impl(const sofa_index* ix, const float* d_q, int64_t B, int k,
                            const sofa_knn_params* p, int64_t* d_ids, float* d_d, hipStream_t st,
                            const KnnMem& mem, sofa_knn_stats& stats, int64_t B0, int depth) {
  const Layout lay = layout_for(ix, B, k, p);
  const AuxLayout aux = aux_layout_for(ix, B0, k);
  // a re-search takes a subset of its caller's queries, which never needs
  // more than the top-level batch reserved
  if (lay.total > mem.base_bytes || depth > kResearchDepth)
    return set_error(SOFA_EINTERNAL, "search at depth %d needs %zu workspace bytes, %zu reserved", depth,
                     lay.total, mem.base_bytes);
  char* base = mem.base;
  auto at = [&](int i) { return (void*)(base + lay.off[i]); };
  if (p && p->znormalise) {
    // the search, its fall-backs and their copies all read the normalised queries
    SOFA_TRY(launch_znorm(d_q, B, ix->n, (float*)at(W_QZ), st));
    d_q = (const float*)at(W_QZ);
  }
  SearchArgs a{};
  a.X = ix->X.as<float>();
  a.words = ix->words.as<uint8_t>();
  a.ids = ix->ids.as<int32_t>();
  a.env = ix->env.as<uint8_t>();
  a.N = ix->N;
  a.n = ix->n;
  a.n_pad = ix->n_pad;
  a.L = ix->L;
  a.n_leaves = ix->n_leaves;
  a.n_blocks = ix->n_blocks;
  a.B = (int)B;
  a.k = k;
  a.cap = cap_for(k, p, B);
  a.seed_leaf = (p && p->no_seed_leaf) ? 0 : 1;
  a.Qp = (float*)at(W_QP);
  a.tables = (float*)at(W_TAB);
  a.sq = (uint4*)at(W_SQ);
  a.U = (uint32_t*)at(W_U);
  a.U0 = (float*)at(W_U0);
  a.best = (uint64_t*)at(W_BEST);
  a.masks = (uint64_t*)at(W_MASK);
  a.lbh = (uint16_t*)at(W_LBH);
  a.counter = (uint32_t*)at(W_CTR);
  a.res = (uint64_t*)at(W_RES);
  a.rescnt = (uint32_t*)at(W_RCNT);
  a.evmin = (uint64_t*)at(W_FLAG);
  a.hist = (uint32_t*)at(W_HIST);
  a.hbase = (float*)at(W_HBASE);
  a.stats = (unsigned long long*)at(W_STATS);
  // FP32 distance error bound: per-lane sequential sums of n_pad/16 terms, a
  // 4-level tree, and the rounded difference squared
  const double u = 0x1p-24;
  const double eps = (double)(ix->n_pad / 16 + 16) * u * 1.01;
  a.lb_f = 1.0f + 0x1p-16f;
  a.upd_f = (float)(1.0 + 2.0 * eps + 4.0 * u);
  a.band_f = (float)(1.0 + 3.0 * eps + 4.0 * u);
  a.abandon_f = (float)(1.0 + 5.0 * eps + 4.0 * u);
  a.eta_x = ix->eta_x;
  int32_t* status = (int32_t*)at(W_STAT);
  unsigned* bad = (unsigned*)at(W_BAD);
  const int approx = p ? p->approx_leaves : 0;
  const bool bf = !approx && p && (p->prune == 1 || p->prune == 2);
  {
    // the flag, the statistics and (prune) the dropped-candidate bounds and
    // per-query leaf counts cleared in one launch
    FillRanges f{};
    f.p[0] = bad;
    f.n[0] = 1;
    f.p[1] = (uint32_t*)a.stats;
    f.n[1] = 2 * kStatShards * kStatSlots;
    if (bf) {
      f.p[2] = (uint32_t*)at(W_CEV);
      f.n[2] = B;
      f.v[2] = 0xFFFFFFFFu;
      f.p[3] = (uint32_t*)at(W_QCNT);
      f.n[3] = B;
    }
    SOFA_TRY(launch_fill_ranges(f, st));
  }
  hipEvent_t* ev = mem.ev;
  if (ev) (void)hipEventRecord(ev[0], st);
  // approximate search: no radius, prune or fallback applies
  SOFA_TRY(launch_prepare(a, d_q, (p && !approx) ? p->d_radius : nullptr, ix->bins, (float*)at(W_POOL),
                          (double*)at(W_QN), bad, st));
  const bool use_model = !approx && p && p->radius_model && !p->d_radius;
  if (use_model)
    SOFA_TRY(launch_model_radius(p->radius_model, (const float*)at(W_POOL), ix->bins.ncol_pool, B,
                                 (float*)at(W_MLP), a.U0, st));
  const bool has_radius = !approx && p && (p->d_radius || use_model);
  int bf_passes = 0;
  if (approx > 0) {
    // no seed: its leaf (chosen on the FP32 bound) need not be among the
    // scanned ones (chosen on the rounded codes), and its bound would cut them
    a.seed_leaf = 0;
    SOFA_TRY(launch_approx(a, approx, (int32_t*)at(W_APPROX), st, ev));
    SOFA_TRY(launch_finalize(a, d_ids, d_d, status, st, ev));
  } else if (!bf) {
    SOFA_TRY(launch_search(a, d_ids, d_d, status, st, ev));
  } else {
    uint32_t* cev = (uint32_t*)at(W_CEV);
    a.cevmin = cev;  // cleared with the flag above
    SOFA_TRY(launch_front(a, st, ev));
    Bf16Args b{};
    b.prec = p->prune;
    if (b.prec == 2) {
      b.xb = ix->xf.as<uint4>();
      b.meta = ix->xf_meta.as<float4>();
      b.leafmeta = ix->xf_leafmeta.as<float4>();
      b.cscale = ix->xf_cscale.as<float>();
    } else {
      b.xb = ix->xb.as<uint4>();
      b.meta = ix->xb_meta.as<float4>();
      b.leafmeta = ix->xb_leafmeta.as<float4>();
    }
    b.qb = (uint4*)at(W_QB);
    b.qmeta = (float4*)at(W_QMETA);
    b.qscale = (float*)at(W_QSCALE);
    b.perm = (int32_t*)at(W_PERM);
    b.qcount = (uint32_t*)at(W_QCNT);
    b.lcnt = (uint32_t*)at(W_LCNT);
    b.loff = (int64_t*)at(W_LOFF);
    b.lslot = (uint16_t*)at(W_LSLOT);
    b.slotc = (float4*)at(W_SLOTC);
    b.G = (int)((B + kGroup - 1) / kGroup);
    b.cand = (uint32_t*)at(W_CAND);
    b.ccnt = (uint32_t*)at(W_CCNT);
    b.cevmin = cev;
    b.cap = bf16_cap(p, k, B);
    b.counter = (uint32_t*)at(W_BCTR);
    SOFA_TRY(launch_bf16_queries(a, b, st, false));  // qcount cleared above
    const int64_t n_chunks = (ix->N + 255) / 256;
    const int sampling = p->sampling;
    if (sampling == 2) {
      // the query side wrote the first pass's slot terms
      SOFA_TRY(launch_bf16_pass(a, b, 1, 0, 1, n_chunks, 0, true, st, ev ? ev + 7 : nullptr));
      bf_passes = 1;
    } else {
      const bool many = k >= kManyFromK;
      const int* strides = many ? kPassesMany : kPassesFew;
      const int n_passes = many ? (int)(sizeof(kPassesMany) / sizeof(int)) : (int)(sizeof(kPassesFew) / sizeof(int));
      // the (query, leaf) lists are rebuilt from the bounds U of the earlier
      // passes before each of the last two passes of the five-pass schedule
      // (10M x 256, k = 10: 6.5G instead of 7.5G tile pairs) and, without a
      // radius, before the last pass of the three-pass one; a radius near
      // the k = 1 distance leaves nothing to gain there
      const int relist_from = many ? n_passes - 2 : (has_radius ? n_passes : n_passes - 1);
      int64_t prev = 0;
      for (int ps = 0; ps < n_passes; ps++) {
        const int64_t sp = strides[ps];
        if (ps >= relist_from) SOFA_TRY(launch_bf16_relist(a, b, sp, prev, st));
        const int64_t n_sp = (n_chunks + sp - 1) / sp;
        const int64_t n_prev = prev ? (n_chunks + prev - 1) / prev : 0;
        // slot terms already written: by the query side (first pass) or a relist
        SOFA_TRY(launch_bf16_pass(a, b, sp, 0, prev ? 0 : 1, n_sp - n_prev, prev ? (int)(prev / sp) : 0,
                                  ps == 0 || ps >= relist_from, st,
                                  ev ? ev + 7 + 3 * ps : nullptr));
        prev = sp;
      }
      bf_passes = n_passes;
    }
    SOFA_TRY(launch_finalize(a, d_ids, d_d, status, st, ev));
  }
  // the bounds, statuses and counters in one copy to pinned memory
  const size_t back0 = lay.off[W_U], back1 = lay.off[W_BAD] + 4;
  uint8_t* hb = mem.hback;
  if (back1 - back0 > mem.hback_bytes)
    return set_error(SOFA_EINTERNAL, "read-back of %zu bytes, %zu reserved", back1 - back0, mem.hback_bytes);
  SOFA_HIP(hipMemcpyAsync(hb, base + back0, back1 - back0, hipMemcpyDeviceToHost, st));
  SOFA_HIP(hipStreamSynchronize(st));
  const int32_t* hst = reinterpret_cast<const int32_t*>(hb + (lay.off[W_STAT] - back0));
  const float* hu0 = reinterpret_cast<const float*>(hb + (lay.off[W_U0] - back0));
  const uint32_t* hu = reinterpret_cast<const uint32_t*>(hb + (lay.off[W_U] - back0));
  const unsigned hbad = *reinterpret_cast<const unsigned*>(hb + (lay.off[W_BAD] - back0));
  // the counters' shards: sums (slot 4: the maximum)
  unsigned long long hstats[kStatSlots] = {};
  {
    const unsigned long long* sh = reinterpret_cast<const unsigned long long*>(hb + (lay.off[W_STATS] - back0));
    for (int c = 0; c < kStatShards; c++)
      for (int i = 0; i < kStatSlots; i++)
        hstats[i] = i == 4 ? std::max(hstats[i], sh[c * kStatSlots + i]) : hstats[i] + sh[c * kStatSlots + i];
  }
  if (hbad) return set_error(SOFA_EINVAL, "the queries contain non-finite values");
  if (ev && stats.queries == 0) {
    float t[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 6; i++) (void)hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
    stats.ms_prepare = t[0];
    stats.ms_leaf = t[1] + t[3];
    stats.ms_seed = t[2];
    stats.ms_refine = t[4];
    stats.ms_finalize = t[5];
    for (int ps = 0; ps < bf_passes; ps++) {
      float tt = 0, tc = 0;
      (void)hipEventElapsedTime(&tt, ev[7 + 3 * ps], ev[8 + 3 * ps]);
      (void)hipEventElapsedTime(&tc, ev[8 + 3 * ps], ev[9 + 3 * ps]);
      stats.ms_bf16_tiles += tt;
      stats.ms_bf16_refine += tc;
    }
    (void)hipGetLastError();  // timer queries must not leave an error behind
  }
  stats.queries += B;
  stats.leaves_total += B * ix->n_leaves;
  stats.leaves_visited += (int64_t)hstats[0];
  stats.series_lb_checked += (int64_t)hstats[1];
  stats.series_refined += (int64_t)hstats[2];
  stats.series_bf16_checked += (int64_t)hstats[3];
  stats.series_bf16_needed += (int64_t)hstats[5];
  stats.prune_rows_streamed += (int64_t)hstats[6];
  stats.prune_passes += bf_passes;
  stats.max_candidates = std::max<int64_t>(stats.max_candidates, (int64_t)hstats[4]);
  for (int64_t q = 0; q < B; q++) {
    if (hst[q] == 2) stats.overflow_evicted++;
    if (hst[q] == 4) stats.overflow_bf16_drop++;
    if (hst[q] == 5) stats.overflow_band++;
  }
  if (approx > 0) return SOFA_OK;  // whatever the scanned leaves hold is the answer
  std::vector<int64_t> redo, tighten;
  std::vector<float> tighten_r;
  for (int64_t q = 0; q < B; q++) {
    int st_q = hst[q];
    bool has_radius = std::isfinite(hu0[q]);
    float uq = 0.0f;
    memcpy(&uq, &hu[q], 4);
    if (st_q == 4 && bf && depth == 0 && std::isfinite(uq) && uq >= 0.0f) {
      // the prune tier dropped candidates: U is still a valid bound on the
      // k-th distance (k rows were refined), so search once more with it as
      // the radius, on the BF16 tier when the index has it (its bound is
      // tighter than FP8's); that search falls back like any radius search
      tighten.push_back(q);
      tighten_r.push_back((float)(std::sqrt((double)uq) * (1.0 + 1e-6)));
    } else if (st_q == 1 || (st_q >= 2 && has_radius)) {
      redo.push_back(q);
    } else if (st_q >= 2) {
      char* eb = mem.aux + aux.exh;
      uint32_t* pos = (uint32_t*)eb;
      double* d64 = (double*)(eb + (size_t)kExhCap * 4);
      int64_t* id = (int64_t*)(eb + (size_t)kExhCap * 12);
      uint32_t* cnt = (uint32_t*)(eb + (size_t)kExhCap * 20);
      uint32_t s_found = 0;
      if (st_q == 5) {
        // more in-band rows than the finalize ranks in one workgroup, none
        // evicted or dropped: all of them are in the query's list of
        // refined rows, which is ranked in FP64 on its own
        SOFA_TRY(launch_band_rank(a, (int)q, pos, cnt, kExhCap, d64, id, d_ids, d_d, st, &s_found));
      } else {
        // exhaustive pass with the query's valid bound
        SOFA_TRY(launch_exhaustive(a, (int)q, pos, cnt, kExhCap, d64, id, d_ids, d_d, st, &s_found));
        stats.overflow_fallbacks++;
      }
    }
  }
  // search a subset of the queries again (exactness does not depend on the
  // radius or the prune setting) and scatter the results back
  auto research = [&](const std::vector<int64_t>& list, const float* radii, int prune,
                      int sampling) -> sofa_status {
    const int64_t R = (int64_t)list.size();
    if (depth >= kResearchDepth || R > B0)
      return set_error(SOFA_EINTERNAL, "re-search of %lld queries at depth %d", (long long)R, depth + 1);
    // this depth's slice of the fall-back buffers, sized for B0 >= R queries
    char* rs = mem.aux + aux.research[depth];
    float* qcopy = (float*)rs;
    rs += align256((size_t)B0 * ix->n * 4);
    int64_t* rids = (int64_t*)rs;
    rs += align256((size_t)B0 * k * 8);
    float* rd = (float*)rs;
    rs += align256((size_t)B0 * k * 4);
    float* rr = (float*)rs;
    for (int64_t i = 0; i < R; i++)
      SOFA_HIP(hipMemcpyAsync(qcopy + i * ix->n, d_q + list[i] * ix->n, (size_t)ix->n * 4,
                              hipMemcpyDeviceToDevice, st));
    sofa_knn_params p2{};
    if (p) p2.candidate_capacity = p->candidate_capacity;
    p2.prune = prune;
    p2.sampling = sampling;
    if (radii) {
      SOFA_HIP(hipMemcpyAsync(rr, radii, (size_t)R * 4, hipMemcpyHostToDevice, st));
      p2.d_radius = rr;
    }
    sofa_knn_stats s2{};
    SOFA_TRY(knn_impl(ix, qcopy, R, k, &p2, rids, rd, st, mem, s2, B0, depth + 1));
    for (int64_t i = 0; i < R; i++) {
      SOFA_HIP(hipMemcpyAsync(d_ids + list[i] * k, rids + i * k, (size_t)k * 8, hipMemcpyDeviceToDevice, st));
      SOFA_HIP(hipMemcpyAsync(d_d + list[i] * k, rd + i * k, (size_t)k * 4, hipMemcpyDeviceToDevice, st));
    }
    SOFA_HIP(hipStreamSynchronize(st));
    stats.leaves_visited += s2.leaves_visited;
    stats.series_lb_checked += s2.series_lb_checked;
    stats.series_refined += s2.series_refined;
    stats.series_bf16_checked += s2.series_bf16_checked;
    stats.series_bf16_needed += s2.series_bf16_needed;
    stats.prune_rows_streamed += s2.prune_rows_streamed;
    stats.prune_passes += s2.prune_passes;
    stats.overflow_fallbacks += s2.overflow_fallbacks;
    stats.overflow_evicted += s2.overflow_evicted;
    stats.overflow_bf16_drop += s2.overflow_bf16_drop;
    stats.overflow_band += s2.overflow_band;
    stats.radius_fallbacks += s2.radius_fallbacks;
    stats.overflow_retries += s2.overflow_retries;
    return SOFA_OK;
  };
  if (!tighten.empty()) {
    SOFA_TRY(research(tighten, tighten_r.data(), ix->has_bf16 ? 1 : p->prune, 2));
    stats.overflow_retries += (int64_t)tighten.size();
  }
  if (!redo.empty()) {
    // without their radius; without a radius the prune samples first
    const int prune = p ? p->prune : 0;
    const int sampling = p ? (p->sampling == 2 ? 0 : p->sampling) : 0;
    SOFA_TRY(research(redo, nullptr, prune, sampling));
    stats.radius_fallbacks += (int64_t)redo.size();
  }
  return SOFA_OK;
}

extern "C" sofa_status sofa_knn_get_stats(const sofa_workspace* ws, const sofa_index* ix, sofa_knn_stats* out) {
  if (!out) return set_error(SOFA_EINVAL, "null output");
  const sofa_workspace* w = ws ? ws : (ix ? ix->own_ws : nullptr);
  if (!w) {
    memset(out, 0, sizeof *out);
    return SOFA_OK;
  }
  *out = w->stats;
  return SOFA_OK;
}

namespace sofa {
sofa_status launch_all_lb(const SearchArgs& a, float* d_lb, hipStream_t st);
}

extern "C" sofa_status sofa_lower_bounds(const sofa_index* ix, const float* d_queries, int64_t B,
                                         float* d_tables, float* d_lb, void* stream, double* scan_ms) {
  if (!ix || B < 0 || (B > 0 && !d_queries)) return set_error(SOFA_EINVAL, "bad arguments");
  if (B == 0) return SOFA_OK;
  hipStream_t st = S(stream);
  DevBuf qp, pool, qn, tab, sq, u0, bad;
  SOFA_TRY(qp.alloc((size_t)B * ix->n_pad * 4, st));
  SOFA_TRY(pool.alloc((size_t)B * ix->bins.ncol_pool * 4, st));
  SOFA_TRY(qn.alloc((size_t)B * 8, st));
  SOFA_TRY(tab.alloc((size_t)B * kTable * 4, st));
  SOFA_TRY(sq.alloc((size_t)B * 16, st));
  SOFA_TRY(u0.alloc((size_t)B * 4, st));
  SOFA_TRY(bad.alloc(4, st));
  SOFA_TRY(launch_fill_u32(bad.as<uint32_t>(), 0u, 1, st));
  SearchArgs a{};
  a.X = ix->X.as<float>();
  a.words = ix->words.as<uint8_t>();
  a.N = ix->N;
  a.n = ix->n;
  a.n_pad = ix->n_pad;
  a.B = (int)B;
  a.Qp = qp.as<float>();
  a.tables = tab.as<float>();
  a.sq = sq.as<uint4>();
  a.U0 = u0.as<float>();
  a.eta_x = ix->eta_x;
  SOFA_TRY(launch_prepare(a, d_queries, nullptr, ix->bins, pool.as<float>(), qn.as<double>(),
                          bad.as<unsigned>(), st));
  if (d_tables)
    SOFA_HIP(hipMemcpyAsync(d_tables, tab.p, (size_t)B * kTable * 4, hipMemcpyDeviceToDevice, st));
  if (d_lb) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (scan_ms) {
      SOFA_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
      SOFA_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
      SOFA_HIP(hipEventRecord(e0, st));
    }
    sofa_status s = launch_all_lb(a, d_lb, st);
    if (scan_ms) {
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      *scan_ms = ms;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      (void)hipGetLastError();
    }
    SOFA_TRY(s);
  }
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

// the prune tier's lower bound of every (query, row) pair, no pruning
static sofa_status prune_lower_bounds(const sofa_index* ix, const float* d_queries, int64_t B, int prec,
                                      float* d_lb, void* stream) {
  if (!ix || B < 0 || (B > 0 && (!d_queries || !d_lb))) return set_error(SOFA_EINVAL, "bad arguments");
  if (prec == 1 && !ix->has_bf16) return set_error(SOFA_EINVAL, "the index was built without the BF16 copy");
  if (prec == 2 && !ix->has_fp8) return set_error(SOFA_EINVAL, "the index was built without the FP8 copy");
  if (B == 0) return SOFA_OK;
  if (B > 65535) return set_error(SOFA_EINVAL, "B too large");
  hipStream_t st = S(stream);
  const int64_t G = (B + kGroup - 1) / kGroup;
  DevBuf qp, pool, qn, tab, sq, u0, bad, masks, lcnt, loff, lslot, sc, perm, qb, qmeta, qscale,
      ctr, U;
  SOFA_TRY(qp.alloc((size_t)B * ix->n_pad * 4, st));
  SOFA_TRY(pool.alloc((size_t)B * ix->bins.ncol_pool * 4, st));
  SOFA_TRY(qn.alloc((size_t)B * 8, st));
  SOFA_TRY(tab.alloc((size_t)B * kTable * 4, st));
  SOFA_TRY(sq.alloc((size_t)B * 16, st));
  SOFA_TRY(u0.alloc((size_t)B * 4, st));
  SOFA_TRY(U.alloc((size_t)B * 4, st));
  SOFA_TRY(bad.alloc(4, st));
  SOFA_TRY(masks.alloc((size_t)ix->n_blocks * B * 8, st));
  SOFA_TRY(lcnt.alloc((size_t)ix->n_leaves * 4, st));
  SOFA_TRY(loff.alloc((size_t)ix->n_leaves * 8, st));
  SOFA_TRY(lslot.alloc((size_t)ix->n_leaves * B * 2, st));
  SOFA_TRY(sc.alloc((size_t)G * kGroup * 16, st));
  SOFA_TRY(perm.alloc((size_t)B * 4, st));
  SOFA_TRY(qb.alloc((size_t)G * kGroup * ix->n_pad * 2, st));
  SOFA_TRY(qmeta.alloc((size_t)G * kGroup * 16, st));
  SOFA_TRY(qscale.alloc((size_t)G * kGroup * 4, st));
  SOFA_TRY(ctr.alloc(64, st));
  SOFA_TRY(launch_fill_u32(bad.as<uint32_t>(), 0u, 1, st));
  SearchArgs a{};
  a.stats = nullptr;  // no statistics for the inspection call
  a.X = ix->X.as<float>();
  a.N = ix->N;
  a.n = ix->n;
  a.n_pad = ix->n_pad;
  a.L = ix->L;
  a.n_leaves = ix->n_leaves;
  a.n_blocks = ix->n_blocks;
  a.B = (int)B;
  a.Qp = qp.as<float>();
  a.tables = tab.as<float>();
  a.sq = sq.as<uint4>();
  a.U0 = u0.as<float>();
  a.U = U.as<uint32_t>();
  a.masks = masks.as<uint64_t>();
  a.eta_x = ix->eta_x;
  a.lb_f = 1.0f;
  SOFA_TRY(launch_prepare(a, d_queries, nullptr, ix->bins, pool.as<float>(), qn.as<double>(),
                          bad.as<unsigned>(), st));
  SOFA_TRY(launch_fill_u32((uint32_t*)masks.p, 0xFFFFFFFFu, ix->n_blocks * B * 2, st));
  SOFA_TRY(launch_fill_u32(U.as<uint32_t>(), 0x7F800000u, B, st));
  Bf16Args b{};
  b.prec = prec;
  if (prec == 2) {
    b.xb = ix->xf.as<uint4>();
    b.meta = ix->xf_meta.as<float4>();
    b.leafmeta = ix->xf_leafmeta.as<float4>();
    b.cscale = ix->xf_cscale.as<float>();
  } else {
    b.xb = ix->xb.as<uint4>();
    b.meta = ix->xb_meta.as<float4>();
    b.leafmeta = ix->xb_leafmeta.as<float4>();
  }
  b.qb = qb.as<uint4>();
  b.qmeta = qmeta.as<float4>();
  b.qscale = qscale.as<float>();
  b.perm = perm.as<int32_t>();
  b.qcount = u0.as<uint32_t>();  // scratch for the density sort
  b.lcnt = lcnt.as<uint32_t>();
  b.loff = loff.as<int64_t>();
  b.lslot = lslot.as<uint16_t>();
  b.slotc = sc.as<float4>();
  b.G = (int)G;
  b.counter = ctr.as<uint32_t>();
  SOFA_TRY(launch_bf16_queries(a, b, st));
  SOFA_TRY(launch_bf16_dump(a, b, d_lb, st));
  SOFA_HIP(hipStreamSynchronize(st));
  return SOFA_OK;
}

extern "C" sofa_status sofa_bf16_lower_bounds(const sofa_index* ix, const float* d_queries, int64_t B,
                                              float* d_lb, void* stream) {
  return prune_lower_bounds(ix, d_queries, B, 1, d_lb, stream);
}

extern "C" sofa_status sofa_fp8_lower_bounds(const sofa_index* ix, const float* d_queries, int64_t B,
                                             float* d_lb, void* stream) {
  return prune_lower_bounds(ix, d_queries, B, 2, d_lb, stream);
}
