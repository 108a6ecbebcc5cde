/*
 * sofa.h -- C ABI of the MI355X (gfx950) library for exact k-NN search over
 * z-normalised data series with the SFA summary under the GEMINI
 * filter-and-refine scheme (SOFA, Schaefer et al., arXiv 2411.17483).
 *
 * Conventions for every entry point
 *  - Return a sofa_status; no exception or abort crosses the ABI.  On a
 *    non-OK status, sofa_last_error() returns a message for the calling
 *    thread.
 *  - Pointers named d_* are device pointers on the current HIP device; the
 *    caller owns them and the library never frees them.  Pointers without
 *    the prefix are host pointers.
 *  - Series are FP32, row-major, one row of n values per series.  Row ids are
 *    the row numbers of the array given to sofa_build (0-based).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    that stream; the functions that must read a flag back (validation,
 *    fall-back decisions) synchronise that stream before returning, as stated
 *    per function.
 *  - Handles (sofa_bins, sofa_index, sofa_workspace, sofa_radius) are owned
 *    by the caller and released with the matching *_free function.  An index
 *    is read-only after sofa_build; concurrent sofa_knn calls on one index
 *    are allowed when each uses its own workspace and stream.
 */
#ifndef SOFA_H
#define SOFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SOFA_OK = 0,
  SOFA_EINVAL = 1,    /* bad argument: sizes, parameters, non-finite input */
  SOFA_ENOMEM = 2,    /* device allocation failed or workspace too small */
  SOFA_EDEVICE = 3,   /* a HIP runtime call failed */
  SOFA_EBUSY = 4,     /* workspace in use by another call */
  SOFA_EINTERNAL = 5  /* an internal limit was exceeded (message says which) */
} sofa_status;

/* Thread-local message describing the last non-OK status of this thread. */
const char* sofa_last_error(void);

/* ------------------------------------------------------------------------ */
/* Device memory.  By default the library takes device memory with hipMalloc
 * and returns it with hipFree.  sofa_set_allocator installs the caller's
 * functions instead (for example backed by PyTorch's caching allocator, so
 * that one pool owns all device memory); both NULL restore the default.
 *
 *  alloc(bytes, stream, ctx) returns device memory of at least `bytes`
 *    bytes on the current device, aligned to 256 bytes, or NULL (the call
 *    that needed it then fails with SOFA_ENOMEM).  `stream` is the
 *    hipStream_t of the call the memory is for, or NULL for memory that
 *    outlives one call (index arrays, bins, networks).
 *  free(p, stream, ctx) takes back a pointer that alloc returned, with the
 *    same stream.  Before calling it the library synchronises that stream
 *    (the device, for NULL), so no queued kernel still uses the memory.
 *
 * Process-wide and thread-safe.  Memory keeps the allocator it came from: a
 * buffer taken before a change is returned to the functions that gave it.
 * The functions must stay callable until every object (bins, index,
 * workspace, network, server) created while they were installed is freed.
 * They may be called from the serving threads.  Pinned host staging memory
 * is not routed through them.  SOFA_EINVAL if exactly one of the two
 * functions is NULL. */
typedef void* (*sofa_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*sofa_free_fn)(void* p, void* stream, void* ctx);
sofa_status sofa_set_allocator(sofa_alloc_fn alloc, sofa_free_fn free, void* ctx);

/* z-normalisation (Section II, the z-normalised Euclidean distance): each of
 * the m rows of d_in (m x n FP32, device) becomes (x - mean) / sd in d_out
 * (m x n FP32, device; may equal d_in), with the mean and the population
 * standard deviation sd = sqrt(mean((x - mean)^2)) taken in FP64 and the
 * quotient formed in FP64 and rounded to FP32 once.  A row with sd = 0 (a
 * constant row) becomes all zeros.  Non-finite input gives non-finite
 * output (the build and the search then reject it).  1 <= n <= 2^20.
 * Asynchronous on `stream`. */
sofa_status sofa_znormalise(const float* d_in, int64_t m, int32_t n, float* d_out, void* stream);

/* Opaque handles (defined with their entry points below). */
typedef struct sofa_bins sofa_bins;
typedef struct sofa_index sofa_index;
typedef struct sofa_workspace sofa_workspace;
typedef struct sofa_radius sofa_radius;

/* ------------------------------------------------------------------------ */
/* Learned SFA quantisation (Section IV-E, transformation and learned
 * quantisation and feature selection; Algorithm 1, MCB).
 *
 * The pool holds the real and imaginary parts of the orthonormal DFT
 * coefficients k = 1..pool (DC omitted: it is zero for z-normalised series,
 * Section IV-E, Eq. 1); pool value 2(k-1) is Re X_k, 2(k-1)+1 is Im X_k.
 * MCB keeps the l pool values of largest variance over the sample (ties: lower pool
 * index first), in decreasing-variance order, and learns alpha-1 breakpoints
 * per kept value: equi-depth beta(a) = v_(floor(a*m/alpha)) of the sorted
 * sample, or equi-width beta(a) = min + a*(max-min)/alpha.  Bins are
 * half-open [beta(a-1), beta(a)); the outer bins are open to -inf / +inf. */
typedef struct {
  int32_t l;       /* kept values per word, 1..16 (default 16) */
  int32_t alpha;   /* symbols per value, 1..256 (default 256) */
  int32_t pool;    /* DFT coefficients in the pool, 1..32 and <= n/2-1 (default 16) */
  int32_t binning; /* 0 = equi-depth (default), 1 = equi-width */
  /* 0 = SFA (default: Section IV-E, Algorithms 1-2).  1 = iSAX (Section
   * IV-D): the means of l equal segments (n % l == 0), each scaled by
   * sqrt(n/l) so that the basis rows are orthonormal, kept in time order and
   * quantised with the alpha-1 equal-depth quantiles of N(0,1) (scaled the
   * same way); `pool` and `binning` are ignored (the pool becomes the l
   * segment values) and the lower bound weighs every value by 1 instead of
   * SFA's 2.  The whole path (tables, envelopes, scans, prune tiers) is the
   * same for both. */
  int32_t summary;
  /* SFA only: 0 (default) keeps the l pool values of largest variance
   * (Algorithm 1); 1 keeps the first l pool values (Re/Im of k = 1, 2, ...),
   * the variant without variance selection of the TLB ablation (Section V-E) */
  int32_t selection;
  /* sofa_learn_bins only: 0 (default) the rows are z-normalised already;
   * 1 z-normalises each sampled row on the device first (as
   * sofa_znormalise), for bins that match an index built with znormalise */
  int32_t znormalise;
} sofa_bin_params;

/* Learns bins from the stride sample of m rows of d_series (rows
 * floor(i*N/m), i < m), all arithmetic in FP64 on the device: DFT of the
 * sample, variance per pool value, top-l selection, sort and breakpoints.
 * d_series: N x n FP32 device array.  Requires 1 <= m <= N, m <= 2^25,
 * n >= 2*pool+2, n % 4 == 0, n <= 1024.  Synchronous (returns when *out is
 * complete). */
sofa_status sofa_learn_bins(const float* d_series, int64_t N, int32_t n, int64_t m,
                            const sofa_bin_params* params, void* stream, sofa_bins** out);

/* Builds a bins object from given values (e.g. saved bins): sel[l] pool
 * indices, beta[l * (alpha-1)] FP64 breakpoints row-major, var[2*pool] the
 * pool variances (may be NULL).  Host pointers. */
sofa_status sofa_bins_create(int32_t n, const sofa_bin_params* params, const int32_t* sel,
                             const double* beta, const double* var, sofa_bins** out);

/* Copies the learned values out to host arrays (any pointer may be NULL):
 * sel[l], beta[l*(alpha-1)], var[2*pool]; params receives l, alpha, pool,
 * binning; n receives the series length. */
sofa_status sofa_bins_get(const sofa_bins* bins, sofa_bin_params* params, int32_t* n,
                          int32_t* sel, double* beta, double* var);

/* Releases the handle and the device memory it holds.  NULL does nothing. */
void sofa_bins_free(sofa_bins* bins);

/* Projection onto the Fourier pool (Algorithm 2, step 1) and quantisation
 * (Algorithm 2, step 2) of m arbitrary rows, for inspection and checks:
 *  d_pool  (nullable) m x 2*pool FP32: every pool value of every row;
 *  d_sel   (nullable) m x 16 FP32: the l kept values in word order
 *          (columns >= l are zero);
 *  d_words (nullable) m x 16 uint8: the SFA word (bytes >= l are zero).
 * The projection runs on the matrix cores (FP32 MFMA) against a partial DFT
 * basis; sofa_bins_get_eta() states its error bound.  Asynchronous. */
sofa_status sofa_transform(const sofa_bins* bins, const float* d_x, int64_t m,
                           float* d_pool, float* d_sel, uint8_t* d_words, void* stream);

/* Error bound of the FP32 projection: for a row x, every computed pool value
 * c satisfies |c - c_exact| <= eta_per_norm * ||x||_2 (+ 1e-30). */
double sofa_bins_eta_per_norm(const sofa_bins* bins);

/* ------------------------------------------------------------------------ */
/* Index (Section IV-G, SOFA index; the MESSI tree of Sections IV-A and IV-B is
 * replaced by fixed-size leaves over a sorted flat array).
 *
 * sofa_build SFA-transforms every row, sorts the rows by a key that
 * interleaves the symbols' leading bits (most significant bit first, values
 * in word order, like the iSAX-style refinement of Section IV-B), cuts the
 * sorted order into leaves of leaf_size rows, and stores per leaf the
 * smallest and largest symbol of each word position (its envelope).  It
 * keeps its own permuted copy of the rows, so d_series may be freed after
 * the call returns. */
typedef struct {
  int32_t leaf_size; /* rows per leaf, a multiple of 64 in [64, 4096] (default 256) */
  /* bit 0: keep a BF16 copy for the batched-distance prune (n <= 256);
   * bit 1: keep an FP8 (OCP e4m3) copy (n <= 1024), scaled by a power of two
   * per 256-row chunk so that every value fits the e4m3 range.  Both need
   * leaf_size to be a multiple of 256. */
  int32_t precision;
  /* sort key: 0 (default) spends 8/8/8/8, 4/4/4/4, 2 x 8 key bits on word
   * positions 0-3, 4-7, 8-15 (positions are in decreasing-variance order),
   * interleaved most significant first; 1 spends 4 bits on every position */
  int32_t key_scheme;
  /* 0 (default): the rows are z-normalised already and are used as given.
   * 1: the build z-normalises every row on the device first (as
   * sofa_znormalise, into a temporary N x n copy, so the build briefly needs
   * that much more device memory); the index then holds the normalised rows. */
  int32_t znormalise;
} sofa_build_params;

/* d_series: N x n FP32 device array, z-normalised (or raw with znormalise
 * set).  Non-finite values give SOFA_EINVAL.  N must be < 2^31.
 * Synchronous (returns when the index is complete). */
sofa_status sofa_build(const sofa_bins* bins, const float* d_series, int64_t N, int32_t n,
                       const sofa_build_params* params, void* stream, sofa_index** out);

typedef struct {
  int64_t N;
  int32_t n, n_pad, leaf_size, l, alpha;
  int64_t n_leaves;
  int64_t device_bytes; /* device memory held by the index */
  double eta_x;         /* projection error bound used for the data words */
  int32_t has_bf16;
  int32_t has_fp8;
} sofa_index_info;

/* Fills *info from the index on the host, with no device work.  SOFA_EINVAL
 * if either pointer is NULL. */
sofa_status sofa_index_get_info(const sofa_index* index, sofa_index_info* info);

/* Copies the index layout to caller device arrays (any may be NULL):
 * d_words N x 16 uint8 in leaf order, d_ids N int32 (row id of each leaf-order
 * position), d_env n_leaves x 32 uint8 (16 lower then 16 upper symbols),
 * d_keys N uint64 sort keys in leaf order.  Asynchronous. */
sofa_status sofa_index_export(const sofa_index* index, uint8_t* d_words, int32_t* d_ids,
                              uint8_t* d_env, uint64_t* d_keys, void* stream);

/* Releases the index, its device arrays and its own workspace.  Work queued
 * on it must have finished.  NULL does nothing. */
void sofa_index_free(sofa_index* index);

/* ------------------------------------------------------------------------ */
/* Exact k-NN (Section II similarity search and its k-NN extension; GEMINI,
 * Section II-A; SFA lower bound, Eq. 2 and Eq. 3).
 *
 * Result: for every query, the k rows with the smallest squared Euclidean
 * distance, ranked by (FP64 squared distance summed in time order, row id)
 * ascending; d_ids B x k int64 row ids, d_dists B x k FP32 distances (not
 * squared).  The GPU filters with the SFA lower bound, refines survivors
 * with FP32 distances, and recomputes the candidates inside the FP32 error
 * band of the k-th distance in FP64, so ids equal those of an FP64 brute
 * force and dists are within 1e-6 relative of it.
 *
 * A workspace holds the per-batch scratch memory.  Create one per concurrent
 * stream; sofa_knn returns SOFA_ENOMEM when a batch does not fit its byte
 * limit (the serving layer treats that as "not admitted"). */
/* max_bytes = 0: no limit (grows on demand). */
sofa_status sofa_workspace_create(int64_t max_bytes, sofa_workspace** out);
/* Bytes a batch of B queries with k needs on index (no allocation): the
 * batch's regions and its fall-back buffers (the copies of re-searched
 * queries and the exhaustive pass's lists), which are reserved with it so
 * that a fall-back never allocates. */
sofa_status sofa_workspace_bytes_for(const sofa_index* index, int64_t B, int32_t k,
                                     int32_t prune, int64_t* bytes);
void sofa_workspace_free(sofa_workspace* ws);

typedef struct {
  /* Batched-distance prune before the FP32 refinement: 0 off, 1 BF16 MFMA
   * (needs an index built with precision bit 0), 2 FP8 e4m3 MFMA (needs
   * precision bit 1).  The prune discards a row only when a rigorous lower
   * bound of its distance exceeds the query's bound, so results are the same
   * for every setting. */
  int32_t prune;
  /* Nullable device array of B radii (distance units, not squared).  A
   * finite radius seeds the best-so-far bound with radius^2 so the first
   * pass already prunes.  A query for which fewer than k results lie within
   * its radius is searched again without it, so results stay exact. */
  const float* d_radius;
  /* Nullable learned-radius model (its k must equal k): when set and
   * d_radius is NULL, the radii come from the model applied to the queries'
   * Fourier pool values, computed inside the call. */
  const sofa_radius* radius_model;
  /* 0 (default): seed the bound with the exact distances of the leaf with
   * the smallest envelope bound (the approximate first answer of Section
   * IV-C); 1: skip that seed. */
  int32_t no_seed_leaf;
  sofa_workspace* ws; /* NULL: the index's own workspace (one caller at a time) */
  /* Candidate slots per query in the workspace, and the length of each
   * query's list of refined rows (0 = library defaults: candidates for the
   * BF16 prune 32768, or 2^18 for k > 16 within 1 GiB per batch; for the
   * FP8 prune 2^18, or 2^20 for k > 16 within 2 GiB per batch; never below
   * 32768.  Refined rows: 32768, or 2^18 for k > 16 within 1 GiB per batch,
   * never below 65536).  A smaller value only costs time: when in-band candidates are
   * dropped the query is searched again with its tightened bound, or finished
   * by an exhaustive pass, so results stay exact. */
  int32_t candidate_capacity;
  /* BF16/FP8 prune only: 0 (default) and 1 run the 256-row chunks in passes
   * of decreasing stride (1024, 32, 1 for k <= 3; 2048, 256, 32, 4, 1 from
   * k = 4 on), each selecting candidates with the bound the earlier passes
   * established, with the (query, leaf) lists rebuilt from that bound before
   * the last passes; 2 runs one pass over all chunks (best when the radius
   * is tight, e.g. k = 1). */
  int32_t sampling;
  /* 0 (default): exact search.  1..64: APPROXIMATE search, no exactness
   * guarantee: the first answer of Section IV-C (scan the leaf of smallest
   * lower bound) widened to the approx_leaves leaves of smallest envelope
   * bound per query, whose rows get exact distances and the FP64 ranking;
   * the k best of those rows are returned (ids -1 / +inf distances when they
   * hold fewer than k rows).  prune, radii and fallbacks do not apply.  The
   * paper names approximate search as future work (Section VI). */
  int32_t approx_leaves;
  /* 0 (default): the queries are z-normalised already.  1: each query is
   * z-normalised on the device first (as sofa_znormalise, into the
   * workspace); the caller's array is left unchanged. */
  int32_t znormalise;
} sofa_knn_params;

/* d_queries: B x n FP32 device array, z-normalised.  1 <= k <= min(N, 100).
 * Non-finite query values give SOFA_EINVAL.  Synchronises `stream` before
 * returning (it reads per-query status flags to run fall-backs). */
sofa_status sofa_knn(const sofa_index* index, const float* d_queries, int64_t B, int32_t k,
                     const sofa_knn_params* params, int64_t* d_ids, float* d_dists,
                     void* stream);

/* The search of sofa_knn for callers that cannot allocate device memory
 * (code that forbids hipMalloc, tight serving loops, harnesses without an
 * allocator).  Same arguments, checks and results as sofa_knn; params->ws
 * must be NULL.  It calls no hipMalloc, hipFree or allocator hook: every
 * device buffer of the batch (its regions and the fall-back buffers) lies in
 * one static array of SOFA_NOALLOC_SCRATCH_BYTES per GPU, which the library
 * holds on each device it runs on until the process ends; the host reads its
 * status flags back into a static host buffer.  A batch that needs more than
 * the array (sofa_workspace_bytes_for, with the radius model's scratch), or
 * more than SOFA_NOALLOC_MAX_QUERIES queries, gives SOFA_ENOMEM before any
 * device work.  Calls share the array, so they are serialised inside the
 * library (across threads and devices) and each one synchronises `stream`
 * before returning; two processes each hold their own array.  No stage
 * timers or counters are recorded (sofa_knn_get_stats does not see these
 * calls). */
#define SOFA_NOALLOC_SCRATCH_BYTES (128ll << 20)
#define SOFA_NOALLOC_MAX_QUERIES 4096
sofa_status sofa_knn_noalloc(const sofa_index* index, const float* d_queries, int64_t B, int32_t k,
                             const sofa_knn_params* params, int64_t* d_ids, float* d_dists,
                             void* stream);

/* Counters of the last sofa_knn call on a workspace (or the index's own). */
typedef struct {
  int64_t queries;
  int64_t leaves_total;       /* B * n_leaves */
  int64_t leaves_visited;     /* (query, leaf) pairs that passed the envelope bound */
  int64_t series_lb_checked;  /* word lower bounds evaluated */
  int64_t series_refined;     /* FP32 exact distances computed */
  int64_t series_bf16_checked;/* batched-distance bounds evaluated */
  int64_t radius_fallbacks;   /* queries searched again without their radius */
  int64_t overflow_fallbacks; /* queries finished by the exhaustive pass */
  double ms_total;            /* wall time of the call on its stream (HIP events) */
  /* time of each stage of the first pass, from HIP events recorded on the
   * call's stream around the launches: query preparation (padding, MFMA
   * projection, tables), envelope bounds (both passes), seed, refinement,
   * final FP64 ranking */
  double ms_prepare, ms_leaf, ms_seed, ms_refine, ms_finalize;
  /* with the BF16 prune, the refinement stage splits into the MFMA tile
   * kernel(s) and the exact refinement of their candidates */
  double ms_bf16_tiles, ms_bf16_refine;
  /* queries whose batched-distance candidates overflowed, by cause: a
   * candidate inside the final band was evicted or dropped; a BF16/FP8
   * candidate was dropped; the final band held more rows than the ranking
   * buffer (1,024 rows; without a radius such a band is ranked in FP64 from
   * the query's list of refined rows, with no exhaustive pass).
   * max_candidates: the largest BF16/FP8 candidate count of one query in
   * one pass. */
  int64_t overflow_evicted, overflow_bf16_drop, overflow_band, max_candidates;
  /* queries whose BF16/FP8 candidates overflowed and that were searched once
   * more with their tightened bound as the radius (on the BF16 tier when the
   * index has it) before any exhaustive pass */
  int64_t overflow_retries;
  /* (query, row) pairs the batched-distance tiles had to evaluate: the rows
   * of each leaf times the queries on the leaf's list when its pass ran
   * (series_bf16_checked counts them in whole groups of 64 queries) */
  int64_t series_bf16_needed;
  /* launches of the batched-distance tile kernel (one per sampled pass) */
  int64_t prune_passes;
  /* rows of the BF16/FP8 copy the tile kernel streamed from memory: each
   * 256-row chunk with a non-empty query list, once per pass (times 2 n_pad
   * bytes for BF16, n_pad for FP8, these are the bytes it must read) */
  int64_t prune_rows_streamed;
} sofa_knn_stats;

/* Copies the counters of the last call on ws (or, with ws NULL, on the
 * index's own workspace) to *out; all zero when no call has run there.
 * SOFA_EINVAL if out is NULL. */
sofa_status sofa_knn_get_stats(const sofa_workspace* ws, const sofa_index* index,
                               sofa_knn_stats* out);

/* Lower-bound tables and bounds for inspection: for each query, the FP32
 * table T[j][s] = w_j * mind_j(s, v_j)^2 over word position j and symbol s
 * (Eq. 3, widened by the projection error bounds and rounded down), and the
 * word lower bound of every (query, leaf-order row) pair: a full scan of the
 * packed words (16 B per row) with the tables in LDS.
 *  d_tables (nullable) B x 16 x 256 FP32;  d_lb (nullable) B x N FP32;
 *  scan_ms (nullable): duration of the word scan kernel alone, from HIP
 *  events on `stream`.  Synchronous. */
sofa_status sofa_lower_bounds(const sofa_index* index, const float* d_queries, int64_t B,
                              float* d_tables, float* d_lb, void* stream, double* scan_ms);

/* ------------------------------------------------------------------------ */
/* Learned radius.  A small network predicts ln(d_k), the logarithm of a
 * query's k-th nearest-neighbour distance, from the query's Fourier pool
 * values; sofa_knn seeds its best-so-far bound with the predicted radius so
 * the first pass already prunes, and searches a query again without the
 * radius when fewer than k results fall inside it (results stay exact).
 *
 * Network: y = W3 g(W2 g(W1 xs + b1) + b2) + b3 with xs the standardised
 * input ((x - mu) / sd per feature), g(z) = z Phi(z) (exact GELU).  Weights
 * W1 [H1][D], W2 [H2][H1], W3 [H2] are kept in FP32 (master) and used
 * rounded to BF16 (round to nearest even); biases stay FP32; all sums
 * accumulate in FP32.  Training minimises the mean squared error to ln(d_k)
 * with Adam (Kingma & Ba 2015, bias-corrected) on the FP32 master; gradients
 * are taken at the BF16-rounded weights.  Parameters are one flat FP32
 * vector: W1, b1, W2, b2, W3, b3 (74,497 values for D=32, H1=H2=256). */
typedef struct {
  int32_t in_dim;   /* D: features = the 2*pool Fourier pool values (default 32) */
  int32_t hidden1;  /* H1 (default 256) */
  int32_t hidden2;  /* H2 (default 256) */
  int32_t k;        /* the k the model predicts d_k for */
  float lr, beta1, beta2, eps;  /* Adam (defaults 1e-3, 0.9, 0.999, 1e-8 when 0) */
  uint64_t seed;    /* initial weights: Philox4x32-10 normal draws, He scaling */
} sofa_radius_params;

/* Creates a network of the given sizes (0 takes the default; D in [1, 64],
 * H1 and H2 in [1, 4096], 1 <= k <= 100, else SOFA_EINVAL), its weights
 * drawn from seed, standardisation mu = 0 and sd = 1, Adam moments zero.
 * Allocates device memory (SOFA_ENOMEM or SOFA_EDEVICE on failure, with
 * *out NULL) and synchronises the device. */
sofa_status sofa_radius_create(const sofa_radius_params* params, sofa_radius** out);
/* Releases the network and its device memory.  NULL does nothing. */
void sofa_radius_free(sofa_radius* model);
/* The length of the flat parameter vector (0 for NULL). */
int64_t sofa_radius_num_params(const sofa_radius* model);

/* Host copies in and out: params[num_params] FP32 master, mu[D], sd[D],
 * margin (log units), step (Adam steps taken).  Any pointer may be NULL. */
sofa_status sofa_radius_get(const sofa_radius* model, float* params, float* mu, float* sd,
                            float* margin, int64_t* step);
sofa_status sofa_radius_set(sofa_radius* model, const float* params, const float* mu,
                            const float* sd, const float* margin, const int64_t* step);

/* Feature standardisation from n training rows d_feat (n x D, device):
 * mu = mean, sd = population standard deviation (1 where it is 0). */
sofa_status sofa_radius_standardize(sofa_radius* model, const float* d_feat, int64_t n,
                                    void* stream);

/* Gradients of the loss mean_b (y_b - t_b)^2 over a batch (no update):
 * d_grad[num_params] FP32, d_loss (nullable) the loss.  B <= 65536. */
sofa_status sofa_radius_gradients(sofa_radius* model, const float* d_feat, const float* d_target,
                                  int64_t B, float* d_grad, float* d_loss, void* stream);

/* One training step: forward, backward and one Adam update. */
sofa_status sofa_radius_train_step(sofa_radius* model, const float* d_feat,
                                   const float* d_target, int64_t B, float* d_loss,
                                   void* stream);

/* Epochs of train steps over n rows in order, in batches of `batch`;
 * h_epoch_loss[epochs] (nullable) receives the mean batch loss per epoch.
 * Synchronous. */
sofa_status sofa_radius_fit(sofa_radius* model, const float* d_feat, const float* d_target,
                            int64_t n, int32_t epochs, int32_t batch, float* h_epoch_loss,
                            void* stream);

/* Predicted ln(d_k) (no margin), d_y[B]. */
sofa_status sofa_radius_forward(const sofa_radius* model, const float* d_feat, int64_t B,
                                float* d_y, void* stream);

/* Margin = the given quantile of the residuals t - y over held-out rows;
 * the radius is exp(y + margin).  Synchronous. */
sofa_status sofa_radius_calibrate(sofa_radius* model, const float* d_feat, const float* d_target,
                                  int64_t n, double quantile, void* stream);

/* Radii exp(y + margin) for B feature rows. */
sofa_status sofa_radius_predict(const sofa_radius* model, const float* d_feat, int64_t B,
                                float* d_radius, void* stream);

/* Batched-distance lower bounds for inspection (index built with the BF16
 * copy): for every (query, leaf-order row) pair the bound
 *   |q|^2 + |x|^2 - 2 (P + g|qh||xh| + |q| r_x + r_q |xh|)
 * that the BF16 prune compares with the k-th-distance bound, computed by the
 * same MFMA kernel the search uses (P: FP32 accumulation of the BF16
 * products, qh/xh the BF16 copies, r = |x - xh|).  d_lb: B x N FP32. */
sofa_status sofa_bf16_lower_bounds(const sofa_index* index, const float* d_queries, int64_t B,
                                   float* d_lb, void* stream);

/* The same for the FP8 tier (index built with precision bit 1): xh =
 * s_c e4m3(x / s_c) with s_c the power-of-two scale of the row's 256-row
 * chunk, qh = s_q e4m3(q / s_q), P the FP32 accumulation of the e4m3
 * products (exact in FP32), and the bound
 *   |q|^2 + |x|^2 - 2 (s_q s_c P + g|qh||xh| + |q| r_x + r_q |xh|)
 * with g = (n_pad + 64) 2^-23.  d_lb: B x N FP32. */
sofa_status sofa_fp8_lower_bounds(const sofa_index* index, const float* d_queries, int64_t B,
                                  float* d_lb, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching (not part of the paper,
 * which answers one query at a time, Section V; the loop only schedules
 * sofa_knn calls, so every answer is the exact one).
 *
 * Requests carry one query each, for any registered collection and any k.
 * They wait in a queue per collection.  `slots` batches run at once, each on
 * its own HIP stream (default priority) with its own workspace and host
 * thread, so their kernels overlap on the device.  A free slot takes, among
 * the collections with fewer than per_collection batches in flight, the
 * queue whose oldest request is oldest overall, up to max_batch of its
 * requests, and admits the batch only if the server's device memory stays
 * within memory_budget: the slots' staging buffers, plus per slot what its
 * workspace holds (a workspace keeps the capacity of its largest batch,
 * fall-back buffers included; a running slot is charged the larger of that
 * and its batch's bytes, sofa_workspace_bytes_for with the batch's radius
 * model).  When a batch does not fit, the idle slots free their workspaces;
 * then the batch is halved; then it waits for memory to free.  A query that
 * alone exceeds the budget fails with SOFA_ENOMEM.  Requests
 * that arrive while batches run join the next batch of their collection.
 * A batch runs at the largest k of its requests and each request keeps its
 * first k results, which are exactly its own k nearest (the ranking is the
 * total order on (distance, id)): a result does not depend on the batch it
 * ran in.
 *
 * The indexes and radius models stay owned by the caller and must outlive
 * the server.  Threads: submit and wait may be called from any thread. */
typedef struct sofa_server sofa_server;

typedef struct {
  int32_t slots;         /* concurrent batches (default 4, at most 16) */
  int32_t max_batch;     /* queries per batch (default 256) */
  int64_t memory_budget; /* device bytes of the server: staging buffers and
                          * the slots' workspaces (default 8 GiB) */
  int32_t per_collection; /* batches of one collection in flight (default 1) */
} sofa_server_params;

typedef struct {
  int64_t submitted, completed, batches;
  int64_t max_batch;             /* largest batch run */
  int64_t in_flight_bytes_peak;  /* largest device bytes charged to the server */
  int64_t memory_waits;          /* batches halved or delayed for memory */
  double busy_ms;                /* summed wall time of the batches */
  /* algorithmic HBM bytes of the batches' searches on the prune tiers: the
   * prune-copy rows each search streamed (prune_rows_streamed of
   * sofa_knn_stats times the row's bytes) plus 4 n_pad bytes for every row
   * it refined exactly (series_refined) */
  double hbm_bytes;
} sofa_server_stats;

/* Creates a server with the given parameters (NULL: defaults) and starts no
 * thread until the first request.  SOFA_EINVAL for slots above 16 or
 * max_batch above 65535; SOFA_ENOMEM if the staging buffers cannot be had. */
sofa_status sofa_server_create(const sofa_server_params* params, sofa_server** out);
/* Registers an index; prune as in sofa_knn_params (the index must hold the
 * copy).  n <= 1024.  *out_id is the collection id used by submit. */
sofa_status sofa_server_add_collection(sofa_server* server, const sofa_index* index, int32_t prune,
                                       int32_t* out_id);
/* Uses a learned-radius model for the collection's queries with k = the
 * model's k (queries with other k run without a radius). */
sofa_status sofa_server_set_model(sofa_server* server, int32_t collection, const sofa_radius* model);
/* h_query: n FP32 host values (z-normalised), copied before returning.
 * 1 <= k <= min(N, 100).  *ticket identifies the request. */
sofa_status sofa_server_submit(sofa_server* server, int32_t collection, const float* h_query,
                               int32_t k, int64_t* ticket);
/* Waits for a request (timeout_ms < 0: no limit; SOFA_EBUSY on timeout, the
 * ticket stays valid) and copies its k ids (int64, original rows) and
 * distances (FP32, ascending by (distance, id)) to host arrays (either may
 * be NULL).  times_ms (nullable, 3 doubles): submit-to-result latency,
 * submit-to-start queueing, size of the batch it ran in.  The ticket is
 * released on return (except on timeout). */
sofa_status sofa_server_wait(sofa_server* server, int64_t ticket, int64_t* h_ids, float* h_dists,
                             double* times_ms, int32_t timeout_ms);
sofa_status sofa_server_get_stats(sofa_server* server, sofa_server_stats* out);
/* Finishes the queued requests, stops the slots and frees the server. */
void sofa_server_free(sofa_server* server);

#ifdef __cplusplus
}
#endif

#endif /* SOFA_H */
