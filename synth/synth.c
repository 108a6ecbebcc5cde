/*
 * synth.c -- seeded synthetic data series shaped like the paper's workloads.
 *
 * This module only makes inputs.  It holds none of the search method's
 * arithmetic and is shared, as an input source, by the CPU oracle checks and
 * by the GPU library's tests and benchmark.
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), a counter-based
 * generator: every value is a pure function of (seed, stream tag, row,
 * block), so rows can be generated in any order by any number of threads and
 * the bits never change.  Normal deviates use the Box-Muller transform.
 *
 * Generators (per row, each z-normalised in FP64 with the population
 * standard deviation, then stored as FP32):
 *   random walk (RW):  x_t = sum_{s<=t} z_s,  z ~ N(0,1)
 *   high frequency (HF): x_t = sum_{i=1..8} sin(2 pi f_i t / n + phi_i) + e_t,
 *       f_i ~ U(0, n/2) cycles per series, phi_i ~ U(0, 2 pi), e ~ N(0, 0.5^2)
 *   mix: row i is RW when i is even, HF when i is odd.
 *   band-limited high frequency (BAND): as HF with f_i ~ U(4, 16) cycles per
 *       series, energy that a 16-value Fourier word holds but that segment
 *       means of 16 samples (n = 256) largely average away.
 * Queries: source row j ~ U{0..N-1}; q = znorm(x_j + N(0, sigma^2)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SYN_PI 3.14159265358979323846

typedef struct { uint32_t v[4]; } syn_u4;

static inline uint32_t syn_mulhi(uint32_t a, uint32_t b, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *lo = (uint32_t)p;
  return (uint32_t)(p >> 32);
}

/* Philox4x32 with 10 rounds: multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key
 * increments 0x9E3779B9 / 0xBB67AE85 (the published constants). */
static syn_u4 syn_philox(syn_u4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; r++) {
    uint32_t lo0, lo1;
    uint32_t hi0 = syn_mulhi(0xD2511F53u, c.v[0], &lo0);
    uint32_t hi1 = syn_mulhi(0xCD9E8D57u, c.v[2], &lo1);
    syn_u4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

typedef struct {
  uint32_t k0, k1;
  uint64_t row;
} syn_stream;

static syn_stream syn_make_stream(uint64_t seed, uint32_t tag, uint64_t row) {
  syn_stream s;
  s.k0 = (uint32_t)seed;
  s.k1 = (uint32_t)(seed >> 32) ^ (tag * 0x85EBCA6Bu);
  s.row = row;
  return s;
}

static syn_u4 syn_block(const syn_stream* s, uint32_t block) {
  syn_u4 c;
  c.v[0] = block;
  c.v[1] = 0x5EED5EEDu;
  c.v[2] = (uint32_t)s->row;
  c.v[3] = (uint32_t)(s->row >> 32);
  return syn_philox(c, s->k0, s->k1);
}

/* uniform in [0,1) with 53 random bits from two 32-bit words */
static inline double syn_u01(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* two standard normal deviates from one Philox block (Box-Muller) */
static inline void syn_normal2(const syn_stream* s, uint32_t block, double* z0, double* z1) {
  syn_u4 r = syn_block(s, block);
  double u1 = 1.0 - syn_u01(r.v[0], r.v[1]); /* (0,1] */
  double u2 = syn_u01(r.v[2], r.v[3]);
  double rad = sqrt(-2.0 * log(u1));
  double th = 2.0 * SYN_PI * u2;
  *z0 = rad * cos(th);
  *z1 = rad * sin(th);
}

/* n normals into z (n even or odd) */
static void syn_normals(const syn_stream* s, int n, double* z) {
  for (int t = 0; t < n; t += 2) {
    double a, b;
    syn_normal2(s, (uint32_t)(t / 2), &a, &b);
    z[t] = a;
    if (t + 1 < n) z[t + 1] = b;
  }
}

static void syn_znorm_store(const double* x, int n, float* out) {
  double mu = 0.0;
  for (int t = 0; t < n; t++) mu += x[t];
  mu /= n;
  double var = 0.0;
  for (int t = 0; t < n; t++) var += (x[t] - mu) * (x[t] - mu);
  var /= n;
  double sd = sqrt(var);
  for (int t = 0; t < n; t++) out[t] = (float)(sd > 0.0 ? (x[t] - mu) / sd : 0.0);
}

static void syn_rw_row(uint64_t seed, uint64_t row, int n, double* buf, float* out) {
  syn_stream s = syn_make_stream(seed, 1u, row);
  syn_normals(&s, n, buf);
  double acc = 0.0;
  for (int t = 0; t < n; t++) {
    acc += buf[t];
    buf[t] = acc;
  }
  syn_znorm_store(buf, n, out);
}

/* f_i ~ U(f_lo, f_hi) cycles per series */
static void syn_sines_row(uint64_t seed, uint64_t row, int n, double f_lo, double f_hi, double* buf,
                          float* out) {
  syn_stream sp = syn_make_stream(seed, 2u, row); /* frequencies and phases */
  syn_stream sn = syn_make_stream(seed, 3u, row); /* additive noise */
  syn_normals(&sn, n, buf);
  for (int t = 0; t < n; t++) buf[t] *= 0.5;
  for (int i = 0; i < 8; i++) {
    syn_u4 r = syn_block(&sp, (uint32_t)i);
    double f = f_lo + syn_u01(r.v[0], r.v[1]) * (f_hi - f_lo);
    double ph = syn_u01(r.v[2], r.v[3]) * 2.0 * SYN_PI;
    double w = 2.0 * SYN_PI * f / n;
    /* sin(w t + ph) by the angle-addition recurrence, re-anchored with a
     * direct evaluation every 32 steps */
    double cw = cos(w), sw = sin(w);
    double sv = 0.0, cv = 0.0;
    for (int t = 0; t < n; t++) {
      if ((t & 31) == 0) {
        sv = sin(w * t + ph);
        cv = cos(w * t + ph);
      }
      buf[t] += sv;
      double ns = sv * cw + cv * sw;
      double nc = cv * cw - sv * sw;
      sv = ns;
      cv = nc;
    }
  }
  syn_znorm_store(buf, n, out);
}

static void syn_hf_row(uint64_t seed, uint64_t row, int n, double* buf, float* out) {
  syn_sines_row(seed, row, n, 0.0, 0.5 * n, buf, out);
}

static void syn_band_row(uint64_t seed, uint64_t row, int n, double* buf, float* out) {
  syn_sines_row(seed, row, n, 4.0, 16.0, buf, out);
}

/* kind: 0 = random walk, 1 = high frequency, 2 = mix (even rows RW, odd HF),
 * 3 = band-limited high frequency.
 * Writes rows [row0, row0+rows) of the collection into out (rows x n). */
void syn_generate(float* out, long long row0, long long rows, int n, int kind,
                  unsigned long long seed, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* buf = (double*)malloc(sizeof(double) * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(static, 1024)
#endif
    for (long long r = 0; r < rows; r++) {
      uint64_t row = (uint64_t)(row0 + r);
      int hf = (kind == 1) || (kind == 2 && (row & 1));
      if (kind == 3)
        syn_band_row(seed, row, n, buf, out + (size_t)r * n);
      else if (hf)
        syn_hf_row(seed, row, n, buf, out + (size_t)r * n);
      else
        syn_rw_row(seed, row, n, buf, out + (size_t)r * n);
    }
    free(buf);
  }
}

/* Noisy-copy queries: for query b, source row j = floor(u * N) with u from
 * stream tag 4, then q = znorm(x_j + sigma * z) with z from stream tag 5. */
void syn_queries(const float* X, long long N, int n, long long B, double sigma,
                 unsigned long long seed, float* Q, long long* src, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* buf = (double*)malloc(sizeof(double) * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(static, 16)
#endif
    for (long long b = 0; b < B; b++) {
      syn_stream ss = syn_make_stream(seed, 4u, (uint64_t)b);
      syn_u4 r = syn_block(&ss, 0u);
      long long j = (long long)(syn_u01(r.v[0], r.v[1]) * (double)N);
      if (j >= N) j = N - 1;
      src[b] = j;
      syn_stream sn = syn_make_stream(seed, 5u, (uint64_t)b);
      syn_normals(&sn, n, buf);
      const float* x = X + (size_t)j * n;
      for (int t = 0; t < n; t++) buf[t] = (double)x[t] + sigma * buf[t];
      syn_znorm_store(buf, n, Q + (size_t)b * n);
    }
    free(buf);
  }
}

/* Query source rows only (no values): lets a caller fetch the source rows
 * itself when the collection is not held in one host array. */
void syn_query_sources(long long N, long long B, unsigned long long seed, long long* src) {
  for (long long b = 0; b < B; b++) {
    syn_stream ss = syn_make_stream(seed, 4u, (uint64_t)b);
    syn_u4 r = syn_block(&ss, 0u);
    long long j = (long long)(syn_u01(r.v[0], r.v[1]) * (double)N);
    if (j >= N) j = N - 1;
    src[b] = j;
  }
}

/* Noisy copies of given source rows (rows x n, already fetched). */
void syn_noisy_copies(const float* rows, long long B, int n, double sigma,
                      unsigned long long seed, float* Q) {
  double* buf = (double*)malloc(sizeof(double) * (size_t)n);
  for (long long b = 0; b < B; b++) {
    syn_stream sn = syn_make_stream(seed, 5u, (uint64_t)b);
    syn_normals(&sn, n, buf);
    const float* x = rows + (size_t)b * n;
    for (int t = 0; t < n; t++) buf[t] = (double)x[t] + sigma * buf[t];
    syn_znorm_store(buf, n, Q + (size_t)b * n);
  }
  free(buf);
}
