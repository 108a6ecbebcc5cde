/*
 * sofa_oracle.c -- plain, slow, FP64 CPU oracle for exact k-NN search with
 * the SFA summary (SOFA, Schaefer et al., arXiv 2411.17483).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or constant with the GPU library: it is written from the paper's
 * definitions alone.  Every function states the passage it follows.
 *
 * Compile with -ffp-contract=off so that a*b+c is never fused: the distance
 * of record is the FP64 sum of squared differences taken in sequential order
 * of the time index.
 *
 * Parity pins (see tests/test_oracle_*.py): Parseval's identity, closed-form
 * DFT of pure sinusoids, numpy.fft agreement, lower bound <= distance on every
 * pair of small sets, unquantised full-spectrum lower bound == distance,
 * brute-force k-NN against numpy lexsort, equi-depth/equi-width breakpoints on
 * constructed samples, MLP gradients against central finite differences,
 * Adam's first step, iSAX breakpoints against an independent normal quantile,
 * PAA bound == distance on piecewise-constant series, the TLB on pairs worked
 * by hand and on equal bounds and distances (where it is one).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* z-normalisation (Section II, definition of the z-normalised Euclidean
 * distance).  Population standard deviation; a constant series maps to all
 * zeros. */
void orc_znorm(const double* x, int n, double* out) {
  double mu = 0.0;
  for (int t = 0; t < n; t++) mu += x[t];
  mu /= n;
  double var = 0.0;
  for (int t = 0; t < n; t++) var += (x[t] - mu) * (x[t] - mu);
  var /= n;
  double sd = sqrt(var);
  for (int t = 0; t < n; t++) out[t] = (sd > 0.0) ? (x[t] - mu) / sd : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Squared Euclidean distance of two z-normalised series (Section II).  The
 * inputs are the FP32 values of record, promoted to FP64; the squares are
 * summed in increasing time order with no fused multiply-add. */
double orc_dist2(const float* q, const float* x, int n) {
  double s = 0.0;
  for (int t = 0; t < n; t++) {
    double d = (double)q[t] - (double)x[t];
    double sq = d * d;
    s = s + sq;
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Orthonormal DFT coefficient k of one series (Section IV-E, Eq. 1 context):
 * X_k = n^{-1/2} sum_t x_t exp(-2 pi i k t / n).  The angle uses the integer
 * reduction (k*t mod n) so that large k*t products do not lose accuracy.  A
 * direct O(n) sum per coefficient, not an FFT. */
void orc_dft_coef(const float* x, int n, int k, double* re, double* im) {
  double sr = 0.0, si = 0.0;
  for (int t = 0; t < n; t++) {
    long long kt = ((long long)k * t) % n;
    double ang = 2.0 * ORC_PI * (double)kt / (double)n;
    sr += (double)x[t] * cos(ang);
    si -= (double)x[t] * sin(ang);
  }
  double s = 1.0 / sqrt((double)n);
  *re = sr * s;
  *im = si * s;
}

/* The candidate pool of one series: real and imaginary parts of the DFT
 * coefficients k = 1..P (the DC term is omitted because it is zero after
 * z-normalisation, Section IV-E, Eq. 1).  Pool index 2(k-1) is Re X_k and 2(k-1)+1
 * is Im X_k.  out has 2P entries. */
void orc_dft_pool(const float* x, int n, int P, double* out) {
  for (int k = 1; k <= P; k++) {
    double re, im;
    orc_dft_coef(x, n, k, &re, &im);
    out[2 * (k - 1)] = re;
    out[2 * (k - 1) + 1] = im;
  }
}

/* Weight of a Fourier value of coefficient k in the lower bound (Eq. 1):
 * 1 for the DC term and the Nyquist term (they appear once in the spectrum),
 * 2 otherwise (the conjugate coefficient n-k carries the same energy). */
double orc_weight(int k, int n) { return (k == 0 || 2 * k == n) ? 1.0 : 2.0; }

/* ------------------------------------------------------------------------ */
/* Sorting helpers (insertion-free: a plain merge sort on doubles). */
static void orc_msort(double* a, double* tmp, long lo, long hi) {
  if (hi - lo < 2) return;
  long mid = lo + (hi - lo) / 2;
  orc_msort(a, tmp, lo, mid);
  orc_msort(a, tmp, mid, hi);
  long i = lo, j = mid, o = lo;
  while (i < mid && j < hi) tmp[o++] = (a[j] < a[i]) ? a[j++] : a[i++];
  while (i < mid) tmp[o++] = a[i++];
  while (j < hi) tmp[o++] = a[j++];
  for (long t = lo; t < hi; t++) a[t] = tmp[t];
}

/* Breakpoints of one Fourier value from its sample (Algorithm 1, step 3;
 * Section IV-E, transformation and learned quantisation).  alpha symbols give alpha-1 finite breakpoints; the outer
 * bins are open to -inf / +inf.
 *  equi-depth (binning 0): beta(a) = v_(floor(a*m/alpha)), the order
 *    statistic of the sorted sample, a = 1..alpha-1.
 *  equi-width (binning 1): beta(a) = min + a*(max-min)/alpha. */
void orc_breakpoints(const double* vals, long m, int alpha, int binning, double* beta) {
  double* v = (double*)malloc(sizeof(double) * m);
  double* tmp = (double*)malloc(sizeof(double) * m);
  memcpy(v, vals, sizeof(double) * m);
  orc_msort(v, tmp, 0, m);
  for (int a = 1; a < alpha; a++) {
    if (binning == 0) {
      long idx = (long)(((long long)a * m) / alpha);
      beta[a - 1] = v[idx];
    } else {
      beta[a - 1] = v[0] + (double)a * (v[m - 1] - v[0]) / (double)alpha;
    }
  }
  free(v);
  free(tmp);
}

/* Variance-based selection (Section IV-E, feature selection; Algorithm 1,
 * step 2): population variance of each pool value over the sample, then the
 * l values with the largest variance.  Ties go to the lower pool index.  The
 * word keeps the selected values in decreasing-variance order. */
void orc_select(const double* var, int npool, int l, int* sel) {
  char* used = (char*)calloc(npool, 1);
  for (int j = 0; j < l; j++) {
    int best = -1;
    for (int p = 0; p < npool; p++) {
      if (used[p]) continue;
      if (best < 0 || var[p] > var[best]) best = p;
    }
    sel[j] = best;
    used[best] = 1;
  }
  free(used);
}

/* MCB (Algorithm 1): stride sample of m rows (row floor(i*N/m)), DFT pool of
 * each sampled row, variance per pool value, top-l selection, then alpha
 * bins per selected value.  Outputs: var[2P], sel[l], beta[l][alpha-1]. */
/* first != 0: keep the first l pool values instead of the l of largest
 * variance (the ablation's variant without variance selection, Section V-E). */
void orc_learn_bins(const float* X, long N, int n, long m, int P, int l, int alpha,
                    int binning, int first, double* var, int* sel, double* beta) {
  int np = 2 * P;
  double* F = (double*)malloc(sizeof(double) * m * np);
  for (long i = 0; i < m; i++) {
    long row = (long)(((long long)i * N) / m);
    orc_dft_pool(X + (size_t)row * n, n, P, F + (size_t)i * np);
  }
  for (int p = 0; p < np; p++) {
    double mu = 0.0;
    for (long i = 0; i < m; i++) mu += F[(size_t)i * np + p];
    mu /= (double)m;
    double s = 0.0;
    for (long i = 0; i < m; i++) {
      double d = F[(size_t)i * np + p] - mu;
      s += d * d;
    }
    var[p] = s / (double)m;
  }
  if (first)
    for (int j = 0; j < l; j++) sel[j] = j;
  else
    orc_select(var, np, l, sel);
  double* col = (double*)malloc(sizeof(double) * m);
  for (int j = 0; j < l; j++) {
    for (long i = 0; i < m; i++) col[i] = F[(size_t)i * np + sel[j]];
    orc_breakpoints(col, m, alpha, binning, beta + (size_t)j * (alpha - 1));
  }
  free(col);
  free(F);
}

/* Quantisation (Algorithm 2, step 2; Section IV-E bins): the symbol of a
 * value c for selected value j is the number of finite breakpoints that are
 * <= c, i.e. the index of the half-open bin [beta(a-1), beta(a)) holding c. */
int orc_symbol(double c, const double* beta_j, int alpha) {
  int s = 0;
  for (int a = 1; a < alpha; a++)
    if (beta_j[a - 1] <= c) s++;
  return s;
}

/* SFA word of one series (Algorithm 2): selected pool values, quantised. */
void orc_sfa_word(const float* x, int n, int P, int l, int alpha, const int* sel,
                  const double* beta, unsigned char* word, double* coefs_sel) {
  double* pool = (double*)malloc(sizeof(double) * 2 * P);
  orc_dft_pool(x, n, P, pool);
  for (int j = 0; j < l; j++) {
    double c = pool[sel[j]];
    if (coefs_sel) coefs_sel[j] = c;
    word[j] = (unsigned char)orc_symbol(c, beta + (size_t)j * (alpha - 1), alpha);
  }
  free(pool);
}

/* mind_i of Eq. 3: distance from a numeric value v to the bin of symbol s,
 * zero inside [beta(s), beta(s+1)), otherwise the gap to the nearer edge.
 * The outer bins extend to -inf / +inf. */
double orc_mind(double v, int s, const double* beta_j, int alpha) {
  double lo = (s == 0) ? -INFINITY : beta_j[s - 1];
  double hi = (s == alpha - 1) ? INFINITY : beta_j[s];
  if (v < lo) return lo - v;
  if (v > hi) return v - hi;
  return 0.0;
}

/* Squared SFA lower bound (Eq. 2): sum over selected values of
 * w_j * mind_j(symbol_j, query value_j)^2, with the DC term omitted. */
double orc_sfa_lb2(const double* qsel, const unsigned char* word, const double* beta,
                   const double* w, int l, int alpha) {
  double s = 0.0;
  for (int j = 0; j < l; j++) {
    double m = orc_mind(qsel[j], word[j], beta + (size_t)j * (alpha - 1), alpha);
    s += w[j] * m * m;
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* iSAX (Section IV-D): the series is cut into l segments of equal length
 * n/l, each segment is replaced by its mean (PAA), and each mean is quantised
 * with breakpoints that split N(0,1) into alpha equally likely bins. */

/* PAA: the mean of each of the l segments (n divisible by l). */
void orc_paa(const float* x, int n, int l, double* out) {
  int seg = n / l;
  for (int j = 0; j < l; j++) {
    double s = 0.0;
    for (int t = j * seg; t < (j + 1) * seg; t++) s += (double)x[t];
    out[j] = s / (double)seg;
  }
}

/* The alpha-1 breakpoints: beta(a) solves Phi(beta) = a/alpha with
 * Phi(x) = erfc(-x/sqrt(2))/2; found by halving an interval in which Phi
 * crosses a/alpha until its ends are adjacent doubles. */
void orc_isax_breakpoints(int alpha, double* beta) {
  for (int a = 1; a < alpha; a++) {
    double p = (double)a / (double)alpha, lo = -50.0, hi = 50.0;
    for (;;) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (0.5 * erfc(-mid / sqrt(2.0)) < p) lo = mid;
      else hi = mid;
    }
    beta[a - 1] = 0.5 * (lo + hi);
  }
}

/* iSAX word: the symbol of each PAA mean (half-open bins, as orc_symbol). */
void orc_isax_word(const float* x, int n, int l, int alpha, const double* beta,
                   unsigned char* word, double* paa) {
  double* m = (double*)malloc(sizeof(double) * l);
  orc_paa(x, n, l, m);
  for (int j = 0; j < l; j++) {
    if (paa) paa[j] = m[j];
    word[j] = (unsigned char)orc_symbol(m[j], beta, alpha);
  }
  free(m);
}

/* Squared iSAX lower bound of a query's PAA means against a word: n/l times
 * the sum of squared gaps between each query mean and the bin of the word's
 * symbol (the same gap as orc_mind, one breakpoint set for every segment). */
double orc_isax_lb2(const double* qpaa, const unsigned char* word, const double* beta, int n,
                    int l, int alpha) {
  double s = 0.0;
  for (int j = 0; j < l; j++) {
    double m = orc_mind(qpaa[j], word[j], beta, alpha);
    s += m * m;
  }
  return (double)(n / l) * s;
}

/* Squared PAA distance (the unquantised bound): n/l times the sum of squared
 * differences of the segment means. */
double orc_paa_dist2(const float* q, const float* x, int n, int l) {
  double* a = (double*)malloc(sizeof(double) * l);
  double* b = (double*)malloc(sizeof(double) * l);
  orc_paa(q, n, l, a);
  orc_paa(x, n, l, b);
  double s = 0.0;
  for (int j = 0; j < l; j++) s += (a[j] - b[j]) * (a[j] - b[j]);
  free(a);
  free(b);
  return (double)(n / l) * s;
}

/* Squared DFT lower bound (Eq. 1) on a set of unquantised Fourier values. */
double orc_dft_lb2(const double* a, const double* b, const double* w, int cnt) {
  double s = 0.0;
  for (int j = 0; j < cnt; j++) s += w[j] * (a[j] - b[j]) * (a[j] - b[j]);
  return s;
}

/* ------------------------------------------------------------------------ */
/* Exact k-NN by brute force (Section II, similarity search; the k-NN
 * extension of Section IV-C): every series is ranked by the key
 * (squared FP64 distance, original row id), ascending, and the first k are
 * returned.  Queries run in parallel; each one scans the collection in row
 * order and keeps a sorted list of its k best keys. */
void orc_knn(const float* X, long N, int n, const float* Q, long B, int k,
             long long* ids, double* d2, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (long b = 0; b < B; b++) {
    double* bd = (double*)malloc(sizeof(double) * k);
    long long* bi = (long long*)malloc(sizeof(long long) * k);
    int cnt = 0;
    const float* q = Q + (size_t)b * n;
    for (long i = 0; i < N; i++) {
      double d = orc_dist2(q, X + (size_t)i * n, n);
      if (cnt == k && !(d < bd[k - 1])) continue; /* equal distance: lower id already kept */
      int pos = (cnt < k) ? cnt : k - 1;
      while (pos > 0 && d < bd[pos - 1]) {
        bd[pos] = bd[pos - 1];
        bi[pos] = bi[pos - 1];
        pos--;
      }
      bd[pos] = d;
      bi[pos] = i;
      if (cnt < k) cnt++;
    }
    for (int j = 0; j < k; j++) {
      ids[(size_t)b * k + j] = (j < cnt) ? bi[j] : -1;
      d2[(size_t)b * k + j] = (j < cnt) ? bd[j] : INFINITY;
    }
    free(bd);
    free(bi);
  }
}

/* Exact squared distances of one query to an explicit list of rows, used to
 * check sampled outputs at full size one by one. */
void orc_dist2_rows(const float* X, int n, const float* q, const long long* rows, long cnt,
                    double* out) {
  for (long i = 0; i < cnt; i++) out[i] = orc_dist2(q, X + (size_t)rows[i] * n, n);
}

/* Tightness of the lower bound (Section V-E): mean over (query, series)
 * pairs with nonzero distance of LB / distance (distances, not squares).
 * A diagnostic: the paper's values are for datasets not available here. */
double orc_tlb(const double* lb2, const double* dist2, long cnt) {
  double s = 0.0;
  long c = 0;
  for (long i = 0; i < cnt; i++) {
    if (dist2[i] > 0.0) {
      s += sqrt(lb2[i]) / sqrt(dist2[i]);
      c++;
    }
  }
  return c ? s / (double)c : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Learned radius network: y = W3 g(W2 g(W1 x + b1) + b2) + b3 with
 * g(x) = x * Phi(x) = 0.5 x (1 + erf(x / sqrt 2)) (exact GELU), trained
 * with the mean squared error against ln(d_k) and Adam (Kingma & Ba, 2015).
 * The weights used in the products are the BF16-rounded copies passed in
 * by the caller (W1r, W2r, W3r); the arithmetic is FP64.
 * Layout: W1 [H1][D], W2 [H2][H1], W3 [H2] (one output), row-major. */
static double orc_gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }
static double orc_gelu_grad(double x) {
  double phi = exp(-0.5 * x * x) / sqrt(2.0 * ORC_PI);
  return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * phi;
}

void orc_mlp_forward(const float* x, long B, int D, int H1, int H2, const double* W1,
                     const double* b1, const double* W2, const double* b2, const double* W3,
                     double b3, double* y) {
  double* h1 = (double*)malloc(sizeof(double) * H1);
  double* a1 = (double*)malloc(sizeof(double) * H1);
  for (long b = 0; b < B; b++) {
    const float* xb = x + (size_t)b * D;
    for (int i = 0; i < H1; i++) {
      double s = b1[i];
      for (int d = 0; d < D; d++) s += W1[(size_t)i * D + d] * (double)xb[d];
      h1[i] = s;
      a1[i] = orc_gelu(s);
    }
    double out = b3;
    for (int i = 0; i < H2; i++) {
      double s = b2[i];
      for (int j = 0; j < H1; j++) s += W2[(size_t)i * H1 + j] * a1[j];
      out += W3[i] * orc_gelu(s);
    }
    y[b] = out;
  }
  free(h1);
  free(a1);
}

/* Loss and gradients of L = (1/B) sum_b (y_b - t_b)^2 with respect to every
 * parameter, by the chain rule through the two GELU layers. */
double orc_mlp_backward(const float* x, const float* t, long B, int D, int H1, int H2,
                        const double* W1, const double* b1, const double* W2,
                        const double* b2, const double* W3, double b3, double* gW1,
                        double* gb1, double* gW2, double* gb2, double* gW3, double* gb3) {
  memset(gW1, 0, sizeof(double) * H1 * D);
  memset(gb1, 0, sizeof(double) * H1);
  memset(gW2, 0, sizeof(double) * H2 * H1);
  memset(gb2, 0, sizeof(double) * H2);
  memset(gW3, 0, sizeof(double) * H2);
  *gb3 = 0.0;
  double* h1 = (double*)malloc(sizeof(double) * H1);
  double* a1 = (double*)malloc(sizeof(double) * H1);
  double* h2 = (double*)malloc(sizeof(double) * H2);
  double* a2 = (double*)malloc(sizeof(double) * H2);
  double* d2 = (double*)malloc(sizeof(double) * H2);
  double* d1 = (double*)malloc(sizeof(double) * H1);
  double loss = 0.0;
  for (long b = 0; b < B; b++) {
    const float* xb = x + (size_t)b * D;
    for (int i = 0; i < H1; i++) {
      double s = b1[i];
      for (int d = 0; d < D; d++) s += W1[(size_t)i * D + d] * (double)xb[d];
      h1[i] = s;
      a1[i] = orc_gelu(s);
    }
    double y = b3;
    for (int i = 0; i < H2; i++) {
      double s = b2[i];
      for (int j = 0; j < H1; j++) s += W2[(size_t)i * H1 + j] * a1[j];
      h2[i] = s;
      a2[i] = orc_gelu(s);
      y += W3[i] * a2[i];
    }
    double r = y - (double)t[b];
    loss += r * r;
    double dy = 2.0 * r / (double)B;
    *gb3 += dy;
    for (int i = 0; i < H2; i++) {
      gW3[i] += dy * a2[i];
      d2[i] = dy * W3[i] * orc_gelu_grad(h2[i]);
      gb2[i] += d2[i];
    }
    for (int j = 0; j < H1; j++) {
      double s = 0.0;
      for (int i = 0; i < H2; i++) {
        gW2[(size_t)i * H1 + j] += d2[i] * a1[j];
        s += d2[i] * W2[(size_t)i * H1 + j];
      }
      d1[j] = s * orc_gelu_grad(h1[j]);
      gb1[j] += d1[j];
      for (int d = 0; d < D; d++) gW1[(size_t)j * D + d] += d1[j] * (double)xb[d];
    }
  }
  free(h1);
  free(a1);
  free(h2);
  free(a2);
  free(d2);
  free(d1);
  return loss / (double)B;
}

/* One Adam step (Kingma & Ba, 2015, Algorithm 1) on a flat parameter vector:
 * m <- b1 m + (1-b1) g ; v <- b2 v + (1-b2) g^2 ;
 * p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void orc_adam(double* p, const double* g, double* m, double* v, long cnt, int step,
              double lr, double beta1, double beta2, double eps) {
  double c1 = 1.0 - pow(beta1, step);
  double c2 = 1.0 - pow(beta2, step);
  for (long i = 0; i < cnt; i++) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double mh = m[i] / c1;
    double vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision copies for the batched-distance prune.  Round-to-nearest-
 * even conversion of an FP64 value to the BF16 grid (8 significant bits,
 * FP32 exponent range) and to the OCP FP8 E4M3 grid (4 significant bits,
 * exponent bias 7, largest finite 448, subnormal step 2^-9, saturating).
 * Both are written from the formats' definitions. */
static double orc_round_sig(double x, int sig_bits, int min_exp) {
  /* round x to sig_bits significant bits, with exponent floor min_exp for
   * subnormals (values below 2^min_exp keep the spacing 2^(min_exp-sig+1)) */
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(fabs(x), &e); /* |x| = f * 2^e, f in [0.5,1) -> leading bit 2^(e-1) */
  int lead = e - 1;
  if (lead < min_exp) lead = min_exp;
  double ulp = ldexp(1.0, lead - (sig_bits - 1));
  double q = x / ulp;
  double r = nearbyint(q); /* default rounding mode: nearest, ties to even */
  return r * ulp;
}
double orc_to_bf16(double x) { return orc_round_sig(x, 8, -126); }
double orc_to_e4m3(double x) {
  double r = orc_round_sig(x, 4, -6);
  if (r > 448.0) r = 448.0;
  if (r < -448.0) r = -448.0;
  return r;
}
