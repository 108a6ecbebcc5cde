// kernels.h -- launchers shared between the library's translation units.
#pragma once

#include "sofa_internal.h"

namespace sofa {

// MCB learning (k_learn.hip): fills h_var[2*pool], h_sel[16], h_beta[l*(alpha-1)].
sofa_status launch_learn(const float* X, int64_t N, int n, int64_t m, int pool, int l, int alpha,
                         int binning, int summary, int selection, hipStream_t st, double* h_var,
                         int* h_sel, double* h_beta);
// the fixed iSAX breakpoints, l x (alpha - 1) row-major
void isax_breakpoints(int n, int l, int alpha, double* beta);
// Device tables of a bins object (basis rows, FP32 breakpoints, selection).
sofa_status launch_bins_tables(sofa_bins* b, hipStream_t st);

// z-normalisation of m rows of n values (k_build.hip); out may equal in.
// With src_rows > m, output row r is the normalised input row
// floor(r * src_rows / m) (the stride sample of a src_rows-row array).
sofa_status launch_znorm(const float* in, int64_t m, int n, float* out, hipStream_t st,
                         int64_t src_rows = 0);

// MFMA projection (k_build.hip).  out: m x (16*ng) FP32 (nullable);
// words: m x 16 u8 quantised with beta32 (nullable, requires ng == 1);
// norm2: m FP64 squared norms (nullable); bad: set to 1 if any value is not finite.
sofa_status launch_project(const float* X, int64_t m, int n, int64_t ldx, const float* bt, int ng,
                           int n_pad, float* out, int ld_out, const float* beta32, int l,
                           uint8_t* words, double* norm2, unsigned* bad, hipStream_t st);

// Sort key of a word (used by the build and by the query routing): the
// symbols are scaled to 8 bits and their bits interleaved most significant
// first.  Scheme 0 gives word positions 0-3 eight bits each, 4-7 four bits,
// 8-15 two bits (positions are in decreasing-variance order, so the leaves
// split first where the Fourier values spread most); scheme 1 gives every
// position its top four bits.
__host__ __device__ inline uint64_t sfa_key(const uint32_t (&s8)[16], int scheme) {
  uint64_t key = 0;
  for (int b = 7; b >= 0; b--) {
    for (int j = 0; j < 16; j++) {
      int nbits = scheme == 1 ? 4 : (j < 4 ? 8 : (j < 8 ? 4 : 2));
      if (b >= 8 - nbits) key = (key << 1) | ((s8[j] >> b) & 1u);
    }
  }
  return key;
}

// p[0..n) = v on stream st (k_search.hip)
sofa_status launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// up to four fills p[i][0..n[i]) = v[i] in one launch (unused entries: n = 0)
struct FillRanges {
  uint32_t* p[4];
  int64_t n[4];
  uint32_t v[4];
};
sofa_status launch_fill_ranges(const FillRanges& f, hipStream_t st);

// Index layout (k_build.hip): sort by the interleaved key, permute, envelopes.
sofa_status launch_layout(sofa_index* ix, const float* X, const uint8_t* words_in,
                          const double* norm2_in, hipStream_t st);

}  // namespace sofa
