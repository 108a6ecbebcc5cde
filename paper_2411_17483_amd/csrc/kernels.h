// kernels.h -- launchers shared between the library's translation units.
#pragma once

#include "sofa_internal.h"

namespace sofa {

// MCB learning (k_learn.hip): fills h_var[2*pool], h_sel[16], h_beta[l*(alpha-1)].
sofa_status launch_learn(const float* X, int64_t N, int n, int64_t m, int pool, int l, int alpha,
                         int binning, hipStream_t st, double* h_var, int* h_sel, double* h_beta);
// Device tables of a bins object (basis rows, FP32 breakpoints, selection).
sofa_status launch_bins_tables(sofa_bins* b, hipStream_t st);

// MFMA projection (k_build.hip).  out: m x (16*ng) FP32 (nullable);
// words: m x 16 u8 quantised with beta32 (nullable, requires ng == 1);
// norm2: m FP64 squared norms (nullable); bad: set to 1 if any value is not finite.
sofa_status launch_project(const float* X, int64_t m, int n, int64_t ldx, const float* bt, int ng,
                           int n_pad, float* out, int ld_out, const float* beta32, int l,
                           uint8_t* words, double* norm2, unsigned* bad, hipStream_t st);

// Index layout (k_build.hip): sort by the interleaved key, permute, envelopes.
sofa_status launch_layout(sofa_index* ix, const float* X, const uint8_t* words_in,
                          const double* norm2_in, hipStream_t st);

}  // namespace sofa
