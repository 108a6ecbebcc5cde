// mlp.h -- the learned-radius network's layout and handle (internal).
#pragma once

#include "kernels.h"

namespace sofa {

// flat parameter vector: W1 [H1][D], b1 [H1], W2 [H2][H1], b2 [H2], W3 [H2], b3 [1]
struct MlpDims {
  int D = 32, H1 = 256, H2 = 256;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, n = 0;
  void layout() {
    oW1 = 0;
    ob1 = oW1 + (int64_t)H1 * D;
    oW2 = ob1 + H1;
    ob2 = oW2 + (int64_t)H2 * H1;
    oW3 = ob2 + H2;
    ob3 = oW3 + H2;
    n = ob3 + 1;
  }
  __host__ __device__ int64_t total() const { return n; }
  __host__ __device__ bool is_weight(int64_t i) const {
    return (i >= oW1 && i < ob1) || (i >= oW2 && i < ob2) || (i >= oW3 && i < ob3);
  }
};

struct MlpAct {
  float *xs, *z1, *h1, *z2, *h2, *dz2, *y, *dy;
};

size_t mlp_act_floats(const MlpDims& d, int64_t B);
MlpAct act_views(float* base, const MlpDims& d, int64_t B);
// radii of a search's queries into U0; scratch: model_radius_scratch_floats
// floats (none when the fused inference kernel holds the activations in LDS)
sofa_status launch_model_radius(const sofa_radius* m, const float* pool, int64_t ld, int64_t B,
                                float* scratch, float* U0, hipStream_t st);
bool infer_fits(const MlpDims& d);
size_t model_radius_scratch_floats(const MlpDims& d, int64_t B);

}  // namespace sofa

struct sofa_radius {
  sofa::MlpDims dims;
  int k = 1;
  float lr = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  float margin = 0.0f;
  int64_t step = 0;
  sofa::DevBuf p, wr, g, m1, m2, mu, sd, loss;  // master, rounded copy, gradient, Adam moments
  sofa::DevBuf act;                             // activations of the largest training batch
  sofa::DevBuf part;                            // split-K partial weight gradients
  int64_t act_rows = 0;
};
