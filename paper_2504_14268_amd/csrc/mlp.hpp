// mlp.hpp -- device layout of the MLP policy trainer (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace mpcg {

constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kNAct * kMlpH + kNAct;

// bfloat16 weights for the matrix cores: row-major [out][in] (w*b) and, for
// the backward products, transposed [in][out] (w*t); fp32 biases.
struct MlpWeights {
  uint16_t *w1b, *w2b, *w3b, *w2t, *w3t;
  float *b1, *b2, *b3;
};

// fp32 master parameters and Adam moments (parameter order W1 | b1 | W2 | b2 |
// W3 | b3), and the current bfloat16 copies.
struct MlpState {
  float *master, *m, *v;
  MlpWeights cur;
};

__device__ void mlp_store_copy(const MlpWeights &dst, int p, float w);

void launch_mlp_copies(const MlpWeights &dst, const float *params, hipStream_t s);
void launch_mlp_forward(const MlpWeights &W, const float *feat, int n, float *logits, const float *rew,
                        const uint8_t *done, float gamma, float *target, float *ymax_buf, hipStream_t s);
void launch_mlp_grad(const MlpWeights &W, const float *feat, const int32_t *act, const float *target, int b0, int B,
                     float *part, float *part_loss, hipStream_t s);
void launch_mlp_update(const MlpState &st, const float *part, const float *part_loss, int nwg, int adam, int t,
                       float lr, float b1, float b2, float eps, float *grad_out, float *loss_out, hipStream_t s);

}  // namespace mpcg
