// learn.h -- learned vertex ordering launchers.  Used only inside csrc/.
#pragma once
#include <stdint.h>

#include "graph.h"

namespace pmc {

constexpr int MLP_PARAMS = 4801;  // W1 8x64, b1 64, W2 64x64, b2 64, w3 64, b3 1

// Eight features per vertex (row-major n x 8 floats).
void run_features(const GraphView &g, const int32_t *core, const int32_t *rank,
                  const int32_t *order, int32_t kmax, float *feat, Scratch &sc);
// score[i] = MLP(feat[i]).
void run_mlp_forward(const float *params, const float *feat, int64_t n, float *score,
                     Scratch &sc);
// One full-batch step on the mean squared error; Adam when lr > 0.  Returns
// the loss before the step; grad_out (optional, device) gets the gradient.
float run_mlp_train_step(float *params, float *m, float *v, int64_t step, float lr,
                         const float *feat, const float *label, int64_t n, float *grad_out,
                         Scratch &sc);

}  // namespace pmc
