// Cost-model MLP: sizes and launch helpers.
#pragma once

#include "ccut_internal.h"

namespace ccut {

constexpr int MLP_IN = 8, MLP_HIDDEN = 64, MLP_OUT = 3;
constexpr int MLP_PARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN +
                           MLP_HIDDEN * MLP_OUT + MLP_OUT;  // 4931
constexpr int MLP_PART_STRIDE = 4936;   // floats per chunk: gradient + squared error, padded
static_assert(MLP_PART_STRIDE > MLP_PARAMS, "chunk stride");
constexpr int MLP_ROWS_PER_BLOCK = 32;

uint64_t mlp_work_floats(int64_t rows, int epochs);
int mlp_forward(const float* P, const float* X, int64_t rows, float* Y, hipStream_t s);
int mlp_grad(const float* P, const float* X, const float* T, int64_t rows, float* work, float* grad, float* loss,
             hipStream_t s);
int mlp_train(float* P, const float* X, const float* T, int64_t rows, int epochs, float lr, float* work,
              float* losses_host, int graph_epochs, hipStream_t s);

}  // namespace ccut
