// Learned damping / depth network: sizes, head constants and launchers
// (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbp {

constexpr int MLP_IN = 16, MLP_H = 64, MLP_OUT = 2;
constexpr int MLP_NPARAMS = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;  // 5378
constexpr float MLP_DMAX = 0.9f;    // damping head range [0, 0.9]
constexpr float MLP_CDELTA = 2.5f;  // log-depth correction range [-2.5, 2.5]

void launch_mlp_infer(const float *X, int n, const uint16_t *P, float *out_d, float *out_delta, hipStream_t s);
// the same with the features already rounded to BF16 (bits), 32 B per row
void launch_mlp_infer_bf16(const uint16_t *X, int n, const uint16_t *P, float *out_d, float *out_delta,
                           hipStream_t s);
void launch_mlp_train_step(const float *X, const float *Y, const float *M, int n_rows, const int *idx, int n_batch,
                           float *theta, float *m1, float *m2, float *grad, float *part_grad, float *part_loss,
                           float *loss, uint16_t *bf16, float lr, int step, bool update, hipStream_t s);
void launch_to_bf16(const float *theta, uint16_t *out, hipStream_t s);
int mlp_partial_blocks(int n_batch);

// Allocation-free training step: largest batch its fixed scratch holds, and
// the device-side address of that scratch on the current device (looked up
// on the first call per device; at most MLP_MAX_DEVICES devices).
constexpr int MLP_STATIC_MAX_BATCH = 8192;
constexpr int MLP_MAX_DEVICES = 64;
hipError_t mlp_static_scratch(float **ptr, size_t *floats);

}  // namespace gbp
