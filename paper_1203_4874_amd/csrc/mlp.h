// Sizes and layouts of the learned form's network (mlp.hip).  Internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cbp {

constexpr int MLP_FEAT = 32;
constexpr int MLP_HIDDEN = 128;
constexpr int MLP_OUT = 2;
// packed FP32 parameter vector: W1 [128][32], b1, W2 [128][128], b2, W3 [2][128], b3
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_HIDDEN * MLP_FEAT;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_HIDDEN;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_HIDDEN * MLP_HIDDEN;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_HIDDEN;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_OUT * MLP_HIDDEN;
constexpr int MLP_NPARAM = MLP_OFF_B3 + MLP_OUT;
constexpr uint32_t MLP_MAGIC = 0x4D504243u;  // "CBPM"
constexpr uint32_t MLP_VERSION = 1;

// Inference blob (device memory): the matrix-core layers in bfloat16 bits,
// the 2-output head and the biases in FP32.
struct mlp_blob {
  uint32_t magic, version, feat, hidden;
  unsigned short W1[MLP_HIDDEN * MLP_FEAT];
  unsigned short W2[MLP_HIDDEN * MLP_HIDDEN];
  float W3[MLP_OUT * MLP_HIDDEN];
  float b1[MLP_HIDDEN];
  float b2[MLP_HIDDEN];
  float b3[MLP_OUT];
};

// Device bytes of a training state for batches of up to `rows` rows.
size_t mlp_state_bytes(int rows);
hipError_t mlp_set_params(void* state, int rows, const float* params, hipStream_t st);
hipError_t mlp_get_params(const void* state, int rows, float* params, hipStream_t st);
hipError_t mlp_save_state(const void* state, int rows, float* out, hipStream_t st);
hipError_t mlp_load_state(void* state, int rows, const float* in, hipStream_t st);
hipError_t mlp_gradients(void* state, int rows, const float* X, const float* T, int n, float* loss,
                         float* grads, hipStream_t st);
hipError_t mlp_adam_step(void* state, int rows, float lr, int step, hipStream_t st);
hipError_t mlp_export(const void* state, int rows, void* blob, hipStream_t st);
hipError_t mlp_forward_blob(const void* blob, const float* X, int n, float* out, hipStream_t st);

}  // namespace cbp
