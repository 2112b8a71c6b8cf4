// Shapes, parameter layout and buffers of the weight-seeding network (shared by its kernels and
// its host API). Parameter vector (float, this order, weights row-major [in][out]):
//   W0 [96 x 128] (input rows 81..95 are padding and stay zero), b0 [128], W1 [128 x 128], b1 [128],
//   W2 [128 x 128], b2 [128], W3 [128 x 256], b3 [256].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "philox.hpp"

namespace nfm {

constexpr int kMlpIn = 81, kMlpInPad = 96, kMlpHid = 128, kMlpOut = 256;
// Blocks of the loss's first reduction pass; their partial sums follow the loss in its buffer.
constexpr int kMlpLossBlocks = 64;

__host__ __device__ constexpr int mlp_in(int layer) { return layer == 0 ? kMlpInPad : kMlpHid; }
__host__ __device__ constexpr int mlp_out(int layer) { return layer == 3 ? kMlpOut : kMlpHid; }
__host__ __device__ constexpr int mlp_w_off(int layer) {
  return layer == 0 ? 0 : mlp_w_off(layer - 1) + mlp_in(layer - 1) * mlp_out(layer - 1) + mlp_out(layer - 1);
}
__host__ __device__ constexpr int mlp_b_off(int layer) { return mlp_w_off(layer) + mlp_in(layer) * mlp_out(layer); }
constexpr int kMlpNParam = mlp_b_off(3) + kMlpOut;
static_assert(kMlpNParam == 78464, "parameter count");

struct MlpBuffers {
  float *params, *grads, *adam_m, *adam_v, *norm;  // norm: mean[81], sd[81]
  uint16_t* wbf16;                                // BF16 weights, each layer transposed to [out][in]
  float *Xn, *Z1, *A1, *Z2, *A2, *Z3, *A3, *Y, *dY, *dZa, *dZb, *loss;
  uint16_t *Xb, *Hb1, *Hb2;
};

hipError_t mlp_init(const MlpBuffers& m, uint64_t seed, hipStream_t s);
hipError_t mlp_forward_f32(const MlpBuffers& m, const float* X, int B, int Bp, float* Y, hipStream_t s);
hipError_t mlp_loss_grad(const MlpBuffers& m, const float* X, const float* T, const float* Mk, int B, int Bp,
                         hipStream_t s);
hipError_t mlp_adam(const MlpBuffers& m, float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t mlp_to_bf16(const MlpBuffers& m, hipStream_t s);
hipError_t mlp_infer_bf16(const MlpBuffers& m, const float* X, int B, int Bp, float* Y, hipStream_t s);

}  // namespace nfm
