// Kernels of the weight-seeding network (a learned start for the weight iteration of Sec. II):
// 81 inputs -> 3 x 128 GELU -> 256 outputs. FP32 training (forward, backward, Adam) and BF16
// inference, with the dense products on the matrix cores.
//
// Products: one 64-lane wave computes a 16 x 16 tile of C = op(A) op(B) with
// v_mfma_f32_16x16x4_f32 (FP32) or v_mfma_f32_16x16x16_bf16 (BF16, FP32 accumulation). Operand
// lanes: lane l holds A(i0 + l%16, k0 + l/16) and B(k0 + l/16, j0 + l%16) (FP32; BF16: four
// consecutive k per lane, k0 + 4(l/16) + 0..3); the result tile has C(i0 + 4(l/16) + r, j0 + l%16)
// in accumulator r. Dimensions are padded (16 rows per tile, K a multiple of 4 / 16), so every
// access is in bounds without masks.
#include "mlp_internal.hpp"

namespace nfm {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C[M x N] = op(A) op(B), then the epilogue:
//   EPI 0: C = acc              EPI 1: C = acc + bias[col]
//   EPI 2: C2 = acc + bias[col] (pre-activation), C = gelu(C2)
//   EPI 3: C = acc * gelu'(aux[row][col])
// One workgroup per 16 x 16 tile of C; its S waves each reduce a contiguous K / S share, and wave 0
// adds the other waves' partial tiles in wave order before the epilogue (a fixed order).
template <bool TA, bool TB, int EPI, int S>
__global__ void __launch_bounds__(64 * S) k_gemm_f32(int M, int N, int K, const float* __restrict__ A, int lda,
                                                     const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                     int ldc, const float* __restrict__ bias,
                                                     const float* __restrict__ aux, float* __restrict__ C2) {
  __shared__ v4f part[S > 1 ? S - 1 : 1][64];
  const int tj = blockIdx.x, ti = blockIdx.y;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, li = l & 15, lk = l >> 4;
  const int ia = ti * 16 + li, jb = tj * 16 + li;
  const int kper = K / S, kb = wv * kper;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
  for (int k0 = kb; k0 < kb + kper; k0 += 4) {
    const int k = k0 + lk;
    const float a = TA ? A[(size_t)k * lda + ia] : A[(size_t)ia * lda + k];
    const float b = TB ? B[(size_t)jb * ldb + k] : B[(size_t)k * ldb + jb];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  if constexpr (S > 1) {
    if (wv > 0) part[wv - 1][l] = acc;
    __syncthreads();
    if (wv > 0) return;
#pragma unroll
    for (int q = 0; q < S - 1; ++q) acc += part[q][l];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = ti * 16 + 4 * lk + r, col = jb;
    float v = acc[r];
    if (EPI == 1) v += bias[col];
    if (EPI == 2) {
      v += bias[col];
      C2[(size_t)row * ldc + col] = v;
      v = gelu_f(v);
    }
    if (EPI == 3) v *= gelu_grad_f(aux[(size_t)row * ldc + col]);
    C[(size_t)row * ldc + col] = v;
  }
  (void)M;
  (void)N;
}

template <bool TA, bool TB, int EPI>
static hipError_t gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                       const float* bias, const float* aux, float* C2, hipStream_t s) {
  if (M % 16 || N % 16 || K % 4 || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  // the layers' K (96, 128, 256) split over four waves; any other multiple of 4 runs on one
  if (K % 16 == 0)
    hipLaunchKernelGGL((k_gemm_f32<TA, TB, EPI, 4>), dim3(N / 16, M / 16), dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, bias, aux, C2);
  else
    hipLaunchKernelGGL((k_gemm_f32<TA, TB, EPI, 1>), dim3(N / 16, M / 16), dim3(64), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, bias, aux, C2);
  return hipGetLastError();
}

// Column sums of X [M x N] (bias gradients; N a multiple of 16). A block of 256 threads takes 16
// columns: thread (slice, col) sums rows slice, slice + 16, ... in order, then the 16 slices of a
// column are added in order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_colsum(int M, int N, const float* __restrict__ X, float* __restrict__ out) {
  __shared__ float part[16][17];
  const int col = threadIdx.x & 15, slice = threadIdx.x >> 4;
  const int j = blockIdx.x * 16 + col;
  float s = 0.f;
  if (j < N)
    for (int i = slice; i < M; i += 16) s += X[(size_t)i * N + j];
  part[slice][col] = s;
  __syncthreads();
  if (slice == 0 && j < N) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += part[k][col];
    out[j] = t;
  }
}

// Xn [Bp x 96] = (X - mean) / sd on the 81 inputs of the first B rows, zero elsewhere.
__global__ void k_normalize(int B, int Bp, const float* __restrict__ X, const float* __restrict__ norm,
                            float* __restrict__ Xn) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Bp * kMlpInPad) return;
  const int i = e / kMlpInPad, k = e % kMlpInPad;
  float v = 0.f;
  if (i < B && k < kMlpIn) v = (X[(size_t)i * kMlpIn + k] - norm[k]) / norm[kMlpIn + k];
  Xn[e] = v;
}

// Masked mean squared error L = sum m (y - t)^2 / sum m over the first B rows, and its gradient
// dY = 2 m (y - t) / sum m (zero on padded rows), in two passes with sums in a fixed order.
// Pass 1: block b sums m and m (y - t)^2 over its contiguous share of the n = B * 256 elements
// (per thread in order, then a tree over the block) into part[b] and part[kMlpLossBlocks + b].
__global__ void __launch_bounds__(256) k_loss_partial(int n, const float* __restrict__ Y, const float* __restrict__ T,
                                                      const float* __restrict__ Mk, float* __restrict__ part) {
  __shared__ float s_m[256], s_e[256];
  const int chunk = (n + kMlpLossBlocks - 1) / kMlpLossBlocks;
  const int e0 = blockIdx.x * chunk, e1 = min(n, e0 + chunk);
  float sm = 0.f, se = 0.f;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const float m = Mk[e], d = Y[e] - T[e];
    sm += m;
    se += m * d * d;
  }
  s_m[threadIdx.x] = sm;
  s_e[threadIdx.x] = se;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_m[threadIdx.x] += s_m[threadIdx.x + h];
      s_e[threadIdx.x] += s_e[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_m[0];
    part[kMlpLossBlocks + blockIdx.x] = s_e[0];
  }
}

// Pass 2: every block adds the partial sums in the same tree order (so all blocks hold the same
// total), block 0 stores the loss, and each thread writes one element of dY [Bp x 256].
__global__ void __launch_bounds__(256) k_loss_final(int n, int total, const float* __restrict__ Y,
                                                    const float* __restrict__ T, const float* __restrict__ Mk,
                                                    const float* __restrict__ part, float* __restrict__ dY,
                                                    float* __restrict__ loss) {
  __shared__ float s_m[kMlpLossBlocks], s_e[kMlpLossBlocks];
  if ((int)threadIdx.x < kMlpLossBlocks) {
    s_m[threadIdx.x] = part[threadIdx.x];
    s_e[threadIdx.x] = part[kMlpLossBlocks + threadIdx.x];
  }
  __syncthreads();
  for (int h = kMlpLossBlocks / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_m[threadIdx.x] += s_m[threadIdx.x + h];
      s_e[threadIdx.x] += s_e[threadIdx.x + h];
    }
    __syncthreads();
  }
  const float msum = s_m[0];
  const float inv = msum > 0.f ? 1.0f / msum : 0.f;
  if (blockIdx.x == 0 && threadIdx.x == 0) loss[0] = s_e[0] * inv;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < total) dY[e] = e < n ? 2.0f * Mk[e] * (Y[e] - T[e]) * inv : 0.f;
}

// Adam with bias correction: c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Glorot-uniform weights from the Philox stream (counter (e >> 2, layer, 0, 6) under the seed),
// zero biases and zero padding rows of the first layer.
__global__ void k_mlp_init(float* __restrict__ p, uint32_t key0, uint32_t key1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpNParam) return;
  float v = 0.f;
  for (int layer = 0; layer < 4; ++layer) {
    const int o = mlp_w_off(layer), nin = mlp_in(layer), nout = mlp_out(layer);
    if (e >= o && e < o + nin * nout) {
      const int row = (e - o) / nout;
      const int fan_in = layer == 0 ? kMlpIn : nin;
      if (row < fan_in) {
        const int q = e - o;
        const u32x4 r = philox4x32_10((uint32_t)(q >> 2), (uint32_t)layer, 0u, 6u, key0, key1);
        const uint32_t w = r.v[q & 3];
        const float a = sqrtf(6.0f / (float)(fan_in + nout));
        v = a * (2.0f * ((float)(w >> 8) + 0.5f) * (1.0f / 16777216.0f) - 1.0f);
      }
    }
  }
  p[e] = v;
}

// ------------------------------------------------------------------ BF16 inference

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// BF16 copy of the weights, transposed to [out][in] so that each lane's four k are contiguous.
__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ wt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  for (int layer = 0; layer < 4; ++layer) {
    const int o = mlp_w_off(layer), nin = mlp_in(layer), nout = mlp_out(layer);
    if (e < nin * nout) {
      const int i = e / nout, j = e % nout;
      wt[o + j * nin + i] = bf16_rne(p[o + e]);
    }
  }
}

__global__ void k_normalize_bf16(int B, int Bp, const float* __restrict__ X, const float* __restrict__ norm,
                                 uint16_t* __restrict__ Xb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Bp * kMlpInPad) return;
  const int i = e / kMlpInPad, k = e % kMlpInPad;
  float v = 0.f;
  if (i < B && k < kMlpIn) v = (X[(size_t)i * kMlpIn + k] - norm[k]) / norm[kMlpIn + k];
  Xb[e] = bf16_rne(v);
}

// C = A [M x K] (bf16, row-major) times W (bf16, stored [N][K]) + bias (fp32);
// HIDDEN: C = bf16(gelu(.)) into Cb; otherwise fp32 into Cf.
template <bool HIDDEN>
__global__ void __launch_bounds__(64) k_gemm_bf16(int K, const uint16_t* __restrict__ A, const uint16_t* __restrict__ Wt,
                                                  const float* __restrict__ bias, int N, uint16_t* __restrict__ Cb,
                                                  float* __restrict__ Cf) {
  const int tj = blockIdx.x, ti = blockIdx.y;
  const int l = threadIdx.x, li = l & 15, lk = l >> 4;
  const int ia = ti * 16 + li, jb = tj * 16 + li;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int k = k0 + 4 * lk;
    const uint2 av = *(const uint2*)(A + (size_t)ia * K + k);
    const uint2 bv = *(const uint2*)(Wt + (size_t)jb * K + k);
    v4s a, b;
    a[0] = (short)(av.x & 0xFFFFu);
    a[1] = (short)(av.x >> 16);
    a[2] = (short)(av.y & 0xFFFFu);
    a[3] = (short)(av.y >> 16);
    b[0] = (short)(bv.x & 0xFFFFu);
    b[1] = (short)(bv.x >> 16);
    b[2] = (short)(bv.y & 0xFFFFu);
    b[3] = (short)(bv.y >> 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = ti * 16 + 4 * lk + r;
    const float v = acc[r] + bias[jb];
    if (HIDDEN)
      Cb[(size_t)row * N + jb] = bf16_rne(gelu_f(v));
    else
      Cf[(size_t)row * N + jb] = v;
  }
}

// ------------------------------------------------------------------ sequences

hipError_t mlp_forward_f32(const MlpBuffers& m, const float* X, int B, int Bp, float* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3((Bp * kMlpInPad + 255) / 256), dim3(256), 0, s, B, Bp, X, m.norm, m.Xn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float* P = m.params;
  if ((e = gemm<false, false, 2>(Bp, kMlpHid, kMlpInPad, m.Xn, kMlpInPad, P + mlp_w_off(0), kMlpHid, m.A1, kMlpHid,
                                 P + mlp_b_off(0), nullptr, m.Z1, s)) != hipSuccess)
    return e;
  if ((e = gemm<false, false, 2>(Bp, kMlpHid, kMlpHid, m.A1, kMlpHid, P + mlp_w_off(1), kMlpHid, m.A2, kMlpHid,
                                 P + mlp_b_off(1), nullptr, m.Z2, s)) != hipSuccess)
    return e;
  if ((e = gemm<false, false, 2>(Bp, kMlpHid, kMlpHid, m.A2, kMlpHid, P + mlp_w_off(2), kMlpHid, m.A3, kMlpHid,
                                 P + mlp_b_off(2), nullptr, m.Z3, s)) != hipSuccess)
    return e;
  return gemm<false, false, 1>(Bp, kMlpOut, kMlpHid, m.A3, kMlpHid, P + mlp_w_off(3), kMlpOut, Y, kMlpOut,
                               P + mlp_b_off(3), nullptr, nullptr, s);
}

hipError_t mlp_loss_grad(const MlpBuffers& m, const float* X, const float* T, const float* Mk, int B, int Bp,
                         hipStream_t s) {
  hipError_t e = mlp_forward_f32(m, X, B, Bp, m.Y, s);
  if (e != hipSuccess) return e;
  static_assert(kMlpLossBlocks <= 256 && (kMlpLossBlocks & (kMlpLossBlocks - 1)) == 0, "loss partials");
  hipLaunchKernelGGL(k_loss_partial, dim3(kMlpLossBlocks), dim3(256), 0, s, B * kMlpOut, m.Y, T, Mk, m.loss + 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3((Bp * kMlpOut + 255) / 256), dim3(256), 0, s, B * kMlpOut, Bp * kMlpOut, m.Y, T,
                     Mk, m.loss + 1, m.dY, m.loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const float* P = m.params;
  float* G = m.grads;
  const int H = kMlpHid;
  // output layer
  if ((e = gemm<true, false, 0>(H, kMlpOut, Bp, m.A3, H, m.dY, kMlpOut, G + mlp_w_off(3), kMlpOut, nullptr, nullptr,
                                nullptr, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(kMlpOut / 16), dim3(256), 0, s, Bp, kMlpOut, m.dY, G + mlp_b_off(3));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // dZ3 = (dY W3^T) * gelu'(Z3)
  if ((e = gemm<false, true, 3>(Bp, H, kMlpOut, m.dY, kMlpOut, P + mlp_w_off(3), kMlpOut, m.dZa, H, nullptr, m.Z3,
                                nullptr, s)) != hipSuccess)
    return e;
  if ((e = gemm<true, false, 0>(H, H, Bp, m.A2, H, m.dZa, H, G + mlp_w_off(2), H, nullptr, nullptr, nullptr, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(H / 16), dim3(256), 0, s, Bp, H, m.dZa, G + mlp_b_off(2));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm<false, true, 3>(Bp, H, H, m.dZa, H, P + mlp_w_off(2), H, m.dZb, H, nullptr, m.Z2, nullptr, s)) !=
      hipSuccess)
    return e;
  if ((e = gemm<true, false, 0>(H, H, Bp, m.A1, H, m.dZb, H, G + mlp_w_off(1), H, nullptr, nullptr, nullptr, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(H / 16), dim3(256), 0, s, Bp, H, m.dZb, G + mlp_b_off(1));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm<false, true, 3>(Bp, H, H, m.dZb, H, P + mlp_w_off(1), H, m.dZa, H, nullptr, m.Z1, nullptr, s)) !=
      hipSuccess)
    return e;
  if ((e = gemm<true, false, 0>(kMlpInPad, H, Bp, m.Xn, kMlpInPad, m.dZa, H, G + mlp_w_off(0), H, nullptr, nullptr,
                                nullptr, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(H / 16), dim3(256), 0, s, Bp, H, m.dZa, G + mlp_b_off(0));
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpBuffers& m, float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kMlpNParam + 255) / 256), dim3(256), 0, s, kMlpNParam, m.params, m.grads, m.adam_m,
                     m.adam_v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_init(const MlpBuffers& m, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_init, dim3((kMlpNParam + 255) / 256), dim3(256), 0, s, m.params, (uint32_t)seed,
                     (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const MlpBuffers& m, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((kMlpHid * kMlpOut + 255) / 256), dim3(256), 0, s, m.params, m.wbf16);
  return hipGetLastError();
}

hipError_t mlp_infer_bf16(const MlpBuffers& m, const float* X, int B, int Bp, float* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize_bf16, dim3((Bp * kMlpInPad + 255) / 256), dim3(256), 0, s, B, Bp, X, m.norm, m.Xb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float* P = m.params;
  const uint16_t* W = m.wbf16;
  hipLaunchKernelGGL((k_gemm_bf16<true>), dim3(kMlpHid / 16, Bp / 16), dim3(64), 0, s, kMlpInPad, m.Xb,
                     W + mlp_w_off(0), P + mlp_b_off(0), kMlpHid, m.Hb1, nullptr);
  hipLaunchKernelGGL((k_gemm_bf16<true>), dim3(kMlpHid / 16, Bp / 16), dim3(64), 0, s, kMlpHid, m.Hb1,
                     W + mlp_w_off(1), P + mlp_b_off(1), kMlpHid, m.Hb2, nullptr);
  hipLaunchKernelGGL((k_gemm_bf16<true>), dim3(kMlpHid / 16, Bp / 16), dim3(64), 0, s, kMlpHid, m.Hb2,
                     W + mlp_w_off(2), P + mlp_b_off(2), kMlpHid, m.Hb1, nullptr);
  hipLaunchKernelGGL((k_gemm_bf16<false>), dim3(kMlpOut / 16, Bp / 16), dim3(64), 0, s, kMlpHid, m.Hb1,
                     W + mlp_w_off(3), P + mlp_b_off(3), kMlpOut, nullptr, Y);
  return hipGetLastError();
}

}  // namespace nfm
