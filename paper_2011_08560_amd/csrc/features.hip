// Inputs of the weight-seeding model: canonical tables for a short high-temperature run, and a
// per-realization feature vector from the couplings and that run's energy histogram.
//
// Feature vector (81 floats per realization):
//   x[0]       L / 12
//   x[1..3]    frustrated fraction of (x,y), (y,z), (z,x) plaquettes; x[4] of all plaquettes
//              (a plaquette (i; d1, d2) has bonds J_d1(i), J_d2(i+e_d1), J_d1(i+e_d2), J_d2(i) and
//              is frustrated when their product is -1)
//   x[5..7]    negative-bond fraction along x, y, z; x[8] of all bonds; x[9] = n_minus mod 2
//   x[10..13]  fraction of elementary cubes with 0, 2, 4, 6 frustrated faces
//   x[14..16]  mean / 6, variance / 6, fourth central moment / 96 of the site sums sum_j J_ij
//   x[17..80]  histogram of E/N in 64 bins over [-2, 0): bin floor((E/N + 2) 32) clipped to
//              [0, 63], as fractions of all entries of the realization's level histogram
// Counts are exact integers; the moments are formed in FP64 from the 7-bin histogram of site sums.
#include "kernels.hpp"
#include "table_builder.hpp"

namespace nfm {

// Canonical Metropolis at temperature T: lnW(k) = -E_k / T given on the two top levels; the table
// builder continues the lowest step below them, which is the same constant step -4/T.
__global__ void k_canonical_lnw(const RealInfo* __restrict__ reals, int n_real, double T, double* __restrict__ lnw,
                                int32_t* __restrict__ k_lo, int32_t* __restrict__ k_top) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_real) return;
  const RealInfo ri = reals[r];
  const int K = ri.K;
  k_lo[r] = K - 2;
  k_top[r] = K - 1;
  lnw[ri.level_off + K - 2] = -(double)(ri.e_base + 4 * (K - 2)) / T;
  lnw[ri.level_off + K - 1] = -(double)(ri.e_base + 4 * (K - 1)) / T;
}

hipError_t launch_canonical_tables(RealInfo* reals, int n_real, double T, double* lnw, int32_t* k_lo, int32_t* k_top,
                                   uint32_t* tables, hipStream_t s) {
  hipLaunchKernelGGL(k_canonical_lnw, dim3((n_real + 255) / 256), dim3(256), 0, s, reals, n_real, T, lnw, k_lo, k_top);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_build_tables(reals, n_real, lnw, k_lo, k_top, tables, s);
}

__device__ __forceinline__ int fj(const uint32_t* jw, int JW, int d, int i) {
  return ((jw[d * JW + (i >> 5)] >> (i & 31)) & 1u) ? -1 : 1;
}

__device__ __forceinline__ int fnb(int L, int i, int d, int step) {
  int x = i % L, y = (i / L) % L, z = i / (L * L);
  if (d == 0) x = (x + step + L) % L;
  if (d == 1) y = (y + step + L) % L;
  if (d == 2) z = (z + step + L) % L;
  return x + L * (y + L * z);
}

__device__ __forceinline__ int plaq_frustrated(const uint32_t* jw, int JW, int L, int i, int d1, int d2) {
  const int a = fnb(L, i, d1, 1), c = fnb(L, i, d2, 1);
  return fj(jw, JW, d1, i) * fj(jw, JW, d2, a) * fj(jw, JW, d1, c) * fj(jw, JW, d2, i) < 0;
}

__global__ void k_features(const RealInfo* __restrict__ reals, const uint32_t* __restrict__ jabi,
                           const unsigned long long* __restrict__ hist, float* __restrict__ x) {
  const RealInfo ri = reals[blockIdx.x];
  const int L = ri.L, N = ri.N, JW = abi_plane_words(N);
  const uint32_t* jw = jabi + ri.jabi_off;
  __shared__ int s_cnt[17];  // fr[3], neg[3], cubes[4], site-sum histogram[7]
  __shared__ unsigned long long s_bin[64];
  for (int k = threadIdx.x; k < 17; k += blockDim.x) s_cnt[k] = 0;
  for (int k = threadIdx.x; k < 64; k += blockDim.x) s_bin[k] = 0ull;
  __syncthreads();
  int fr[3] = {0, 0, 0}, neg[3] = {0, 0, 0}, cub[4] = {0, 0, 0, 0}, sh[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    fr[0] += plaq_frustrated(jw, JW, L, i, 0, 1);
    fr[1] += plaq_frustrated(jw, JW, L, i, 1, 2);
    fr[2] += plaq_frustrated(jw, JW, L, i, 2, 0);
    int ssum = 0;
    for (int d = 0; d < 3; ++d) {
      const int j = fj(jw, JW, d, i);
      neg[d] += j < 0;
      ssum += j + fj(jw, JW, d, fnb(L, i, d, -1));
    }
    const int f = plaq_frustrated(jw, JW, L, i, 0, 1) + plaq_frustrated(jw, JW, L, fnb(L, i, 2, 1), 0, 1) +
                  plaq_frustrated(jw, JW, L, i, 1, 2) + plaq_frustrated(jw, JW, L, fnb(L, i, 0, 1), 1, 2) +
                  plaq_frustrated(jw, JW, L, i, 2, 0) + plaq_frustrated(jw, JW, L, fnb(L, i, 1, 1), 2, 0);
    cub[f / 2] += 1;
    sh[(ssum + 6) / 2] += 1;
  }
  for (int k = 0; k < 3; ++k) atomicAdd(&s_cnt[k], fr[k]);
  for (int k = 0; k < 3; ++k) atomicAdd(&s_cnt[3 + k], neg[k]);
  for (int k = 0; k < 4; ++k) atomicAdd(&s_cnt[6 + k], cub[k]);
  for (int k = 0; k < 7; ++k) atomicAdd(&s_cnt[10 + k], sh[k]);
  const int cap = level_capacity(N);
  const unsigned long long* H = hist + ri.level_off;
  for (int k = threadIdx.x; k < ri.K && k < cap; k += blockDim.x) {
    const unsigned long long h = H[k];
    if (h == 0ull) continue;
    const double e = (double)(ri.e_base + 4 * k) / (double)N;
    int j = (int)floor((e + 2.0) * 32.0);
    j = j < 0 ? 0 : (j > 63 ? 63 : j);
    atomicAdd(&s_bin[j], h);
  }
  __syncthreads();
  float* out = x + (int64_t)blockIdx.x * 81;
  if (threadIdx.x == 0) {
    const double n = (double)N;
    out[0] = (float)((double)L / 12.0);
    for (int o = 0; o < 3; ++o) out[1 + o] = (float)((double)s_cnt[o] / n);
    out[4] = (float)((double)(s_cnt[0] + s_cnt[1] + s_cnt[2]) / (3.0 * n));
    for (int d = 0; d < 3; ++d) out[5 + d] = (float)((double)s_cnt[3 + d] / n);
    const int nneg = s_cnt[3] + s_cnt[4] + s_cnt[5];
    out[8] = (float)((double)nneg / (3.0 * n));
    out[9] = (float)(nneg % 2);
    for (int c = 0; c < 4; ++c) out[10 + c] = (float)((double)s_cnt[6 + c] / n);
    double sum = 0.0;
    for (int v = 0; v < 7; ++v) sum += (double)s_cnt[10 + v] * (double)(2 * v - 6);
    const double mean = sum / n;
    double m2 = 0.0, m4 = 0.0;
    for (int v = 0; v < 7; ++v) {
      const double dv = (double)(2 * v - 6) - mean;
      m2 += (double)s_cnt[10 + v] * dv * dv;
      m4 += (double)s_cnt[10 + v] * dv * dv * dv * dv;
    }
    out[14] = (float)(mean / 6.0);
    out[15] = (float)(m2 / n / 6.0);
    out[16] = (float)(m4 / n / 96.0);
  }
  if (threadIdx.x < 64) {
    unsigned long long tot = 0ull;
    for (int j = 0; j < 64; ++j) tot += s_bin[j];
    out[17 + threadIdx.x] = tot ? (float)((double)s_bin[threadIdx.x] / (double)tot) : 0.0f;
  }
}

hipError_t launch_features(const RealInfo* reals, int n_real, const uint32_t* jabi, const unsigned long long* hist,
                           float* x, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(n_real), dim3(256), 0, s, reals, jabi, hist, x);
  return hipGetLastError();
}

}  // namespace nfm
