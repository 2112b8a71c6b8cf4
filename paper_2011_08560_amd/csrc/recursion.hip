// Weight iteration on the device (Sec. II): the density-of-states estimate is refined from the
// histograms of the last sampling round, re-anchored at new minima, and turned into the next
// log-weights and threshold table, all without leaving the GPU.
//
// Estimate: DOS steps b(k) = S(k+1) - S(k), S = ln Omega up to a constant, S(k_top) = 0.
// Profiles (ln P): flat 0; power law alpha ln((E - E_g + dE)/(dE - E_g)), Eq. (5) with E_g the
// lowest energy found; 1/k: S(k) - ln sum_{j=k_lo..k} exp S(j), Eq. (7). Weights lnW = -S + ln P
// (Eqs. (3), (4)). Update (accumulated statistics, Berg's multicanonical recursion written for a
// target profile): for consecutive visited levels k < k',
//   est = [ln H(k') - lnW(k')] - [ln H(k) - lnW(k)],  g0 = H(k) H(k') / (H(k) + H(k')),
//   p(k) += g0,  b(k) += (g0 / p(k)) (est - (b(k) + ... + b(k'-1))).
// The sequential parts (prefix sums over levels) run on one thread per realization in the same
// operation order as the oracle; the table is built by all threads of the block.
#include "kernels.hpp"
#include "table_builder.hpp"

namespace nfm {

__device__ __forceinline__ double rec_lnP_power(double E, double E_g, double dE, double alpha) {
  return alpha * log(E / (dE - E_g) + 1.0);
}

// S, ln P and lnW on [k_lo, k_top] from b (one thread); with a seeded prior also on
// [k_seed, k_lo): S continues with the seeded steps under the frozen profile lnP(k_lo).
__device__ void rec_weights_seq(const RecInfo& ri, int e_base, const double* b, double* S, double* lnP, double* lnW) {
  const int k_lo = ri.k_lo, k_top = ri.k_top;
  S[k_top] = 0.0;
  for (int k = k_top - 1; k >= k_lo; --k) S[k] = S[k + 1] - b[k];
  const double E_g = (double)(e_base + 4 * k_lo);
  double acc = 0.0;
  for (int k = k_lo; k <= k_top; ++k) {
    const double E = (double)(e_base + 4 * k);
    double lp;
    if (ri.profile == 0) {
      lp = 0.0;
    } else if (ri.profile == 1) {
      lp = rec_lnP_power(E, E_g, ri.pl_dE, ri.pl_alpha);
    } else {
      if (k == k_lo) {
        acc = S[k];
      } else {
        const double m = acc > S[k] ? acc : S[k];
        acc = m + log1p(exp(-fabs(acc - S[k])));
      }
      lp = S[k] - acc;
    }
    lnP[k] = lp;
    lnW[k] = -S[k] + lp;
  }
  for (int k = k_lo - 1; k >= rec_low(ri); --k) {
    S[k] = S[k + 1] - b[k];
    lnP[k] = lnP[k_lo];
    lnW[k] = -S[k] + lnP[k];
  }
}

// One realization per block: weights from the current estimate, table, round-trip bounds.
__global__ void k_rec_weights(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays A,
                              uint32_t* __restrict__ tables, int set_bounds) {
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const int64_t off = rp->level_off;
  if (threadIdx.x == 0) {
    rec_weights_seq(*rc, rp->e_base, A.b + off, A.S + off, A.lnP + off, A.lnW + off);
    if (set_bounds) {
      rp->e_bot = rp->e_base + 4 * rc->k_lo;
      rp->e_top = 0;
    }
  }
  __syncthreads();
  build_table_block(rp, A.lnW + off, rec_low(*rc), rc->k_top, tables);
}

// Initial state: b = p = 0, nothing visited, k_lo = lowest level of any walker's minimum.
__global__ void k_rec_init(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays A, WalkerState ws,
                           int profile, double pl_dE, double pl_alpha) {
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const int64_t off = rp->level_off;
  const int cap = level_capacity(rp->N);
  for (int k = threadIdx.x; k < cap; k += blockDim.x) {
    A.b[off + k] = 0.0;
    A.p[off + k] = 0.0;
    A.S[off + k] = 0.0;
    A.lnP[off + k] = 0.0;
    A.lnW[off + k] = 0.0;
    A.visited[off + k] = 0;
  }
  __shared__ int s_min;
  if (threadIdx.x == 0) s_min = 0x7fffffff;
  __syncthreads();
  int m = 0x7fffffff;
  for (int w = threadIdx.x; w < rp->walkers; w += blockDim.x) m = min(m, ws.E_min[rp->walker_off + w]);
  atomicMin(&s_min, m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int k_top = (-rp->e_base + 3) / 4;  // lowest level with E >= 0
    int k_lo = (s_min - rp->e_base) / 4;
    if (k_lo > k_top) k_lo = k_top;
    rc->k_lo = k_lo;
    rc->k_top = k_top;
    rc->profile = profile;
    rc->pl_dE = pl_dE;
    rc->pl_alpha = pl_alpha;
    rc->flatness = 0.0;
    rc->converged = 0;
    rc->iterations = 0;
    rc->k_lo_changed = 0;
    rc->k_seed = -1;
    rc->pad = 0;
  }
}

// One update from the histogram of the last sampling round, then the next weights and table.
__global__ void k_rec_update(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays A, WalkerState ws,
                             unsigned long long* __restrict__ hist, uint32_t* __restrict__ tables, double f_tol) {
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const int64_t off = rp->level_off;
  __shared__ int s_min;
  if (threadIdx.x == 0) s_min = 0x7fffffff;
  __syncthreads();
  int mn = 0x7fffffff;
  for (int w = threadIdx.x; w < rp->walkers; w += blockDim.x) mn = min(mn, ws.E_min[rp->walker_off + w]);
  atomicMin(&s_min, mn);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long* H = hist + off;
    double* b = A.b + off;
    double* p = A.p + off;
    const double* lnW = A.lnW + off;
    const double* lnP = A.lnP + off;
    unsigned char* visited = A.visited + off;
    const int k_lo_used = rc->k_lo, k_top = rc->k_top;
    const bool seeded = rc->k_seed >= 0;
    int k_min_seen = (s_min - rp->e_base) / 4;
    if (k_min_seen > k_lo_used) k_min_seen = k_lo_used;
    const int k_lo = k_min_seen;
    // new levels: the lowest known step (plain) or their seeded steps, no accumulated weight
    for (int k = k_lo; k < k_lo_used; ++k) {
      if (!seeded) b[k] = b[k_lo_used];
      p[k] = 0.0;
    }
    // weights used while sampling: stored on [low, k_top], continued with the lowest step below
    const int low = rec_low(*rc);
    const double d_lo = (low < k_top) ? lnW[low + 1] - lnW[low] : 0.0;
    auto lnw_at = [&](int k) {
      return k >= low ? lnW[k] : lnW[low] - (double)(low - k) * d_lo;
    };
    auto lnp_at = [&](int k) { return k >= k_lo_used ? lnP[k] : lnP[k_lo_used]; };
    int prev = -1;
    for (int k = k_lo; k <= k_top; ++k) {
      if (H[k] == 0) continue;
      if (prev >= 0) {
        const double Hk = (double)H[prev], Hk1 = (double)H[k];
        const double est = (log(Hk1) - lnw_at(k)) - (log(Hk) - lnw_at(prev));
        double span = 0.0;
        for (int j = prev; j < k; ++j) span += b[j];
        const double g0 = Hk * Hk1 / (Hk + Hk1);
        p[prev] += g0;
        b[prev] += (g0 / p[prev]) * (est - span);
      }
      prev = k;
    }
    double mnv = 0.0, sum = 0.0;
    int n = 0;
    for (int k = k_lo; k <= k_top; ++k) {
      if (H[k] > 0) visited[k] = 1;
      if (!visited[k]) continue;
      const double v = (double)H[k] / exp(lnp_at(k));
      if (n == 0 || v < mnv) mnv = v;
      sum += v;
      ++n;
    }
    const double flat = (n > 0 && sum > 0.0) ? mnv / (sum / (double)n) : 0.0;
    rc->k_lo_changed = (k_lo != k_lo_used);
    rc->k_lo = k_lo;
    rc->flatness = flat;
    rc->converged = (flat >= f_tol && k_lo == k_lo_used) ? 1 : 0;
    rc->iterations += 1;
    // next weights (re-anchored profile), bounds for the next round
    rec_weights_seq(*rc, rp->e_base, b, A.S + off, A.lnP + off, A.lnW + off);
    rp->e_bot = rp->e_base + 4 * k_lo;
    rp->e_top = 0;
  }
  __syncthreads();
  build_table_block(rp, A.lnW + off, rec_low(*rc), rc->k_top, tables);
  const int cap = level_capacity(rp->N);
  for (int k = threadIdx.x; k < cap; k += blockDim.x) hist[off + k] = 0ull;
}

// Production weights from the final estimate (Sec. II: the DOS is determined once and reused by
// every ensemble): flat lnW = -S, power law -S + ln P_SH, 1/k -S + (S - ln sum exp S).
__global__ void k_rec_production(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays A,
                                 uint32_t* __restrict__ tables, int profile, double pl_dE, double pl_alpha) {
  if (threadIdx.x == 0) {
    RecInfo* rc = recs + blockIdx.x;
    rc->profile = profile;
    rc->pl_dE = pl_dE;
    rc->pl_alpha = pl_alpha;
  }
  __syncthreads();
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const int64_t off = rp->level_off;
  if (threadIdx.x == 0) {
    rec_weights_seq(*rc, rp->e_base, A.b + off, A.S + off, A.lnP + off, A.lnW + off);
    rp->e_bot = rp->e_base + 4 * rc->k_lo;
    rp->e_top = 0;
  }
  __syncthreads();
  build_table_block(rp, A.lnW + off, rec_low(*rc), rc->k_top, tables);
}

// Seeded prior from caller-given steps: b(k) = src(k) on [k_seed, k_top) for realizations with
// k_seed >= 0, accumulated weights cleared; others untouched.
__global__ void k_rec_seed_copy(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays A,
                                const double* __restrict__ src, const int32_t* __restrict__ k_seed) {
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const int ks = k_seed[blockIdx.x];
  if (ks < 0) return;
  const int64_t off = rp->level_off;
  const int cap = level_capacity(rp->N);
  for (int k = threadIdx.x; k < cap; k += blockDim.x) {
    if (k >= ks && k < rc->k_top) A.b[off + k] = src[off + k];
    A.p[off + k] = 0.0;
  }
  if (threadIdx.x == 0) rc->k_seed = ks;
}

// Seeded prior from a curve y_j = [S(E) - S(E_top)]/N on the grid e_j = -2 + 2j/255 (256 floats
// per realization): S(k) = N y(E_k/N), linear between grid points, y_255 above; b(k) =
// max(S(k+1) - S(k), 0) on [k_s, k_top), k_s = the lowest level with E >= -2N. A curve with a
// step that is not finite, or without a positive step, is rejected (plain start kept;
// k_seed_out = -1).
__device__ __forceinline__ double seed_curve(const float* y, double e) {
  const double t = (e + 2.0) * 127.5;
  if (t <= 0.0) return (double)y[0];
  if (t >= 255.0) return (double)y[255];
  const int j = (int)floor(t);
  const double f = t - (double)j;
  return (double)y[j] + f * ((double)y[j + 1] - (double)y[j]);
}

__device__ __forceinline__ double seed_step(int N, int e_base, const float* y, int k) {
  const double s0 = (double)N * seed_curve(y, (double)(e_base + 4 * k) / (double)N);
  const double s1 = (double)N * seed_curve(y, (double)(e_base + 4 * (k + 1)) / (double)N);
  return s1 - s0;
}

__global__ void k_rec_seed_grid(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays A,
                                const float* __restrict__ curves, int32_t* __restrict__ k_seed_out) {
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const float* y = curves + (int64_t)blockIdx.x * 256;
  const int N = rp->N, e_base = rp->e_base, k_top = rc->k_top;
  int k_s = (-2 * N - e_base + 3) / 4;
  if (k_s < 0) k_s = 0;
  __shared__ int s_bad;
  __shared__ double s_pos[256];
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  double pos = 0.0;
  for (int k = k_s + (int)threadIdx.x; k < k_top; k += blockDim.x) {
    const double d = seed_step(N, e_base, y, k);
    if (!isfinite(d)) atomicOr(&s_bad, 1);
    if (d > 0.0) pos += d;
  }
  s_pos[threadIdx.x] = pos;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s_pos[threadIdx.x] += s_pos[threadIdx.x + h];
    __syncthreads();
  }
  if (s_bad || !(s_pos[0] > 0.0)) {
    if (threadIdx.x == 0) k_seed_out[blockIdx.x] = -1;
    return;
  }
  const int64_t off = rp->level_off;
  for (int k = k_s + (int)threadIdx.x; k < k_top; k += blockDim.x) {
    const double d = seed_step(N, e_base, y, k);
    A.b[off + k] = d > 0.0 ? d : 0.0;
  }
  const int cap = level_capacity(N);
  for (int k = threadIdx.x; k < cap; k += blockDim.x) A.p[off + k] = 0.0;
  if (threadIdx.x == 0) {
    rc->k_seed = k_s;
    k_seed_out[blockIdx.x] = k_s;
  }
}

// Training targets from the current estimate: on the grid e_j = -2 + 2j/255, y_j = S(e_j N) / N
// with S linear between levels (S(k_top) = 0), mask 1 where e_j N >= E(k_lo) (the estimate is
// defined there), 0 and y = 0 below.
__global__ void k_rec_targets(const RealInfo* __restrict__ reals, const RecInfo* __restrict__ recs, RecArrays A,
                              float* __restrict__ y, float* __restrict__ mask) {
  const RealInfo ri = reals[blockIdx.x];
  const RecInfo rc = recs[blockIdx.x];
  const double* S = A.S + ri.level_off;
  const int j = threadIdx.x;  // 256 threads
  const double N = (double)ri.N;
  const double E = (-2.0 + 2.0 * (double)j / 255.0) * N;
  const double E_lo = (double)(ri.e_base + 4 * rc.k_lo), E_top = (double)(ri.e_base + 4 * rc.k_top);
  float yv = 0.f, mv = 0.f;
  if (E >= E_lo) {
    double v;
    if (E >= E_top) {
      v = S[rc.k_top];
    } else {
      const double t = (E - (double)ri.e_base) / 4.0;
      int k = (int)floor(t);
      if (k < rc.k_lo) k = rc.k_lo;
      if (k > rc.k_top - 1) k = rc.k_top - 1;
      const double f = t - (double)k;
      v = S[k] + f * (S[k + 1] - S[k]);
    }
    yv = (float)(v / N);
    mv = 1.f;
  }
  y[(int64_t)blockIdx.x * 256 + j] = yv;
  mask[(int64_t)blockIdx.x * 256 + j] = mv;
}

hipError_t launch_rec_targets(const RealInfo* reals, const RecInfo* recs, int n_real, RecArrays A, float* y, float* mask,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_rec_targets, dim3(n_real), dim3(256), 0, s, reals, recs, A, y, mask);
  return hipGetLastError();
}

hipError_t launch_rec_seed_copy(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, const double* src,
                                const int32_t* k_seed, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_seed_copy, dim3(n_real), dim3(256), 0, s, reals, recs, A, src, k_seed);
  return hipGetLastError();
}

hipError_t launch_rec_seed_grid(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, const float* curves,
                                int32_t* k_seed_out, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_seed_grid, dim3(n_real), dim3(256), 0, s, reals, recs, A, curves, k_seed_out);
  return hipGetLastError();
}

hipError_t launch_rec_init(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, WalkerState ws, int profile,
                           double pl_dE, double pl_alpha, uint32_t* tables, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_init, dim3(n_real), dim3(256), 0, s, reals, recs, A, ws, profile, pl_dE, pl_alpha);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rec_weights, dim3(n_real), dim3(256), 0, s, reals, recs, A, tables, 1);
  return hipGetLastError();
}

hipError_t launch_rec_weights(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, uint32_t* tables,
                              int set_bounds, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_weights, dim3(n_real), dim3(256), 0, s, reals, recs, A, tables, set_bounds);
  return hipGetLastError();
}

hipError_t launch_rec_update(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, WalkerState ws,
                             unsigned long long* hist, uint32_t* tables, double f_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_update, dim3(n_real), dim3(256), 0, s, reals, recs, A, ws, hist, tables, f_tol);
  return hipGetLastError();
}

hipError_t launch_rec_production(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, uint32_t* tables,
                                 int profile, double pl_dE, double pl_alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_production, dim3(n_real), dim3(256), 0, s, reals, recs, A, tables, profile, pl_dE,
                     pl_alpha);
  return hipGetLastError();
}

}  // namespace nfm
