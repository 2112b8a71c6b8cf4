// Threshold tables from log-weights (Sec. II, Eq. (2) with the weights of Eqs. (3)-(7)).
// A move from level k with u unsatisfied bonds goes to level k + m, m = 3 - u (Delta E = 4m),
// and is accepted with probability min(1, W(k+m)/W(k)). With step log-weights
// d(j) = lnW(j+1) - lnW(j) on [k_lo, k_top), continued as d(j) = 0 above k_top (constant W)
// and d(j) = d(k_lo) below k_lo (lowest known step), the ratio is exp of the sum of m steps
// (ascending j), stored as floor(x 2^32) or 0xFFFFFFFF when x >= 1. The table covers levels
// [max(0, k_lo-3), min(K-1, k_top+3)]; rows outside repeat the edge rows exactly.
#include "kernels.hpp"

namespace nfm {

__device__ __forceinline__ double step_logw(const double* lnw, int k_lo, int k_top, int j) {
  if (j < k_lo) j = k_lo;
  if (j >= k_top) return 0.0;
  return lnw[j + 1] - lnw[j];
}

// One block per realization; threads over (row, u) entries.
__global__ void k_build_tables(RealInfo* __restrict__ reals, const double* __restrict__ lnw_all,
                               const int32_t* __restrict__ k_lo_all, const int32_t* __restrict__ k_top_all,
                               uint32_t* __restrict__ tables) {
  RealInfo* rp = reals + blockIdx.x;
  const int K = rp->K;
  const int k_lo = k_lo_all[blockIdx.x], k_top = k_top_all[blockIdx.x];
  const double* lnw = lnw_all + rp->level_off;  // indexed by level
  const int row0 = k_lo - 3 < 0 ? 0 : k_lo - 3;
  const int row_hi = k_top + 3 > K - 1 ? K - 1 : k_top + 3;
  const int rows = row_hi - row0 + 1;
  uint32_t* tab = tables + rp->table_off;
  for (int e = threadIdx.x; e < rows * 8; e += blockDim.x) {
    const int k = row0 + e / 8, u = e % 8;
    uint32_t thr = 0;
    if (u <= 6) {
      const int m = 3 - u;
      double x = 1.0;
      if (m > 0) {
        double s = 0.0;
        for (int j = k; j <= k + m - 1; ++j) s += step_logw(lnw, k_lo, k_top, j);
        x = exp(s);
      } else if (m < 0) {
        double s = 0.0;
        for (int j = k + m; j <= k - 1; ++j) s += step_logw(lnw, k_lo, k_top, j);
        x = exp(-s);
      }
      thr = x >= 1.0 ? 0xFFFFFFFFu : (uint32_t)floor(ldexp(x, 32));
    }
    tab[e] = thr;
  }
  if (threadIdx.x == 0) {
    rp->row0 = row0;
    rp->rows = rows;
  }
}

hipError_t launch_build_tables(RealInfo* reals, int n_real, const double* lnw, const int32_t* k_lo,
                               const int32_t* k_top, uint32_t* tables, hipStream_t s) {
  hipLaunchKernelGGL(k_build_tables, dim3(n_real), dim3(256), 0, s, reals, lnw, k_lo, k_top, tables);
  return hipGetLastError();
}

}  // namespace nfm
