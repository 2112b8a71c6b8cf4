// Threshold-table construction shared by the table and recursion kernels (header-only so that
// each translation unit gets its own copy; no relocatable device code).
//
// Sec. II, Eq. (2): a move from level k with u unsatisfied bonds goes to k + m, m = 3 - u
// (Delta E = 4m), accepted with probability min(1, W(k+m)/W(k)). With step log-weights
// d(j) = lnW(j+1) - lnW(j) on [k_lo, k_top), continued as d(j) = 0 for j >= k_top (W constant
// above the top energy) and d(j) = d(k_lo) for j < k_lo (lowest known step), the ratio is the
// exp of the sum of the m steps in ascending j; it is stored as floor(x 2^32), or 0xFFFFFFFF
// (always accept) when x >= 1. The table covers [max(0, k_lo-3), min(K-1, k_top+3)]; rows
// outside repeat its edge rows exactly, so lookups clamp.
#pragma once
#include "nfm_internal.hpp"

namespace nfm {

__device__ __forceinline__ double step_logw(const double* lnw, int k_lo, int k_top, int j) {
  if (j < k_lo) j = k_lo;
  if (j >= k_top) return 0.0;
  return lnw[j + 1] - lnw[j];
}

// All threads of the block fill realization rp's table from lnw (indexed by level); thread 0
// records the table's row range. Callers synchronize before using the table.
__device__ inline void build_table_block(RealInfo* rp, const double* lnw, int k_lo, int k_top, uint32_t* tables) {
  const int K = rp->K;
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

}  // namespace nfm
