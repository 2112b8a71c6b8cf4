// Threshold tables of all realizations from caller-given log-weights (Sec. II, Eq. (2) with the
// weights of Eqs. (3)-(7)); construction rules in table_builder.hpp.
#include "kernels.hpp"
#include "table_builder.hpp"

namespace nfm {

// One block per realization; lnw_all is indexed by the realization's level offset.
__global__ void k_build_tables(RealInfo* __restrict__ reals, const double* __restrict__ lnw_all,
                               const int32_t* __restrict__ k_lo_all, const int32_t* __restrict__ k_top_all,
                               uint32_t* __restrict__ tables) {
  RealInfo* rp = reals + blockIdx.x;
  build_table_block(rp, lnw_all + rp->level_off, k_lo_all[blockIdx.x], k_top_all[blockIdx.x], tables);
}

hipError_t launch_build_tables(RealInfo* reals, int n_real, const double* lnw, const int32_t* k_lo,
                               const int32_t* k_top, uint32_t* tables, hipStream_t s) {
  hipLaunchKernelGGL(k_build_tables, dim3(n_real), dim3(256), 0, s, reals, lnw, k_lo, k_top, tables);
  return hipGetLastError();
}

}  // namespace nfm
