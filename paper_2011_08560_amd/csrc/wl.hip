// Wang-Landau estimate of the density of states (cited in Sec. II as an alternative to the
// multicanonical recursion), in the batched form this library samples in: the walkers of a
// realization share one estimate ln g on the levels [0, k_top] (W constant above the top, as for
// the recursion); a step samples some sweeps under lnW = -ln g, then every level's ln g grows by
// ln f times the visits the step's histogram counted there. When the histogram accumulated over
// the current stage is flat (min/mean over the levels it visited >= flat_tol), ln f is halved and
// a new stage begins; the estimate is done once ln f < ln f_final. One realization per block.
#include "kernels.hpp"
#include "table_builder.hpp"

namespace nfm {

// ln g = 0, stage histogram 0, ln f = ln_f0; weights 0 (a random walk in energy) and the table.
__global__ void k_wl_init(RealInfo* __restrict__ reals, WlArrays A, WlInfo* __restrict__ info, double ln_f0,
                          uint32_t* __restrict__ tables) {
  RealInfo* rp = reals + blockIdx.x;
  const int64_t off = rp->level_off;
  const int cap = level_capacity(rp->N);
  const int k_top = (-rp->e_base + 3) / 4;  // lowest level with E >= 0
  for (int k = threadIdx.x; k < cap; k += blockDim.x) {
    A.lng[off + k] = 0.0;
    A.hst[off + k] = 0ull;
    A.lnw[off + k] = 0.0;
  }
  if (threadIdx.x == 0) {
    WlInfo w{};
    w.ln_f = ln_f0;
    w.flatness = 0.0;
    w.stage = 0;
    w.done = 0;
    w.k_top = k_top;
    w.updates = 0;
    info[blockIdx.x] = w;
  }
  __syncthreads();
  build_table_block(rp, A.lnw + off, 0, k_top, tables);
}

// One step's update from the histogram (cleared afterwards), the stage test, the next table.
__global__ void k_wl_update(RealInfo* __restrict__ reals, WlArrays A, WlInfo* __restrict__ info,
                            unsigned long long* __restrict__ hist, double flat_tol, double ln_f_final,
                            uint32_t* __restrict__ tables) {
  RealInfo* rp = reals + blockIdx.x;
  WlInfo* wi = info + blockIdx.x;
  const int64_t off = rp->level_off;
  const int K = rp->K, k_top = wi->k_top;
  const double ln_f = wi->ln_f;
  const bool active = wi->done == 0;
  __shared__ unsigned long long s_min, s_sum;
  __shared__ int s_cnt;
  if (threadIdx.x == 0) {
    s_min = ~0ull;
    s_sum = 0ull;
    s_cnt = 0;
  }
  __syncthreads();
  unsigned long long mn = ~0ull, sum = 0ull;
  int cnt = 0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const unsigned long long h = hist[off + k];
    hist[off + k] = 0ull;
    if (!active || k > k_top) continue;
    if (h) A.lng[off + k] += ln_f * (double)h;
    const unsigned long long hs = A.hst[off + k] + h;
    A.hst[off + k] = hs;
    if (hs) {
      mn = hs < mn ? hs : mn;
      sum += hs;
      ++cnt;
    }
  }
  atomicMin(&s_min, mn);
  atomicAdd(&s_sum, sum);
  atomicAdd(&s_cnt, cnt);
  __syncthreads();
  __shared__ int s_halve;
  if (threadIdx.x == 0) {
    s_halve = 0;
    if (active) {
      const double flat = s_cnt > 0 ? (double)s_min / ((double)s_sum / (double)s_cnt) : 0.0;
      wi->flatness = flat;
      wi->updates += 1;
      if (flat >= flat_tol) {
        s_halve = 1;
        wi->ln_f = 0.5 * ln_f;
        wi->stage += 1;
        if (wi->ln_f < ln_f_final) wi->done = 1;
      }
    }
  }
  __syncthreads();
  if (!active) return;
  for (int k = threadIdx.x; k <= k_top; k += blockDim.x) {
    if (s_halve) A.hst[off + k] = 0ull;
    A.lnw[off + k] = -A.lng[off + k];
  }
  __syncthreads();
  build_table_block(rp, A.lnw + off, 0, k_top, tables);
}

// The recursion's state from the estimate: a level counts as visited when its ln g was raised
// (ln g > 0), k_lo = the lowest of them, b(k) = ln g(k+1) - ln g(k) on [k_lo, k_top), p = 0
// (the recursion's next histogram then weighs in fully), the given target profile.
__global__ void k_wl_to_rec(RealInfo* __restrict__ reals, RecInfo* __restrict__ recs, RecArrays R, WlArrays A,
                            const WlInfo* __restrict__ info, int profile, double pl_dE, double pl_alpha) {
  RealInfo* rp = reals + blockIdx.x;
  RecInfo* rc = recs + blockIdx.x;
  const int64_t off = rp->level_off;
  const int cap = level_capacity(rp->N), k_top = info[blockIdx.x].k_top;
  __shared__ int s_lo;
  if (threadIdx.x == 0) s_lo = k_top;
  __syncthreads();
  int lo = k_top;
  for (int k = threadIdx.x; k < cap; k += blockDim.x) {
    const bool vis = k <= k_top && A.lng[off + k] > 0.0;
    R.b[off + k] = 0.0;
    R.p[off + k] = 0.0;
    R.S[off + k] = 0.0;
    R.lnP[off + k] = 0.0;
    R.lnW[off + k] = 0.0;
    R.visited[off + k] = vis ? 1 : 0;
    if (vis && k < lo) lo = k;
  }
  atomicMin(&s_lo, lo);
  __syncthreads();
  const int k_lo = s_lo;
  for (int k = k_lo + (int)threadIdx.x; k < k_top; k += blockDim.x) R.b[off + k] = A.lng[off + k + 1] - A.lng[off + k];
  if (threadIdx.x == 0) {
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

hipError_t launch_wl_to_rec(RealInfo* reals, RecInfo* recs, int n_real, RecArrays R, WlArrays A, const WlInfo* info,
                            int profile, double pl_dE, double pl_alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_wl_to_rec, dim3(n_real), dim3(256), 0, s, reals, recs, R, A, info, profile, pl_dE, pl_alpha);
  return hipGetLastError();
}

hipError_t launch_wl_init(RealInfo* reals, int n_real, WlArrays A, WlInfo* info, double ln_f0, uint32_t* tables,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_wl_init, dim3(n_real), dim3(256), 0, s, reals, A, info, ln_f0, tables);
  return hipGetLastError();
}

hipError_t launch_wl_update(RealInfo* reals, int n_real, WlArrays A, WlInfo* info, unsigned long long* hist,
                            double flat_tol, double ln_f_final, uint32_t* tables, hipStream_t s) {
  hipLaunchKernelGGL(k_wl_update, dim3(n_real), dim3(256), 0, s, reals, A, info, hist, flat_tol, ln_f_final, tables);
  return hipGetLastError();
}

}  // namespace nfm
