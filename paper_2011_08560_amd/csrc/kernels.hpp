// Host-side launchers of the libnfm kernels (one HIP source file per group).
#pragma once
#include "nfm_internal.hpp"

namespace nfm {

struct RealStatsDev {        // same layout as nfm_real_stats
  uint64_t rt_count;
  uint64_t rt_time;
  int32_t E_min;
  int32_t new_min;
  int32_t walkers_with_trips;
  int32_t pad;
  uint64_t reserved;
};

// lattice.hip
hipError_t launch_gen_couplings(const RealInfo* reals, int n_real, uint32_t* jabi, uint64_t seed, hipStream_t s);
hipError_t launch_pack_couplings(RealInfo* reals, int n_real, const uint32_t* jabi, uint32_t* jk, hipStream_t s);
hipError_t launch_gen_spins(const RealInfo* reals, int r0, int nr, int max_walkers, uint32_t* spins, uint64_t seed,
                            hipStream_t s);
hipError_t launch_pack_spins(const RealInfo* reals, int r, int wl0, int count, const int8_t* src, uint32_t* spins,
                             hipStream_t s);
hipError_t launch_unpack_spins(const RealInfo* reals, int r, int wl0, int count, const uint32_t* spins, int8_t* dst,
                               hipStream_t s);
hipError_t launch_energy(const RealInfo* reals, int n_real, int max_walkers, const uint32_t* jabi,
                         const uint32_t* spins, WalkerState ws, hipStream_t s);
hipError_t launch_reduce_real(const RealInfo* reals, int n_real, WalkerState ws, RealStatsDev* out, hipStream_t s);
// walkers without a completed round trip in the last `window` sweeps (flags optional; count added)
hipError_t launch_stuck(const RealInfo* reals, int n_real, WalkerState ws, uint64_t now, uint64_t since,
                        uint64_t window, uint8_t* flags, uint32_t* count, hipStream_t s);
// per-realization round-trip times and their population mean over [r0, r0 + count)
struct RtSummaryDev {        // same layout as nfm_rt_summary
  double tau_pop;
  uint64_t trips;
  int32_t n_used, n_censored;
};
hipError_t launch_rt_stats(const RealInfo* reals, const RealStatsDev* stats, int r0, int count, uint64_t min_trips,
                           double* tau, RtSummaryDev* out, hipStream_t s);

// tables.hip
hipError_t launch_build_tables(RealInfo* reals, int n_real, const double* lnw, const int32_t* k_lo,
                               const int32_t* k_top, uint32_t* tables, hipStream_t s);

// recursion.hip
hipError_t launch_rec_init(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, WalkerState ws, int profile,
                           double pl_dE, double pl_alpha, uint32_t* tables, hipStream_t s);
hipError_t launch_rec_weights(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, uint32_t* tables,
                              int set_bounds, hipStream_t s);
hipError_t launch_rec_update(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, WalkerState ws,
                             unsigned long long* hist, uint32_t* tables, double f_tol, hipStream_t s);
hipError_t launch_rec_targets(const RealInfo* reals, const RecInfo* recs, int n_real, RecArrays A, float* y, float* mask,
                              hipStream_t s);
hipError_t launch_rec_seed_copy(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, const double* src,
                                const int32_t* k_seed, hipStream_t s);
hipError_t launch_rec_seed_grid(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, const float* curves,
                                int32_t* k_seed_out, hipStream_t s);
hipError_t launch_rec_production(RealInfo* reals, RecInfo* recs, int n_real, RecArrays A, uint32_t* tables,
                                 int profile, double pl_dE, double pl_alpha, hipStream_t s);

// wl.hip
hipError_t launch_wl_init(RealInfo* reals, int n_real, WlArrays A, WlInfo* info, double ln_f0, uint32_t* tables,
                          hipStream_t s);
hipError_t launch_wl_update(RealInfo* reals, int n_real, WlArrays A, WlInfo* info, unsigned long long* hist,
                            double flat_tol, double ln_f_final, uint32_t* tables, hipStream_t s);
hipError_t launch_wl_to_rec(RealInfo* reals, RecInfo* recs, int n_real, RecArrays R, WlArrays A, const WlInfo* info,
                            int profile, double pl_dE, double pl_alpha, hipStream_t s);

// features.hip
hipError_t launch_canonical_tables(RealInfo* reals, int n_real, double T, double* lnw, int32_t* k_lo, int32_t* k_top,
                                   uint32_t* tables, hipStream_t s);
hipError_t launch_features(const RealInfo* reals, int n_real, const uint32_t* jabi, const unsigned long long* hist,
                           float* x, hipStream_t s);

// sweep.hip
// lds_rows / hist_levels: the most table rows / levels (K) of any realization in the launch
// (n_cu: compute units of the device; hist_mode: on-chip histogram 0 auto, 1 window, 2 every level,
// 3 the table rows alone)
hipError_t launch_muca_sweeps(int L, const SweepArgs& a, int n_waves, int lds_rows, int hist_levels, int n_cu,
                              int hist_mode, int ws_mode, bool spec, hipStream_t s);
// persistent launch over n_items waves; order = wave indices, longest first; maxl = the largest L
// among them (at most 8 or 10: the kernel forms for smaller lattices, which hold fewer registers);
// solo: the form whose waves each hold a whole SIMD
hipError_t launch_muca_queue(SweepArgs a, const int32_t* order, int n_items, uint32_t* counter, int grid, int n_cu,
                             int lds_rows, int hist_levels, int hist_mode, bool spec, hipStream_t s, int maxl,
                             bool solo = false);
// resident workgroups per CU of the persistent kernel (0 on error)
int queue_blocks_per_cu(bool spec, int lds_rows, int hist_levels, int hist_mode, int maxl, bool solo = false);
// a short bounded wait on stream s (orders the placement of two launches on two streams)
hipError_t launch_hold(hipStream_t s);
hipError_t launch_pt_sweeps(int L, const SweepArgs& a, int n_waves, hipStream_t s);
// the exchange thresholds of realization r as the sweep kernel computes them (inspection)
hipError_t launch_pt_swap_table(const double* q, int r, int M, int D, uint32_t* swap, hipStream_t s);
// name of the sweep kernel the last launch on this host thread used
const char* last_sweep_kernel();
// record a split persistent launch (the largest lattices in the SIMD-exclusive form beside the
// others) as the last launch
void note_partitioned_launch(bool spec);
bool sweep_supported(int L);

}  // namespace nfm
