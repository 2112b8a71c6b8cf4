// Internal definitions of libnfm shared by the host API and the kernels.
// Geometry of the kernel's spin layout, per-realization records and kernel
// argument blocks. Model and conventions: see include/nfm.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace nfm {

constexpr int kMaxL = 12;
constexpr int kWave = 64;
constexpr uint32_t kTagAcc = 1, kTagSpin = 2, kTagJ = 3, kTagPT = 4, kTagSwap = 5;
constexpr int kMaxReplicas = 64;  // temperature slots of one parallel-tempering set

// Kernel spin layout. A walker's lattice is split by colour c = (x+y+z)&1 and
// plane z; the L/2 sites of colour c in row y of plane z (x = 2j + phi,
// phi = (c+y+z)&1) sit in bits j of a field of F bits at offset y*F of the
// plane-colour bit string, which occupies NWP 32-bit words.
__host__ __device__ constexpr int field_bits(int L) { return L <= 2 ? 1 : L <= 4 ? 2 : L <= 8 ? 4 : 8; }
__host__ __device__ constexpr int plane_words(int L) { return (L * field_bits(L) + 31) / 32; }
__host__ __device__ constexpr int walker_words(int L) { return 2 * L * plane_words(L); }
// Kernel coupling layout per realization: for every (c, z) six bit strings in
// the same field layout: [Jz fwd, Jz bwd, Jy fwd, Jy bwd, Jx partner, Jx other].
__host__ __device__ constexpr int jk_words(int L) { return 2 * L * 6 * plane_words(L); }
__host__ __device__ constexpr int abi_plane_words(int N) { return (N + 31) / 32; }
__host__ __device__ constexpr int level_capacity(int N) { return 3 * N / 2 + 1; }

// Per-realization record (device and host mirror).
struct RealInfo {
  int32_t L, N, K, e_base;
  int32_t walkers, n_minus;
  int32_t row0, rows;        // current threshold table covers levels [row0, row0+rows)
  int32_t e_bot, e_top;      // round-trip bounds
  uint32_t real_id;
  int32_t pad;
  int64_t walker_off;        // global index of the first walker
  int64_t spin_off;          // word offset into the spin buffer
  int64_t level_off;         // offset into per-level arrays (capacity level_capacity(N))
  int64_t table_off;         // word offset into the table buffer (capacity * 8 words)
  int64_t jabi_off;          // word offset of the ABI couplings (3 * JW words)
  int64_t jk_off;            // word offset of the kernel-layout couplings
};

struct WalkerState {         // structure of arrays over all walkers
  int32_t* E;
  int32_t* E_min;
  int32_t* rt_state;
  int32_t* new_min;
  uint64_t* rt_count;
  uint64_t* t_first;
  uint64_t* t_last;
};

struct SweepArgs {
  const RealInfo* reals;
  const int32_t* wave_real;  // per wave of this launch: realization index
  const int32_t* wave_wl;    // per wave: local index of its first walker
  uint32_t* spins;
  const uint32_t* jk;
  const uint32_t* tables;
  WalkerState ws;
  unsigned long long* hist;
  int32_t* trace;             // [trace_nw][trace_cap] int32, walkers trace_w0 .. trace_w0 + trace_nw - 1
  int32_t trace_cap;
  // on-chip histogram window of a realization: levels [max(0, row0 - hist_margin), + hist_n);
  // counts outside it go to HBM directly
  int32_t hist_margin;
  uint64_t trace_t0;         // first traced sweep
  int64_t trace_w0, trace_nw; // traced walkers (global indices)
  uint64_t t0;               // first sweep of this launch
  uint32_t n_sweeps;
  int32_t hist_n;
  uint64_t walker_seed;
  // parallel tempering (unused by the multicanonical kernel)
  const uint32_t* pt_metro;  // per realization kMaxReplicas x 8 Metropolis thresholds, u-order
  const double* pt_q;        // per realization kMaxReplicas: q of the pair (s, s+1), exp(4 dbeta)
  int32_t* pt_slot;          // temperature slot of every walker
  uint64_t* pt_acc;          // accepted exchanges per (set, pair)
  int32_t pt_M, pt_spw;
  uint32_t pt_minv, pt_pad;
};

// Weight-recursion state of one realization (device and host mirror, same layout as nfm_rec_info).
struct RecInfo {
  int32_t k_lo, k_top;       // estimate defined on [k_lo, k_top]; k_top = lowest level with E >= 0
  int32_t profile;           // 0 flat, 1 power law, 2 1/k
  int32_t converged;         // last update: flat to f_tol and no new minimum
  int32_t iterations;        // updates done
  int32_t k_lo_changed;      // last update lowered k_lo
  double pl_dE, pl_alpha;    // power-law parameters of Eq. (5)
  double flatness;           // min/mean of H/P over visited levels, last update
  int32_t k_seed;            // -1, or the lowest level of a seeded prior on the DOS steps
  int32_t pad;
};

// lowest level of the weights and table: a seeded prior extends them below k_lo
__host__ __device__ inline int rec_low(const RecInfo& ri) {
  return (ri.k_seed >= 0 && ri.k_seed < ri.k_lo) ? ri.k_seed : ri.k_lo;
}

// Per-level FP64 arrays of the recursion (indexed by level offset + level).
struct RecArrays {
  double* b;                 // DOS steps S(k+1) - S(k)
  double* p;                 // accumulated weights of the steps
  double* S;                 // ln Omega estimate, S(k_top) = 0
  double* lnP;               // target profile used for the current weights
  double* lnW;               // current log-weights
  unsigned char* visited;    // level ever visited
};

// Wang-Landau state of one realization (device and host mirror, same layout as nfm_wl_info).
struct WlInfo {
  double ln_f;               // current modification factor
  double flatness;           // min/mean of the stage histogram over its visited levels, last update
  int32_t stage;             // halvings of ln f so far
  int32_t done;              // ln f fell below the final value
  int32_t k_top;             // the estimate lives on [0, k_top]; W is constant above
  int32_t updates;           // updates so far
};

// Per-level arrays of the Wang-Landau estimate (indexed by level offset + level).
struct WlArrays {
  double* lng;               // ln g estimate
  unsigned long long* hst;   // histogram of the current stage
  double* lnw;               // log-weights -ln g of the current table
};

}  // namespace nfm
