/*
 * nfm_oracle.h -- plain sequential CPU model of the sampler (TEST INFRASTRUCTURE).
 *
 * This is the checker, not the product. Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg load it. The GPU library never calls
 * it and shares no code with it.
 *
 * Model: 3D bimodal Edwards-Anderson spin glass, Muller/Schnabel/Janke,
 * "Nonflat Histogram Techniques for Spin Glasses", Sec. II, Eq. (1).
 * Sampler: generalized Metropolis with energy weights W(E), Sec. II, Eq. (2).
 *
 * Conventions shared with the GPU library by specification (not by code):
 *   site index   i = x + L*y + L*L*z, periodic boundaries;
 *   couplings    J[d*N + i] in {+1,-1} is the bond between i and i + e_d;
 *   levels       k = (E - e_base)/4, e_base = -3N + 2*(n_minus mod 2);
 *   sweep order  checkerboard: all sites with x+y+z even in ascending i, then
 *                all odd ones; attempt a = 0..N-1 counts position in that order;
 *   random words Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11);
 *                the acceptance word of the attempt at the q-th site of colour c
 *                in plane z (rank among that colour's sites of the plane, ascending
 *                i) in sweep t of walker w of realization r is output[q & 3] of
 *                counter (((c L + z) << 8) | (q >> 2), t, r, (w << 8) | TAG_ACC)
 *                under key = walker seed.
 */
#ifndef NFM_ORACLE_H
#define NFM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_TAG_ACC = 1, ORC_TAG_SPIN = 2, ORC_TAG_J = 3, ORC_TAG_PT = 4, ORC_TAG_SWAP = 5 };
enum { ORC_PROFILE_FLAT = 0, ORC_PROFILE_POWER = 1, ORC_PROFILE_INVK = 2 };

typedef struct {
  int32_t E;         /* current energy */
  int32_t E_min;     /* lowest energy seen so far */
  int32_t rt_state;  /* 0: top not yet reached, 1: top reached, 2: bottom reached after top */
  int32_t new_min;   /* 1 once an energy below e_bot was seen */
  uint64_t rt_count; /* completed round trips top -> bottom -> top */
  uint64_t t_first;  /* attempt stamp of the first arrival at the top */
  uint64_t t_last;   /* attempt stamp at which the last round trip completed */
} orc_walker;

/* Philox4x32-10 block function. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Lattice helpers. */
int32_t orc_n_minus(int32_t L, const int8_t* J);
int32_t orc_e_base(int32_t L, const int8_t* J);
int32_t orc_n_levels(int32_t L, const int8_t* J);
void orc_sweep_order(int32_t L, int32_t* order /* N */);

/* Disorder and initial spins drawn from the Philox stream. */
void orc_gen_couplings(int32_t L, uint64_t disorder_seed, uint32_t real_id, int8_t* J /* 3N */);
void orc_gen_spins(int32_t L, uint64_t walker_seed, uint32_t real_id, uint32_t walker, int8_t* S /* N */);

/* Energy, Eq. (1). */
int32_t orc_energy(int32_t L, const int8_t* J, const int8_t* S);
/* Number of unsatisfied bonds at site i (J S_i S_j = -1). */
int32_t orc_unsatisfied(int32_t L, const int8_t* J, const int8_t* S, int32_t i);

/* Threshold table from log-weights on levels [k_lo, k_top]; rows cover
 * [max(0,k_lo-3), min(K-1,k_top+3)], 8 words per row (u = 0..6, pad). */
int32_t orc_table_rows(int32_t K, int32_t k_lo, int32_t k_top, int32_t* row0);
int32_t orc_build_thresholds(int32_t K, const double* lnw, int32_t k_lo, int32_t k_top,
                             uint32_t* thr, int32_t* row0, int32_t* rows);

/* Metropolis acceptance of an attempt with random word r and stored threshold thr
 * (Eq. (2) with quantised probabilities): thr = 0xFFFFFFFF or r < max(thr, 1). */
int32_t orc_metropolis_accept(uint32_t r, uint32_t thr);

/* Round-trip / minimum bookkeeping after one attempt (stamp tau, energy E). */
void orc_track(orc_walker* w, int32_t E, int32_t e_bot, int32_t e_top, uint64_t tau);

/* Multicanonical sweeps of one walker. Returns 0, or -1 if check_energy is set
 * and the incremental energy ever differs from a recomputation. */
int32_t orc_muca_sweeps(int32_t L, const int8_t* J, int8_t* S, orc_walker* w,
                        const uint32_t* thr, int32_t row0, int32_t rows,
                        int32_t e_bot, int32_t e_top,
                        uint64_t walker_seed, uint32_t real_id, uint32_t walker,
                        uint64_t t0, uint64_t n_sweeps,
                        uint64_t* hist /* K or NULL */, int32_t* trace /* n_sweeps or NULL */,
                        int32_t check_energy);

/* Exact density of states by enumeration of all 2^N states (N <= 32). */
int32_t orc_brute_dos(int32_t L, const int8_t* J, uint64_t* g /* K */);

/* Weight recursion. */
double orc_power_profile(double E, double E_g, double dE, double alpha);
void orc_rec_weights(int32_t K, int32_t e_base, int32_t k_lo, int32_t k_top, int32_t profile,
                     double pl_dE, double pl_alpha, const double* b,
                     double* S, double* lnP, double* lnW);
void orc_rec_update(int32_t K, int32_t k_lo_used, int32_t k_top, int32_t k_min_seen,
                    const double* lnW_used, const double* lnP_used, const uint64_t* H,
                    double* b, double* p, uint8_t* visited, int32_t* k_lo_new,
                    double* flatness);

void orc_rec_weights_ext(int32_t K, int32_t e_base, int32_t k_lo, int32_t k_top, int32_t k_low,
                         int32_t profile, double pl_dE, double pl_alpha, const double* b,
                         double* S, double* lnP, double* lnW);
void orc_rec_update_ext(int32_t K, int32_t k_lo_used, int32_t k_top, int32_t k_low_used, int32_t seeded,
                        int32_t k_min_seen, const double* lnW_used, const double* lnP_used,
                        const uint64_t* H, double* b, double* p, uint8_t* visited, int32_t* k_lo_new,
                        double* flatness);
int32_t orc_seed_from_grid(int32_t N, int32_t e_base, int32_t k_top, const float* y /* 256 */, double* b);

/* Inputs of the weight-seeding model. */
void orc_features(int32_t L, const int8_t* J, double* out /* 16 */);
void orc_hist_bins(int32_t K, int32_t e_base, int32_t N, const uint64_t* H, double* out /* 64 */);

/* Parallel tempering, Sec. II, Eq. (8). Temperatures strictly increasing. */
void orc_pt_metro_table(int32_t M, const double* T, uint32_t* thr /* M x 8 */);
int32_t orc_pt_swap_table(int32_t M, const double* T, int32_t d_cap, uint32_t* thr /* (M-1) x D or NULL */);
/* q^d by binary powering (lowest bit first); q of the pair (T_lo, T_hi) = exp(4 (1/T_hi - 1/T_lo)). */
double orc_pow_bin(double q, int32_t d);
double orc_pt_swap_q(double T_lo, double T_hi);
int32_t orc_pt_sweeps(int32_t L, const int8_t* J, int32_t M, int8_t* S /* M x N */, orc_walker* w /* M */,
                      int32_t* slot /* M */, const uint32_t* metro, const uint32_t* swap, int32_t D,
                      int32_t e_bot, int32_t e_top, uint64_t walker_seed, uint32_t real_id, uint32_t set,
                      uint32_t walker0 /* walker index of configuration 0 */,
                      uint64_t t0, uint64_t n_sweeps, uint64_t* swap_acc /* M-1 or NULL */,
                      int32_t* trace /* M x n_sweeps or NULL */, int32_t check_energy);

#ifdef __cplusplus
}
#endif
#endif
